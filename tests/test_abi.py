"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and the planner (host only, no GPU calls) validates input
and produces the constants the paper fixes."""
import ctypes as C
import os
import re
from fractions import Fraction

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2001_06113_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2001_06113_amd import build

        build.build()
    return _lib.load()


def _header_functions():
    text = open(os.path.join(ROOT, "include", "tdse.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(tdse_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol(lib):
    names = _header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def _problem(dim=2, M=(32, 64), T=1.0, nsteps=100, order=8, A=None, nV=1, f=None, domain=0, precision=0):
    from paper_2001_06113_amd import _lib

    p = _lib.Problem()
    p.dim = dim
    p.domain = domain
    p.M[0], p.M[1] = M[0], (M[1] if len(M) > 1 else 0)
    p.T = T
    p.nsteps = nsteps
    p.order = order
    p.n_start = -1
    p.precision = precision
    p.nV = nV
    size = int(np.prod(M[:dim]))
    V = np.zeros(nV * size)
    p._keep = [V]
    p.V_fields = V.ctypes.data_as(C.POINTER(C.c_double))
    if f is not None:
        fp = np.asarray(f, dtype=np.float64)
        p._keep.append(fp)
        p.f_kind = 1
        p.f_params = fp.ctypes.data_as(C.POINTER(C.c_double))
    if A is not None:
        ap = np.asarray(A, dtype=np.float64)
        p._keep.append(ap)
        p.A_kind = 1
        p.A_params = ap.ctypes.data_as(C.POINTER(C.c_double))
    return p


def _plan(lib, p):
    h = C.c_void_p()
    st = lib.tdse_plan(C.byref(p), C.byref(h))
    return st, h


@pytest.mark.parametrize("kw,status", [
    (dict(dim=3), -2),
    (dict(dim=0), -1),
    (dict(M=(30, 64)), -1),          # not 2^a 3^b
    (dict(M=(6, 64)), -1),           # too small
    (dict(M=(32, 63)), -1),          # odd
    (dict(order=7), -1),
    (dict(order=10), -1),
    (dict(T=0.0), -1),
    (dict(nsteps=0), -1),
    (dict(nV=0), -1),
    (dict(domain=1), -2),
    (dict(precision=7), -1),
])
def test_plan_rejects(lib, kw, status):
    st, h = _plan(lib, _problem(**kw))
    assert st == status, lib.tdse_last_error()
    assert lib.tdse_last_error().decode()


def test_calls_out_of_order(lib):
    st, h = _plan(lib, _problem())
    assert st == 0
    # no workspace bound yet: stepping or reading the state is a state error
    assert lib.tdse_step(h, 1) == -6
    buf = np.zeros(2 * 32 * 64)
    assert lib.tdse_get_state(h, buf.ctypes.data_as(C.c_void_p), 0) == -6
    assert lib.tdse_set_state(h, buf.ctypes.data_as(C.c_void_p), 0) == -6
    sz = C.c_size_t()
    assert lib.tdse_workspace_size(h, C.byref(sz)) == 0
    assert sz.value >= (1 + 7 + 1 + 2) * 32 * 64 * 16
    # a workspace that is too small is refused before any device call
    assert lib.tdse_bind(h, C.c_void_p(256), 16, None) == -3
    lib.tdse_destroy(h)


def test_planner_constants_match_paper(lib):
    from oracle.adams import adams_coefficients

    for order in (2, 4, 6, 8):
        st, h = _plan(lib, _problem(order=order))
        assert st == 0
        v = C.c_double()
        for j, mu in enumerate(adams_coefficients(order)):
            assert lib.tdse_query(h, 16 + j, C.byref(v)) == 0
            assert v.value == float(mu)
        lib.tdse_destroy(h)
    # folded Richardson weights reproduce the tableau of Section 2.2
    st, h = _plan(lib, _problem(order=8))
    w = []
    for l in range(4):
        assert lib.tdse_query(h, 32 + l, C.byref(v)) == 0
        w.append(v.value)
    exact = [Fraction(-1, 2835), Fraction(4, 135), Fraction(-64, 135), Fraction(4096, 2835)]
    assert np.allclose(w, [float(x) for x in exact], rtol=0, atol=1e-16)
    lib.tdse_destroy(h)


def test_planner_phi_closed_form(lib):
    # phi(T) of the sin^2 pulse vs an independent 2000-panel Gauss-Legendre sum
    E0, om, Tp = 1.3, 9.7, 2.0
    st, h = _plan(lib, _problem(A=[E0, om, Tp, 1.0, 0.0], T=Tp))
    assert st == 0
    v = C.c_double()
    gx, gw = np.polynomial.legendre.leggauss(20)
    edges = np.linspace(0, Tp, 2001)
    tot = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        s = 0.5 * (a + b) + 0.5 * (b - a) * gx
        tot += 0.5 * (b - a) * np.sum(gw * E0 * np.sin(np.pi * s / Tp) ** 2 * np.sin(om * s))
    assert lib.tdse_query(h, 64, C.byref(v)) == 0
    assert abs(v.value - tot) < 1e-13
    assert lib.tdse_query(h, 65, C.byref(v)) == 0 and v.value == 0.0
    lib.tdse_destroy(h)


def test_status_strings(lib):
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert lib.tdse_status_string(s).decode().startswith("TDSE_")
