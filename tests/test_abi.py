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


def _problem(dim=2, M=(32, 64), T=1.0, nsteps=100, order=8, A=None, nV=1, f=None, domain=0, precision=0,
             nu=(256, 256), fs_p=8, q=10, panels=1, eps=1e-10, H=0.0, cheb=0):
    from paper_2001_06113_amd import _lib

    p = _lib.Problem()
    p.dim = dim
    p.domain = domain
    for a, n in enumerate(nu):
        p.nu[a] = n
    p.p, p.q, p.panels, p.eps, p.H = fs_p, q, panels, eps, H
    p.cheb = cheb
    p.M[0], p.M[1] = M[0], (M[1] if len(M) > 1 else 0)
    p.M[2] = M[2] if len(M) > 2 else 0
    p.T = T
    p.nsteps = nsteps
    p.order = order
    p.n_start = -1
    p.precision = precision
    p.nV = nV
    size = int(np.prod(M[:dim]))
    V = np.zeros(nV * size if size <= (1 << 24) else 1)   # oversized grids are refused before V is read
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
    (dict(dim=4), -1),
    (dict(dim=3), -1),                               # third axis of size 0
    (dict(dim=3, M=(32, 64, 16), domain=1), -1),     # 3D free space: no FFT size for the third axis
    (dict(dim=3, M=(32, 64, 16), domain=1, nu=(256, 256, 256), precision=1), -2),   # free space: FP64 only
    (dict(dim=3, M=(32, 64, 30)), -1),
    (dict(dim=3, M=(1024, 1024, 512)), -1),          # more than 2^28 points
    (dict(dim=0), -1),
    (dict(M=(30, 64)), -1),          # not 2^a 3^b
    (dict(M=(6, 64)), -1),           # too small
    (dict(M=(32, 63)), -1),          # odd
    (dict(order=7), -1),
    (dict(order=10), -1),
    (dict(T=0.0), -1),
    (dict(nsteps=0), -1),
    (dict(nV=0), -1),
    (dict(domain=2), -1),
    (dict(precision=7), -1),
    # free space
    (dict(domain=1, precision=1), -2),          # FP64 only
    (dict(domain=1, fs_p=6), -2),               # order-16 Alpert rule only
    (dict(domain=1, nu=(300, 256)), -1),        # FFT size not built
    (dict(domain=1, M=(32, 300)), -1),          # M > nu
    (dict(domain=1, M=(32, 63)), -1),           # odd M
    (dict(domain=1, nu=(64, 256)), -1),         # N_E <= M/2
    (dict(domain=1, eps=0.0), -1),              # no tolerance and no H
    (dict(domain=1, q=1), -1),
    (dict(domain=1, panels=0), -1),
    (dict(domain=1, q=32, panels=8, nu=(256, 256), cheb=-1), -1),   # more direct-sum rows than nu/2
    (dict(domain=1, cheb=1), -1),
    (dict(domain=1, cheb=65), -1),
    (dict(domain=1, cheb=-2), -1),
])
def test_plan_rejects(lib, kw, status):
    st, h = _plan(lib, _problem(**kw))
    assert st == status, lib.tdse_last_error()
    assert lib.tdse_last_error().decode()


@pytest.mark.parametrize("V_kind,params,domain,status", [
    (2, (300.0, 0.2, 15.0, 0.0), 0, -1),        # unknown potential kind
    (1, (300.0, 0.2, 15.0, 0.0), 1, -2),        # the moving well is periodic only
    (1, (300.0, 1.5, 15.0, 0.0), 0, -1),        # beta > 1
    (1, (300.0, 0.0, 15.0, 0.0), 0, -1),
    (1, (300.0, 0.2, float("nan"), 0.0), 0, -1),
    (1, (300.0, 0.2, 15.0, 0.0), 0, 0),         # valid, with no fields
])
def test_moving_well_planning(lib, V_kind, params, domain, status):
    p = _problem(dim=1, M=(64,), domain=domain, nV=0)
    p.V_kind = V_kind
    for k, v in enumerate(params):
        p.V_params[k] = v
    p.V_fields = C.POINTER(C.c_double)()
    st, h = _plan(lib, p)
    assert st == status, lib.tdse_last_error()
    if st == 0:
        lib.tdse_destroy(h)


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


@pytest.mark.parametrize("om", [9.7, np.pi])   # the second has omega - 2 pi/Tp = 0
def test_planner_phi_closed_form_cosine_pulse(lib, om):
    # eq. (apulse), A = E0 sin^2(pi t/Tp) cos(w t): phi at T = 0.7 Tp vs the
    # same independent Gauss-Legendre sum
    E0, Tp = 1.3, 2.0
    T = 0.7 * Tp
    p = _problem(A=[E0, om, Tp, 0.0, 1.0], T=T)
    p.A_kind = 4
    st, h = _plan(lib, p)
    assert st == 0, lib.tdse_last_error()
    v = C.c_double()
    gx, gw = np.polynomial.legendre.leggauss(20)
    edges = np.linspace(0, T, 2001)
    tot = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        s = 0.5 * (a + b) + 0.5 * (b - a) * gx
        tot += 0.5 * (b - a) * np.sum(gw * E0 * np.sin(np.pi * s / Tp) ** 2 * np.cos(om * s))
    assert lib.tdse_query(h, 65, C.byref(v)) == 0
    assert abs(v.value - tot) < 1e-13
    assert lib.tdse_query(h, 64, C.byref(v)) == 0 and v.value == 0.0
    lib.tdse_destroy(h)
    p.A_kind = 5
    st, h = _plan(lib, p)
    assert st == -1


def test_free_space_planner_alpert_rule_matches_oracle(lib):
    # the planner's long-double modified-Chebyshev/Golub-Welsch construction
    # against the oracle's exact Hankel solve and mpmath roots
    from oracle.quadrature import alpert_float

    st, h = _plan(lib, _problem(domain=1))
    assert st == 0, lib.tdse_last_error()
    x, w = alpert_float(8, 7)
    v = C.c_double()
    for k in range(8):
        assert lib.tdse_query(h, 96 + k, C.byref(v)) == 0
        assert abs(v.value - x[k]) < 2e-14
        assert lib.tdse_query(h, 112 + k, C.byref(v)) == 0
        assert abs(v.value - w[k]) < 2e-14
    assert lib.tdse_query(h, 96 + 8, C.byref(v)) == -1
    lib.tdse_destroy(h)


def _fs_key(field, axis):
    # per-axis contour keys: axes 0 and 1 in their own blocks, axis 2 in TDSE_Q_FS_AXIS2
    if axis == 2:
        return 136 + field
    return {0: 81, 1: 83, 2: 86}[field] + axis


@pytest.mark.parametrize("dim,M,nu", [(1, (64,), (512,)), (2, (48, 32), (256, 512)), (3, (16, 24, 32), (256, 256, 256))])
def test_free_space_planner_contour_matches_oracle(lib, dim, M, nu):
    # H from the rule of Section 3.2 with ||V|| and phi over the step times,
    # mode counts N = 2 N_E + 2p + N_C of Section 3.4
    from oracle.freespace import FreeSpaceOracle
    from paper_2001_06113_amd import _lib
    from workloads import free_problem_from_seed

    prob = free_problem_from_seed(11, dim, M, 0.2, 40, nu=nu, eps=1e-11, q=7, panels=2)
    orc = FreeSpaceOracle(prob)
    p = _lib.Problem()
    p.dim, p.domain, p.T, p.nsteps, p.order, p.n_start = dim, 1, prob.T, prob.nsteps, 8, -1
    for a in range(dim):
        p.M[a], p.nu[a] = M[a], nu[a]
    p.eps, p.p, p.q, p.panels = prob.eps, 8, 7, 2
    V = np.ascontiguousarray(prob.V_fields[0].ravel())
    fp = np.asarray(prob.f_params[0], dtype=np.float64)
    ap = np.asarray(prob.A_params, dtype=np.float64)
    p._keep = [V, fp, ap]
    p.nV = 1
    p.V_fields = V.ctypes.data_as(C.POINTER(C.c_double))
    p.f_kind, p.f_params = 1, fp.ctypes.data_as(C.POINTER(C.c_double))
    p.A_kind, p.A_params = 1, ap.ctypes.data_as(C.POINTER(C.c_double))
    st, h = _plan(lib, p)
    assert st == 0, lib.tdse_last_error()
    v = C.c_double()
    assert lib.tdse_query(h, 80, C.byref(v)) == 0
    assert abs(v.value - orc.H) < 1e-12 * orc.H
    for a in range(dim):
        # per-axis H: the field lies along axis 0, so a field-free axis gets
        # the rule's value at phi_max = 0, larger than axis 0's
        assert lib.tdse_query(h, _fs_key(2, a), C.byref(v)) == 0
        assert abs(v.value - orc.Hs[a]) < 1e-12 * orc.Hs[a]
    if dim >= 2:
        assert orc.Hs[1] > orc.Hs[0]
    if dim < 3:
        assert lib.tdse_query(h, 86 + dim, C.byref(v)) == -1
    for a in range(dim):
        assert lib.tdse_query(h, _fs_key(0, a), C.byref(v)) == 0
        assert v.value == orc.nodes[a][2]["N"]
        assert lib.tdse_query(h, _fs_key(1, a), C.byref(v)) == 0
        assert v.value == orc.nodes[a][2]["NE"]
    if dim == 1:
        assert lib.tdse_query(h, 82, C.byref(v)) == -1   # no second axis
    if dim < 3:
        assert lib.tdse_query(h, 136, C.byref(v)) == -1   # no third axis
    lib.tdse_destroy(h)


@pytest.mark.parametrize("H", [0.3, 0.95, 1.7, 2.4, 3.0, 4.5, 7.0])
def test_free_space_planner_chebyshev_terms_match_oracle(lib, H):
    # NT of the C-type interpolant (Section 4.1): the planner's Bessel-series
    # rule gives the oracle's count; the automatic choice takes the
    # interpolant only when NT < N_C; -1 and a forced count are honoured
    from oracle.chebyshev import choose_NT

    nt = choose_NT(H)
    v = C.c_double()
    for q, panels, cheb, want in [(16, 4, 0, nt if 0 < nt < 128 else 0), (8, 1, 0, nt if 0 < nt < 16 else 0),
                                  (16, 4, -1, 0), (16, 4, 20, 20)]:
        st, h = _plan(lib, _problem(domain=1, dim=1, M=(64,), nu=(512, 0), q=q, panels=panels, H=H, cheb=cheb))
        assert st == 0, lib.tdse_last_error()
        assert lib.tdse_query(h, 134, C.byref(v)) == 0
        assert v.value == want, (H, q, panels, cheb, v.value, want)
        assert lib.tdse_query(h, 135, C.byref(v)) == -1   # no second axis
        lib.tdse_destroy(h)


def test_sampled_potential_planning(lib):
    # TDSE_V_SAMPLED: nsteps + 1 samples in V_fields, nV ignored; no batch
    p = _problem(nsteps=10, nV=11)
    p.V_kind = 2
    p.nV = 0
    st, h = _plan(lib, p)
    assert st == 0, lib.tdse_last_error()
    lib.tdse_destroy(h)
    p.V_fields = None
    st, h = _plan(lib, p)
    assert st == -1
    q = _problem(nsteps=10, nV=11)
    q.V_kind = 2
    arr = (type(q) * 1)(q)
    h = C.c_void_p()
    assert lib.tdse_plan_batch(arr, 1, C.byref(h)) == -2


def test_periodic_plan_has_no_contour(lib):
    st, h = _plan(lib, _problem())
    v = C.c_double()
    assert lib.tdse_query(h, 80, C.byref(v)) == -1
    lib.tdse_destroy(h)


def test_status_strings(lib):
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert lib.tdse_status_string(s).decode().startswith("TDSE_")


def test_field_update_and_adjoint_sizing(lib):
    # tdse_set_field needs a stepwise-field plan; the adjoint's workspace grows
    # with the checkpoint count; calls before bind are state errors
    st, h = _plan(lib, _problem(A=[1.0, 5.0, 1.0, 1.0, 0.0]))
    assert st == 0
    A = np.zeros(2 * 100)
    assert lib.tdse_set_field(h, A.ctypes.data_as(C.POINTER(C.c_double))) == -1
    lib.tdse_destroy(h)
    p = _problem(nsteps=40)
    steps = np.linspace(0.0, 1.0, 40 * 2)
    p._keep.append(steps)
    p.A_kind = 3
    p.A_steps = steps.ctypes.data_as(C.POINTER(C.c_double))
    st, h = _plan(lib, p)
    assert st == 0, lib.tdse_last_error()
    assert lib.tdse_set_field(h, A.ctypes.data_as(C.POINTER(C.c_double))) == 0
    sizes = []
    for K in (1, 5, 0):
        sz = C.c_size_t()
        assert lib.tdse_adjoint_workspace_size(h, K, C.byref(sz)) == 0
        sizes.append(sz.value)
    assert sizes[0] > sizes[1] > 0 and sizes[2] > 0
    buf = np.zeros(2 * 32 * 64)
    g = np.zeros(80)
    assert lib.tdse_adjoint(h, C.c_void_p(256), sizes[2], 0, buf.ctypes.data_as(C.c_void_p),
                            buf.ctypes.data_as(C.c_void_p), 0, g.ctypes.data_as(C.POINTER(C.c_double)), None) == -6
    lib.tdse_destroy(h)


def test_batch_planner_rejects(lib):
    from paper_2001_06113_amd import _lib

    arr = (_lib.Problem * 2)(_problem(M=(64, 128)), _problem(M=(64, 128), nsteps=50))
    h = C.c_void_p()
    assert lib.tdse_plan_batch(arr, 0, C.byref(h)) == -1
    assert lib.tdse_plan_batch(arr, 2, C.byref(h)) == -1          # different step counts
    assert "share" in lib.tdse_last_error().decode()
    one = (_lib.Problem * 1)(_problem(M=(32, 64)))
    assert lib.tdse_plan_batch(one, 1, C.byref(h)) == -2           # 32-point lines are not batched
    ok = (_lib.Problem * 2)(_problem(M=(64, 128)), _problem(M=(192, 64)))
    assert lib.tdse_plan_batch(ok, 2, C.byref(h)) == 0
    v = C.c_double()
    assert lib.tdse_query(h, 4, C.byref(v)) == 0 and v.value == 2
    assert lib.tdse_query(h, 4096 + 1, C.byref(v)) == 0 and v.value == 64 * 128
    assert lib.tdse_autotune(h, 3) == -6                            # not bound
    lib.tdse_destroy(h)


def test_far_evaluation_sizing_and_checks(lib):
    # workspace of tdse_far_eval: uhat (N1 N2 modes), E2 (N2 ny), and in 2D
    # E1 (N1 nx) and S (N1 ny), each 256-byte aligned; free-space plans only
    al = lambda b: (b + 255) // 256 * 256
    st, h = _plan(lib, _problem(domain=1, M=(32, 64), nu=(256, 512), q=10, panels=1))
    assert st == 0, lib.tdse_last_error()
    v = C.c_double()
    N = []
    for a in range(2):
        assert lib.tdse_query(h, 81 + a, C.byref(v)) == 0
        N.append(int(v.value))
    for nx, ny in ((1, 1), (37, 130), (512, 512)):
        sz = C.c_size_t()
        assert lib.tdse_far_workspace_size(h, nx, ny, C.byref(sz)) == 0
        want = al(16 * N[0] * N[1]) + al(16 * N[1] * ny) + al(16 * N[0] * nx) + al(16 * N[0] * ny)
        assert sz.value == want, (nx, ny)
    sz = C.c_size_t()
    assert lib.tdse_far_workspace_size(h, 0, 5, C.byref(sz)) == -1
    # launches that would not fit a one-dimensional grid are refused up front
    assert lib.tdse_far_workspace_size(h, 1 << 24, 1 << 24, C.byref(sz)) == -1
    ys = np.zeros(4)
    # before bind and set_state: a state error, no device call
    assert lib.tdse_far_eval(h, ys.ctypes.data_as(C.c_void_p), 1, ys.ctypes.data_as(C.c_void_p), 4,
                             ys.ctypes.data_as(C.c_void_p), C.c_void_p(256), 1 << 20) == -6
    lib.tdse_destroy(h)
    st, h = _plan(lib, _problem(dim=1, M=(64,), domain=1, nu=(512, 0), q=10, panels=1))
    assert st == 0, lib.tdse_last_error()
    assert lib.tdse_far_workspace_size(h, 1, 9, C.byref(sz)) == 0
    assert lib.tdse_far_workspace_size(h, 2, 9, C.byref(sz)) == -1
    lib.tdse_destroy(h)
    st, h = _plan(lib, _problem())
    assert st == 0
    assert lib.tdse_far_workspace_size(h, 4, 4, C.byref(sz)) == -2
    lib.tdse_destroy(h)
    # a 3D free-space plan: evaluation at arbitrary points is not offered
    st, h = _plan(lib, _problem(dim=3, M=(8, 8, 8), domain=1, nu=(256, 256, 256), q=4, panels=1))
    assert st == 0, lib.tdse_last_error()
    assert lib.tdse_far_workspace_size(h, 4, 4, C.byref(sz)) == -2
    lib.tdse_destroy(h)
