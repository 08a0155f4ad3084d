"""Pins of the oracle's moving periodic Gaussian well (Example 1 of Section 6).

* At c = 0 the well is a static potential: the run equals the stored-field
  path with the same Gaussian built by the input generator.
* Galilean covariance (A = 0): if w solves the static-well problem from
  w0 = exp(-i c.x/2) u0, then u(x, t) = exp(i(c.x/2 - |c|^2 t/4)) w(x - c t, t)
  solves the moving-well problem from u0.  With c/2 integral the phase is
  2 pi periodic, and with c T a multiple of 2 pi the shift vanishes on the
  grid at t = T, so the two discrete runs must agree to the scheme's
  accuracy (their time-discretization errors differ at O(dt^8)).
* The ground state of the well at rest (the paper's u0) has the eigenvalue
  the example prints (about -243); boosted by e^{i c x/2}, it rides the
  moving well as an exact solution, which the oracle reaches at eighth order.
"""
import os

import numpy as np
import pytest

from oracle.periodic import PeriodicOracle
from workloads import Problem, moving_well_problem, periodic_grid
from workloads.synth import _periodized_gauss


def _static_twin(p, u0):
    V0, beta = p.V_well[0], p.V_well[1]
    X = [periodic_grid(m) for m in p.M]
    X = list(np.meshgrid(*X, indexing="ij")) if p.dim == 2 else X
    field = -V0 * _periodized_gauss(X, [0.0] * p.dim, np.sqrt(2.0) * beta, images=3)
    return Problem(name="static-well", dim=p.dim, domain="periodic", M=p.M, T=p.T, nsteps=p.nsteps,
                   order=p.order, u0=u0, V_fields=[field], f_kind=["const"], f_params=[(0.0, 0.0)])


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("M", [(256,), (48, 64)])
def test_standing_well_equals_stored_field(M):
    p = moving_well_problem(c=(0.0,) * len(M), M=M, nsteps=60)
    u, _ = PeriodicOracle(p).run()
    w, _ = PeriodicOracle(_static_twin(p, p.u0)).run()
    assert _rel(u, w) < 1e-12


# the boost shifts the spectrum by c/2 = 15 modes: the moving axis needs
# 256 points for the shifted spectrum to stay inside the band
@pytest.mark.parametrize("M,c", [((256,), (30.0,)), ((256,), (-30.0,)), ((256, 128), (30.0, 0.0)),
                                 ((128, 256), (0.0, -30.0))])
def test_galilean_covariance(M, c):
    T = 2.0 * np.pi / 15.0          # c T = 4 pi along every axis
    p = moving_well_problem(c=c, M=M, T=T, nsteps=400)
    u, _ = PeriodicOracle(p).run()
    X = [periodic_grid(m) for m in M]
    X = list(np.meshgrid(*X, indexing="ij")) if len(M) == 2 else X
    cx = sum(ca * xa for ca, xa in zip(c, X)) / 2.0
    c2 = sum(ca * ca for ca in c) / 4.0
    w, _ = PeriodicOracle(_static_twin(p, np.exp(-1j * cx) * p.u0)).run()
    pred = np.exp(1j * cx) * np.exp(-1j * c2 * T) * w
    assert _rel(u, pred) < 1e-11


def test_covariance_fails_for_the_wrong_velocity():
    # the same comparison with the boost of the opposite velocity is far off
    T = 2.0 * np.pi / 15.0
    p = moving_well_problem(c=(30.0,), M=(256,), T=T, nsteps=200)
    u, _ = PeriodicOracle(p).run()
    x = periodic_grid(256)
    w, _ = PeriodicOracle(_static_twin(p, np.exp(15j * x) * p.u0)).run()
    pred = np.exp(-15j * x) * np.exp(-225j * T) * w
    assert _rel(u, pred) > 1e-2


# --- Example 1 with the well's ground state ---------------------------------

def _golden_example1():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "example1_moving_well.txt")
    vals = {}
    for line in open(path):
        if not line.startswith("#") and line.strip():
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_periodic_well_ground_state_matches_the_printed_eigenvalue():
    from workloads import periodic_well_ground_state

    g = _golden_example1()
    E, u = periodic_well_ground_state(g["V0"], g["beta"], 256)
    assert abs(E - g["ground_eigenvalue"]) < 0.5              # -243.48
    E2, _ = periodic_well_ground_state(g["V0"], g["beta"], 512)
    assert abs(E - E2) < 1e-9
    assert abs(np.sum(np.abs(u) ** 2) * 2 * np.pi / 256 - 1.0) < 1e-12


def _shifted(g, s):
    # g(x - s) on the periodic grid by trigonometric interpolation
    k = np.fft.fftfreq(g.size, d=2 * np.pi / g.size) * 2 * np.pi
    return np.real(np.fft.ifft(np.fft.fft(g) * np.exp(-1j * k * s)))


@pytest.mark.parametrize("c", [0.0, 30.0])
def test_boosted_ground_state_rides_the_moving_well_exactly(c):
    # u0 = e^{i c x/2} psi_0 makes u = e^{i(c x/2 - c^2 t/4)} e^{-i E t} psi_0(x - c t)
    # an exact solution with the well moving at c (c/2 integral keeps the
    # boost periodic); the oracle converges to it at eighth order in dt
    from workloads import periodic_well_ground_state

    M, T = 256, 2 * np.pi / 15
    E, g = periodic_well_ground_state(300.0, 0.2, M)
    x = periodic_grid(M)
    ex = np.exp(1j * (c * x / 2 - c * c * T / 4)) * np.exp(-1j * E * T) * _shifted(g, c * T)
    errs = []
    for N in (800, 1600):
        prob = moving_well_problem(c=(c,), M=(M,), nsteps=N)
        prob.u0 = (np.exp(1j * c * x / 2) * g).astype(np.complex128)
        u, _ = PeriodicOracle(prob).run()
        errs.append(np.linalg.norm(u - ex) / np.linalg.norm(ex))
    assert errs[1] < 1e-8, errs                    # 5.1e-9 measured
    assert errs[0] / errs[1] > 150, errs           # 2^8 = 256 asymptotically
