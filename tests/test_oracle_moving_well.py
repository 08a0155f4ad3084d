"""Pins of the oracle's moving periodic Gaussian well (Example 1 of Section 6).

* At c = 0 the well is a static potential: the run equals the stored-field
  path with the same Gaussian built by the input generator.
* Galilean covariance (A = 0): if w solves the static-well problem from
  w0 = exp(-i c.x/2) u0, then u(x, t) = exp(i(c.x/2 - |c|^2 t/4)) w(x - c t, t)
  solves the moving-well problem from u0.  With c/2 integral the phase is
  2 pi periodic, and with c T a multiple of 2 pi the shift vanishes on the
  grid at t = T, so the two discrete runs must agree to the scheme's
  accuracy (their time-discretization errors differ at O(dt^8)).
"""
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
