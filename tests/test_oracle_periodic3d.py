"""Pins of the periodic oracle in three dimensions (Sections 2.1-2.2 with
d = 3: the modes k in Z^3, |k|^2 and k . phi over three axes, the transforms
over three axes).  The oracle itself is dimension-generic; these tests pin
what only a 3D run exercises against results fixed by the mathematics."""
import numpy as np
import pytest

from oracle.periodic import PeriodicOracle
from workloads import Problem, periodic_grid, periodic_problem_from_seed


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _stepwise(nsteps, dim, seed):
    # a piecewise-constant vector potential with a component on every axis
    rng = np.random.default_rng(seed)
    base = rng.uniform(-3.0, 3.0, size=dim)
    t = (np.arange(nsteps) + 0.5) / nsteps
    return base[None, :] * np.sin(2 * np.pi * t)[:, None] + rng.uniform(-0.5, 0.5, size=(nsteps, dim))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_plane_waves_reduce_3d_to_1d(axis):
    # V = V(x_axis) and u0 = g(x_axis) exp(i(k_b x_b + k_c x_c)): every mode
    # of the 3D run has fixed k_b, k_c, so |k|^2 = k_a^2 + k_b^2 + k_c^2 and
    # k . dphi split off a factor exp(-i(k_b^2 + k_c^2) t + i(k_b phi_b + k_c phi_c))
    # common to every term of the recurrence, the solve and the extrapolation:
    # u_3D(T) = that factor at T times the plane waves times the 1D run of the
    # scheme on the axis (exactly, up to rounding)
    M = (16, 12, 24)
    N, T = 14, 0.07
    Ma = M[axis]
    xa = periodic_grid(Ma)
    Va = -4.0 * np.exp(-(xa - 0.4) ** 2 / 0.5) + 1.5 * np.cos(2 * xa)
    g = np.exp(-(xa + 0.3) ** 2 / 0.6) * (1 + 0.3j * np.sin(xa))
    others = [b for b in range(3) if b != axis]
    kk = {others[0]: 2, others[1]: -3}
    A3 = _stepwise(N, 3, 5 + axis)
    prob1 = Problem(name="1d", dim=1, domain="periodic", M=(Ma,), T=T, nsteps=N, order=8, u0=g.astype(complex),
                    V_fields=[Va], f_kind=["sin"], f_params=[(0.3, 9.0)], A_kind="stepwise",
                    A_steps=A3[:, [axis]].copy())
    u1, _ = PeriodicOracle(prob1).run()
    X = np.meshgrid(*[periodic_grid(m) for m in M], indexing="ij")
    shape = [1, 1, 1]
    shape[axis] = Ma
    V3 = np.broadcast_to(Va.reshape(shape), M).copy()
    wave = np.exp(1j * sum(kk[b] * X[b] for b in others))
    u0 = g.reshape(shape) * wave
    prob3 = Problem(name="3d", dim=3, domain="periodic", M=M, T=T, nsteps=N, order=8, u0=u0,
                    V_fields=[V3], f_kind=["sin"], f_params=[(0.3, 9.0)], A_kind="stepwise", A_steps=A3)
    orc = PeriodicOracle(prob3)
    u3, _ = orc.run()
    ph = orc.phi(T)
    fac = np.exp(-1j * sum(kk[b] ** 2 for b in others) * T + 1j * sum(kk[b] * ph[b] for b in others))
    ex = fac * u1.reshape(shape) * wave
    assert _rel(u3, ex) < 1e-12
    # a different axis assignment is off (negative control)
    bad = fac * u1.reshape(shape) * np.exp(1j * (kk[others[0]] * X[others[1]] + kk[others[1]] * X[others[0]]))
    assert _rel(u3, bad) > 1e-2


def test_free_plane_waves_exact_3d():
    # V = 0: a sum of plane waves e^{i k.x} evolves to e^{-i|k|^2 T + i k.phi(T)} e^{i k.x}
    M = (8, 16, 12)
    N, T = 10, 0.3
    X = np.meshgrid(*[periodic_grid(m) for m in M], indexing="ij")
    ks = [(1, -2, 3), (-3, 0, 2), (2, 5, -4)]
    amps = [1.0, 0.5 - 0.2j, 0.3j]
    u0 = sum(a * np.exp(1j * (k[0] * X[0] + k[1] * X[1] + k[2] * X[2])) for a, k in zip(amps, ks))
    A3 = _stepwise(N, 3, 11)
    prob = Problem(name="free3d", dim=3, domain="periodic", M=M, T=T, nsteps=N, order=8, u0=u0,
                   V_fields=[np.zeros(M)], f_kind=["const"], f_params=[(0.0, 0.0)], A_kind="stepwise", A_steps=A3)
    orc = PeriodicOracle(prob)
    u, _ = orc.run()
    ph = orc.phi(T)
    ex = sum(a * np.exp(-1j * (k[0] ** 2 + k[1] ** 2 + k[2] ** 2) * T + 1j * (k[0] * ph[0] + k[1] * ph[1] + k[2] * ph[2]))
             * np.exp(1j * (k[0] * X[0] + k[1] * X[1] + k[2] * X[2])) for a, k in zip(amps, ks))
    assert np.max(np.abs(u - ex)) < 1e-12


def test_eighth_order_in_time_3d():
    # self-convergence of the order-8 scheme on the 3D recipe: the error
    # falls by about 2^8 per halving of dt until rounding
    sols = {}
    for N in (24, 48, 96, 384):
        prob = periodic_problem_from_seed(21, 3, (12, 16, 12), 0.2, N)
        sols[N], _ = PeriodicOracle(prob).run()
    ref = sols[384]
    e1, e2 = (np.linalg.norm(sols[N] - ref) for N in (24, 48))
    assert e1 / e2 > 150, (e1, e2)
    assert np.linalg.norm(sols[96] - ref) < e2 / 100
