"""Pins of the free-space oracle and its Gamma quadrature (Sections 3.2-3.4).

Each check uses something independent of the oracle's own formulas: a
closed-form integral, the Fourier transform of a Gaussian, the exact Gaussian
wave packet of eq. (wavepacket), or a convergence rate the paper reports."""
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

from oracle.freespace import FreeSpaceOracle
from oracle.quadrature import alpert_endpoint_rule, alpert_moments, choose_H, gamma_rule
from workloads import Problem, free_grid, free_problem_from_seed


def test_alpert_rule_nodes_and_weights_are_a_positive_rule_in_range():
    x, w = alpert_endpoint_rule(8, 7)
    assert len(x) == 8
    assert all(0 < float(v) < 7 for v in x)
    assert all(float(v) > 0 for v in w)
    # the Bernoulli-polynomial moments reproduce sum_{k<kappa} k^m + B_{m+1}/(m+1),
    # i.e. the omitted trapezoid nodes 0..kappa-1 plus the endpoint correction
    c = alpert_moments(8, 7)
    assert c[0] == Fraction(13, 2)          # 7 nodes minus half the endpoint node
    assert c[1] == Fraction(21 + 1, 1) - Fraction(11, 12)   # 0+1+..+6 = 21, B_2/2 = 1/12


def test_alpert_rule_sixteenth_order():
    # int_0^inf e^{-t} cos t dt = 1/2; error ratio -> 2^16 or more per halving
    # of h (Section 6, Example 2 reports about 16th order for p = 8)
    mp.mp.dps = 50
    x, w = alpert_endpoint_rule(8, 7)
    f = lambda t: mp.exp(-t) * mp.cos(t)
    errs = []
    for h in (mp.mpf("0.4"), mp.mpf("0.2"), mp.mpf("0.1")):
        s = sum(wk * f(xk * h) for xk, wk in zip(x, w)) + mp.nsum(lambda j: f(j * h), [7, mp.inf])
        errs.append(abs(h * s - mp.mpf(1) / 2))
    assert errs[-1] < 1e-24
    assert errs[1] / errs[2] > 2 ** 15


@pytest.mark.parametrize("M,nu", [(64, 512), (128, 1024)])
def test_gamma_quadrature_inverts_gaussian_transform(M, nu):
    # (1/2pi) sum_k w_k e^{i zeta_k x} ghat(zeta_k) = g(x) on [-1,1] for the
    # entire transform ghat(z) = s sqrt(pi) exp(-s^2 z^2/4 - i z x0) of
    # g(x) = exp(-(x - x0)^2 / s^2)
    H = choose_H(1e-12, 0.0, 0.0, 1)
    z, w, info = gamma_rule(M, H, nu, 8, 7, 16, 2)
    assert info["N"] == 2 * info["NE"] + 16 + 64
    x = free_grid(M)
    s, x0 = 0.15, 0.2
    ghat = s * np.sqrt(np.pi) * np.exp(-s ** 2 * z ** 2 / 4 - 1j * z * x0)
    approx = (np.exp(1j * np.outer(x, z)) @ (w * ghat)) / (2 * np.pi)
    assert np.max(np.abs(approx - np.exp(-(x - x0) ** 2 / s ** 2))) < 1e-13


def _wavepacket(x, t, sig):
    # eq. (wavepacket) with k0 = 0, divided by sigma so that ||u0|| = 1
    s = sig ** 2 + 2j * t
    return sig ** 1.5 / np.pi ** 0.25 / np.sqrt(s) * np.exp(-(x / np.sqrt(2)) ** 2 / s) / sig


@pytest.mark.parametrize("E0", [0.0, 20.0])
def test_free_wavepacket_exact(E0):
    # V = 0: the scheme applies the exact propagator on Gamma, so u(x,T) =
    # u_wp(x + phi(T), T) to quadrature accuracy (Section 6, Example 2)
    M, nu, T = 128, 1024, 0.1
    x = free_grid(M)
    prob = Problem(name="wp", dim=1, domain="free", M=(M,), T=T, nsteps=20, order=8,
                   u0=_wavepacket(x, 0, 0.1).astype(complex), V_fields=[np.zeros(M)], f_kind=["const"],
                   f_params=[(0, 0)], A_kind="pulse_sin2" if E0 else "none",
                   A_params=(E0, 50.0, T, 1.0) if E0 else (), eps=1e-12, q=16, panels=2, nu=(nu,))
    orc = FreeSpaceOracle(prob)
    u, _ = orc.run()
    ph = orc.phi(T)[0]
    if E0:
        assert abs(ph) > 0.2
    assert np.max(np.abs(u - _wavepacket(x + ph, T, 0.1))) < 1e-12


def test_free_wavepacket_2d_exact():
    M, nu, T = 64, 512, 0.05
    x = free_grid(M)
    u0 = np.multiply.outer(_wavepacket(x - 0.1, 0, 0.12), _wavepacket(x + 0.05, 0, 0.1))
    prob = Problem(name="wp2", dim=2, domain="free", M=(M, M), T=T, nsteps=10, order=8, u0=u0.astype(complex),
                   V_fields=[np.zeros((M, M))], f_kind=["const"], f_params=[(0, 0)], A_kind="pulse_sin2",
                   A_params=(15.0, 40.0, T, 1.0, 0.0), eps=1e-12, q=16, panels=2, nu=(nu, nu))
    orc = FreeSpaceOracle(prob)
    u, _ = orc.run()
    ph = orc.phi(T)
    ex = np.multiply.outer(_wavepacket(x - 0.1 + ph[0], T, 0.12), _wavepacket(x + 0.05 + ph[1], T, 0.1))
    assert np.max(np.abs(u - ex)) < 1e-11


def test_round_trip_on_compactly_supported_function():
    prob = free_problem_from_seed(5, 1, (64,), 0.1, 10, nu=(512,), eps=1e-12, q=16, panels=2)
    orc = FreeSpaceOracle(prob)
    f = prob.u0
    assert np.max(np.abs(orc.Finv(orc.F(f)) - f)) < 1e-10


def test_free_space_eighth_order_in_time():
    # a potential resolved on the grid: self-convergence ratio ~2^8 per halving
    # of dt until rounding (Section 6, Examples 3 and 4 report eighth order)
    x = free_grid(32)
    sols = {}
    for N in (80, 160, 320, 1280):
        prob = free_problem_from_seed(6, 1, (32,), 0.05, N, nu=(256,), eps=1e-13, q=16, panels=2)
        prob.V_fields = [-5 * np.exp(-x ** 2 / 0.3 ** 2) * (1 - x ** 2) ** 4]
        sols[N], _ = FreeSpaceOracle(prob, H=2.0).run()
    ref = sols[1280]
    e1, e2, e3 = (np.linalg.norm(sols[N] - ref) for N in (80, 160, 320))
    assert e1 / e2 > 120 and e3 < 1e-12, (e1, e2, e3)


def test_H_rule():
    # Remark on the choice of H: log(eps / ((1 + ||V||) eps_m)) / (2 d (1 + phimax))
    H = choose_H(1e-10, 3.0, 0.5, 2)
    assert abs(H - np.log(1e-10 / (4.0 * 2.0 ** -52)) / 6.0) < 1e-14


# --- evaluation at arbitrary points (Remark on evaluation outside [-1,1]) ---

def _wp_problem(M, nu, T, nsteps, E0):
    x = free_grid(M)
    return Problem(name="wp", dim=1, domain="free", M=(M,), T=T, nsteps=nsteps, order=8,
                   u0=_wavepacket(x, 0, 0.1).astype(complex), V_fields=[np.zeros(M)], f_kind=["const"],
                   f_params=[(0, 0)], A_kind="pulse_sin2" if E0 else "none",
                   A_params=(E0, 50.0, T, 1.0) if E0 else (), eps=1e-12, q=16, panels=2, nu=(nu,))


@pytest.mark.parametrize("E0", [0.0, 20.0])
def test_far_evaluation_matches_exact_wavepacket_outside_the_box(E0):
    # V = 0: uhat(T) on Gamma_K is the exact transform times the exact
    # propagator, so the representation gives the exact wave packet at any
    # real x; by T = 0.1 the packet has spread well past [-1,1]
    prob = _wp_problem(128, 1024, 0.1, 20, E0)
    orc = FreeSpaceOracle(prob)
    _, info = orc.run()
    ph = orc.phi(0.1)[0]
    xs = np.linspace(-2.0, 2.0, 161)
    ex = _wavepacket(xs + ph, 0.1, 0.1)
    assert np.max(np.abs(ex[np.abs(xs) > 1.2])) > 0.3
    got = orc.evaluate(info["uhat"], [xs])
    assert np.max(np.abs(got - ex)) < 2e-11
    # the error grows with |x| - 1 as exp(H (|x| - 1)) amplifies the
    # truncation and rounding on Gamma_K; at |x| = 3 it is still below 1e-7
    xs3 = np.array([-3.0, -2.5, 2.5, 3.0])
    assert np.max(np.abs(orc.evaluate(info["uhat"], [xs3]) - _wavepacket(xs3 + ph, 0.1, 0.1))) < 1e-7


def test_far_evaluation_2d_exact_wavepacket():
    M, nu, T = 64, 512, 0.05
    x = free_grid(M)
    u0 = np.multiply.outer(_wavepacket(x - 0.1, 0, 0.12), _wavepacket(x + 0.05, 0, 0.1))
    prob = Problem(name="wp2", dim=2, domain="free", M=(M, M), T=T, nsteps=10, order=8, u0=u0.astype(complex),
                   V_fields=[np.zeros((M, M))], f_kind=["const"], f_params=[(0, 0)], A_kind="pulse_sin2",
                   A_params=(15.0, 40.0, T, 1.0, 0.0), eps=1e-12, q=16, panels=2, nu=(nu, nu))
    orc = FreeSpaceOracle(prob)
    _, info = orc.run()
    ph = orc.phi(T)
    px, py = np.linspace(-1.6, 1.6, 23), np.linspace(-1.8, 1.4, 19)
    ex = np.multiply.outer(_wavepacket(px - 0.1 + ph[0], T, 0.12), _wavepacket(py + 0.05 + ph[1], T, 0.1))
    assert np.max(np.abs(orc.evaluate(info["uhat"], [px, py]) - ex)) < 1e-11


def test_far_evaluation_at_grid_points_reproduces_the_marched_solution():
    # with V != 0 the mode state at T is B_N - i mu_0 dt F(V u_N) while the
    # marched grid values are F^-1(B_N) / (1 + i mu_0 dt V): the two agree on
    # the grid to the accuracy of F applied to V u (1.5e-9 here), and flipping
    # the sign of the V term breaks the agreement by O(mu_0 dt |V u|) (5e-2)
    prob = free_problem_from_seed(5, 1, (64,), 0.1, 10, nu=(512,), eps=1e-12, q=16, panels=2)
    orc = FreeSpaceOracle(prob)
    u, info = orc.run()
    x = free_grid(64)
    got = orc.evaluate(info["uhat"], [x])
    assert np.max(np.abs(got - u)) < 1e-8      # 1.5e-9 measured
    W = orc.F(orc.V(prob.T) * u)
    wrong = orc.evaluate(info["uhat"] + 2j * orc.mu[0] * prob.dt * W, [x])
    assert np.max(np.abs(wrong - u)) > 1e-4
