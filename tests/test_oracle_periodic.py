"""Pins of the periodic oracle against facts the paper and the mathematics fix.

None of these compares the oracle with itself: each uses a closed form, an
invariant, a textbook value, an independent ODE solver or a value printed in
the paper.
"""
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle.adams import adams_coefficients, richardson_extrapolate
from oracle.periodic import PeriodicOracle, make_phi
from workloads import Problem, periodic_grid, periodic_problem_from_seed

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- constants (P8)

def test_am8_matches_table1():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "am8_table1.txt")) if l.strip() and not l.startswith("#")]
    printed = [Fraction(int(n), int(d)) for _, n, d in rows]
    assert adams_coefficients(8) == printed


def test_am_low_orders_textbook():
    # second order is the trapezoid rule (Section 2.2); 3rd/4th order are the
    # classical Adams-Moulton weights
    assert adams_coefficients(2) == [Fraction(1, 2), Fraction(1, 2)]
    assert adams_coefficients(3) == [Fraction(5, 12), Fraction(8, 12), Fraction(-1, 12)]
    assert adams_coefficients(4) == [Fraction(9, 24), Fraction(19, 24), Fraction(-5, 24), Fraction(1, 24)]
    for n in range(1, 11):
        assert sum(adams_coefficients(n)) == 1


def test_am_exact_on_polynomials():
    # an n-point implicit Adams rule integrates degree n-1 polynomials exactly
    for n in (2, 4, 6, 8):
        mu = adams_coefficients(n)
        for deg in range(n):
            # int_{-1}^{0} s^deg ds vs sum_j mu_j (-j)^deg
            exact = Fraction((-1) ** deg, deg + 1)
            assert sum(mu[j] * Fraction(-j) ** deg for j in range(n)) == exact
        deg = n
        exact = Fraction((-1) ** deg, deg + 1)
        assert sum(mu[j] * Fraction(-j) ** deg for j in range(n)) != exact


# ---------------------------------------------------------------- Richardson (P9)

def test_richardson_local_order_nine():
    lam = -0.7 + 2.3j

    def trap(h, nsub):
        y = 1.0 + 0j
        for _ in range(nsub):
            y = y * (1 + lam * h / 2) / (1 - lam * h / 2)
        return y

    errs = []
    for dt in (0.4, 0.2, 0.1):
        U = [trap(dt / 2 ** l, 2 ** l) for l in range(4)]
        errs.append(abs(richardson_extrapolate(U) - np.exp(lam * dt)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    # local error O(dt^9): ratio -> 2^9 = 512
    assert 330 < r1 < 640 and 400 < r2 < 600, (r1, r2)


# ---------------------------------------------------------------- helpers

def _gauss_problem(M, T, nsteps, order=8, x0=(0.3,), sig=0.5, V=None, f=None, A=None, images=3):
    """Unnormalised periodised Gaussian u0 with known Fourier coefficients."""
    d = len(M)
    axes = [periodic_grid(m) for m in M]
    X = np.meshgrid(*axes, indexing="ij")
    u0 = np.ones(M, dtype=np.complex128)
    for a in range(d):
        s = np.zeros(M)
        for m in range(-images, images + 1):
            s += np.exp(-(X[a] - x0[a] - 2 * np.pi * m) ** 2 / sig ** 2)
        u0 = u0 * s
    Vf = [np.zeros(M)] if V is None else [V]
    fk, fp = (["const"], [(0.0, 0.0)]) if f is None else (["sin"], [f])
    p = Problem(name="t", dim=d, domain="periodic", M=tuple(M), T=T, nsteps=nsteps, order=order,
                u0=u0, V_fields=Vf, f_kind=fk, f_params=fp)
    if A is not None:
        p.A_kind = "pulse_sin2"
        p.A_params = tuple(A)
    return p


def _pulse_phi(t, E0, om, Tp):
    """Closed form of int_0^t E0 sin^2(pi s/Tp) sin(om s) ds."""
    Om = 2 * np.pi / Tp

    def c(w):  # (1 - cos(w t)) / w
        return 2 * np.sin(w * t / 2) ** 2 / w if w != 0 else 0.0

    return 0.5 * E0 * (c(om) - 0.5 * (c(om + Om) + c(om - Om)))


def _exact_free(M, t, x0, sig, shift):
    """Free-particle solution of the periodised Gaussian by its Fourier series
    (Poisson summation: c_k = sig/(2 sqrt(pi)) exp(-sig^2 k^2/4 - i k x0))."""
    d = len(M)
    out = None
    kk = np.arange(-200, 201)
    for a in range(d):
        x = periodic_grid(M[a])
        ck = sig / (2 * np.sqrt(np.pi)) * np.exp(-sig ** 2 * kk ** 2 / 4 - 1j * kk * x0[a])
        ph = np.exp(-1j * kk ** 2 * t + 1j * kk * shift[a])
        ua = (ck * ph)[None, :] * np.exp(1j * np.outer(x, kk))
        ua = ua.sum(axis=1)
        out = ua if out is None else np.multiply.outer(out, ua)
    return out


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ---------------------------------------------------------------- P1/P2 exact free evolution

@pytest.mark.parametrize("M", [(64,), (48, 64)])
def test_free_particle_exact(M):
    d = len(M)
    x0 = (0.3, -0.8)[:d]
    T, N = 0.7, 35
    p = _gauss_problem(M, T, N, x0=x0, sig=0.55)
    u, _ = PeriodicOracle(p).run()
    ex = _exact_free(M, T, x0, 0.55, (0.0,) * d)
    assert _rel(u, ex) < 1e-12


@pytest.mark.parametrize("M", [(64,), (64, 48)])
def test_free_particle_with_advection_exact(M):
    d = len(M)
    x0 = (-0.4, 0.6)[:d]
    T, N = 0.5, 40
    E0, om = 3.0, 11.0
    direction = (1.0, 0.0) if d == 2 else (1.0,)
    p = _gauss_problem(M, T, N, x0=x0, sig=0.5, A=(E0, om, T) + tuple(direction) + ((0.0,) if d == 1 else ()))
    u, _ = PeriodicOracle(p).run()
    shift = (_pulse_phi(T, E0, om, T), 0.0)[:d]
    ex = _exact_free(M, T, x0, 0.5, shift)
    assert _rel(u, ex) < 1e-12


def test_phi_quadrature_matches_closed_form():
    p = periodic_problem_from_seed(7, 2, (8, 8), 2.0, 200)
    E0, om, Tp = p.A_params[:3]
    phi = make_phi(p)
    for t in (0.0, 0.0137, 0.5, 1.2345, 2.0):
        got = phi(t)
        assert abs(got[0] - _pulse_phi(t, E0, om, Tp)) < 1e-14
        assert got[1] == 0.0


# ---------------------------------------------------------------- P3 uniform V(t)

def test_uniform_time_dependent_potential():
    # V(x,t) = c0 (1 + a sin(w t)) is a gauge phase: u = exp(-i int c) * free solution
    M = (48,)
    c0, amp, om = 6.0, 0.3, 9.0
    T = 1.0
    gauge = np.exp(-1j * c0 * (T + amp * (1 - np.cos(om * T)) / om))
    ex = gauge * _exact_free(M, T, (0.2,), 0.5, (0.0,))
    errs = []
    for N in (100, 200):
        p = _gauss_problem(M, T, N, x0=(0.2,), sig=0.5, V=np.full(M, c0), f=(amp, om))
        u, _ = PeriodicOracle(p).run()
        errs.append(_rel(u, ex))
    # converges to the exact gauge solution at eighth order
    assert errs[1] < 3e-11 and errs[0] / errs[1] > 150, errs


# ---------------------------------------------------------------- P4 trapezoid invariant

def test_trapezoid_cayley_norm_conserved():
    # order 2: ||(1 + i dt/2 V(t_n)) u_n|| is exactly conserved for real V
    p = periodic_problem_from_seed(11, 1, (64,), 1.0, 100, order=2)
    orc = PeriodicOracle(p)
    u, info = orc.run(keep=True)
    dt = p.dt
    vals = [np.linalg.norm((1 + 0.5j * dt * orc.V(n * dt)) * un) for n, un in enumerate(info["us"])]
    assert np.ptp(vals) / vals[0] < 1e-13
    # the plain norm is not conserved by the scheme: make sure the test has teeth
    norms = [np.linalg.norm(un) for un in info["us"]]
    assert np.ptp(norms) / norms[0] > 1e-8


# ---------------------------------------------------------------- independent ODE solve

def _semidiscrete_reference(p, T):
    """Solve i uhat' = (k^2 - k A(t)) uhat + F(V(t) F^-1 uhat) with DOP853 in
    the interaction picture v = exp(i k^2 t - i k phi(t)) uhat."""
    M = p.M[0]
    k = np.fft.fftfreq(M) * M
    phi = make_phi(p)

    def Vt(t):
        return sum(p.f(r, t) * Vr for r, Vr in enumerate(p.V_fields))

    def rhs(t, y):
        v = y[:M] + 1j * y[M:]
        ph = np.exp(-1j * k * k * t + 1j * k * phi(t)[0])
        uh = ph * v
        u = np.fft.ifft(uh) * M
        w = np.fft.fft(Vt(t) * u) / M
        dv = -1j * np.conj(ph) * w
        return np.concatenate([dv.real, dv.imag])

    uh0 = np.fft.fft(p.u0) / M
    sol = solve_ivp(rhs, (0, T), np.concatenate([uh0.real, uh0.imag]), method="DOP853", rtol=1e-13, atol=1e-15)
    v = sol.y[:M, -1] + 1j * sol.y[M:, -1]
    uh = np.exp(-1j * k * k * T + 1j * k * phi(T)[0]) * v
    return np.fft.ifft(uh) * M


def test_matches_independent_ode_solver():
    p = periodic_problem_from_seed(21, 1, (32,), 0.4, 400)
    u, _ = PeriodicOracle(p).run()
    ref = _semidiscrete_reference(p, p.T)
    assert _rel(u, ref) < 1e-10


# ---------------------------------------------------------------- P6 eighth order in time

def test_eighth_order_self_convergence():
    # eighth order in dt (Section 6, Example 1): error ratio -> 2^8 = 256 per
    # halving once every well-resolved mode has |k|^2 dt small
    sols = {}
    for N in (50, 100, 200, 800):
        p = periodic_problem_from_seed(5, 1, (48,), 0.2, N)
        sols[N], _ = PeriodicOracle(p).run()
    ref = sols[800]
    e1, e2, e3 = (np.linalg.norm(sols[N] - ref) for N in (50, 100, 200))
    r1, r2 = e1 / e2, e2 / e3
    assert r1 > 120 and r2 > 180, (r1, r2, e1, e2, e3)


# ---------------------------------------------------------------- P7 spectral in space

def test_spectral_convergence_in_space():
    # same continuous problem sampled on finer grids: u(T) at the coarse grid
    # points converges faster than any power of 1/M
    def solve(M):
        p = _gauss_problem((M,), 0.3, 30, x0=(0.1,), sig=0.35,
                           V=-3.0 * np.cos(periodic_grid(M)) - 2.0 * np.cos(2 * periodic_grid(M)))
        u, _ = PeriodicOracle(p).run()
        return u

    ref = solve(256)
    errs = []
    for M in (32, 48, 64):
        u = solve(M)
        step = 256 // M if 256 % M == 0 else None
        if step is None:
            continue
        errs.append(np.max(np.abs(u - ref[::step])))
    assert errs[0] > 1e3 * errs[1], errs


# ---------------------------------------------------------------- transform convention

def test_transform_is_the_printed_dft():
    # eq. (ftperdisc): fhat_k = (1/M) sum_j exp(-2 pi i j k / M) f_j, k = -M/2..M/2-1
    M = 8
    p = _gauss_problem((M,), 1.0, 10)
    orc = PeriodicOracle(p)
    rng = np.random.default_rng(0)
    f = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    got = orc.F(f)
    for k in range(-M // 2, M // 2):
        direct = sum(np.exp(-2j * np.pi * j * k / M) * f[j] for j in range(M)) / M
        assert abs(got[k % M] - direct) < 1e-14
    back = orc.Finv(got)
    assert np.max(np.abs(back - f)) < 1e-14
    # the mode index used in the phases is k in [-M/2, M/2)
    assert orc.K[0][M // 2] == -M // 2
