"""Pins of the oracle's reverse-mode derivative of the periodic scheme.

dJ/du0: J is a quadratic form in u0 for a fixed field, so the central
difference (J(u0 + e d) - J(u0 - e d)) / 2e equals Re <dJ/du0, d> up to
rounding for any e.  dJ/dA: central differences of the forward oracle.  With
V = 0 the scheme is exact and u(x, T) = u_free(x + phi(T), T) (Lemma 1), so
<x_a>(T) = <x_a>_free(T) - phi_a(T) ||u||^2 and every dJ/dA_m,b equals
-dt ||u||^2 delta_ab for a packet far from the box edges."""
import copy

import numpy as np
import pytest

from oracle.adjoint import adjoint, dipole, dipole_seed
from oracle.periodic import PeriodicOracle
from workloads import periodic_problem_from_seed


def _J(prob, A=None, u0=None, axis=0):
    p = copy.copy(prob)
    if A is not None:
        p.A_steps = A
    if u0 is not None:
        p.u0 = u0
    u, _ = PeriodicOracle(p).run()
    return dipole(p, u, axis)


CASES = [(1, (64,), 12, 8), (2, (24, 32), 10, 8), (1, (48,), 4, 8), (2, (16, 16), 9, 4)]


@pytest.mark.parametrize("dim,M,N,order", CASES)
def test_adjoint_initial_state_dot_product(dim, M, N, order):
    prob = periodic_problem_from_seed(70, dim, M, 0.1, N, order=order, A_kind="stepwise")
    u, _ = PeriodicOracle(prob).run()
    _, g0 = adjoint(prob, dipole_seed(prob, u))
    rng = np.random.default_rng(1)
    d = rng.standard_normal(prob.u0.shape) + 1j * rng.standard_normal(prob.u0.shape)
    fd = (_J(prob, u0=prob.u0 + 1e-2 * d) - _J(prob, u0=prob.u0 - 1e-2 * d)) / 2e-2
    assert abs(fd - np.real(np.vdot(g0, d))) <= 1e-10 * abs(fd)


@pytest.mark.parametrize("dim,M,N,order", CASES)
def test_adjoint_field_gradient_finite_differences(dim, M, N, order):
    prob = periodic_problem_from_seed(71, dim, M, 0.1, N, order=order, A_kind="stepwise")
    u, _ = PeriodicOracle(prob).run()
    gA, _ = adjoint(prob, dipole_seed(prob, u))
    scale = np.max(np.abs(gA))
    for m in sorted({0, 1, N // 2, N - 1}):
        for a in range(dim):
            h = 1e-4
            Ap = np.array(prob.A_steps, dtype=float)
            Am = Ap.copy()
            Ap[m, a] += h
            Am[m, a] -= h
            fd = (_J(prob, A=Ap) - _J(prob, A=Am)) / (2 * h)
            assert abs(fd - gA[m, a]) <= 1e-7 * scale, (m, a, fd, gA[m, a])


@pytest.mark.parametrize("dim", [1, 2])
def test_adjoint_free_particle_closed_form(dim):
    # sigma = 0.3 at the box centre, T = 0.05: the packet's tails at +-pi stay ~1e-20
    M = (96,) if dim == 1 else (64, 64)
    prob = periodic_problem_from_seed(72, dim, M, 0.05, 14, A_kind="stepwise")
    prob.V_fields = [np.zeros(M)]
    X = np.meshgrid(*[-np.pi + 2 * np.pi * np.arange(m) / m for m in M], indexing="ij")
    u0 = np.exp(-sum(x ** 2 for x in X) / 0.3 ** 2).astype(np.complex128)
    prob.u0 = u0 / np.sqrt(np.prod([2 * np.pi / m for m in M]) * np.sum(np.abs(u0) ** 2))
    u, _ = PeriodicOracle(prob).run()
    w = float(np.prod([2 * np.pi / m for m in M]))
    norm2 = w * np.sum(np.abs(u) ** 2)
    for axis in range(dim):
        gA, _ = adjoint(prob, dipole_seed(prob, u, axis))
        expect = np.zeros_like(gA)
        expect[:, axis] = -prob.dt * norm2
        assert np.max(np.abs(gA - expect)) < 1e-12
