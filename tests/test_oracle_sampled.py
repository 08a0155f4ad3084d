"""Pins of potentials given as samples at the step times (V_kind "sampled",
a general non-separable V(x, t)): the Lagrange window in time, and runs of
the scheme (Sections 2.2, 3.3) with sampled potentials against runs of the
same potential given in closed form."""
import copy

import numpy as np
import pytest

from oracle.freespace import FreeSpaceOracle
from oracle.periodic import PeriodicOracle
from oracle.potential import sampled_V, window
from workloads import (free_problem_from_seed, moving_well_problem, periodic_grid, periodic_problem_from_seed,
                       sampled_potential_problem)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("N", [3, 7, 20])
def test_window_reproduces_polynomials(N):
    # degree-7 (or N) Lagrange interpolation is exact on polynomials of that
    # degree, sums to one, and returns the sample itself at a step time
    dt = 0.013
    rng = np.random.default_rng(N)
    deg = min(7, N)
    coef = rng.standard_normal(deg + 1)
    samples = np.array([np.polyval(coef, n * dt) for n in range(N + 1)])[:, None] * np.ones((1, 3))
    for t in np.concatenate([rng.uniform(0, N * dt, 25), [0.0, 0.5 * dt, N * dt - 0.25 * dt]]):
        n0, w = window(t, dt, N)
        assert 0 <= n0 and n0 + len(w) <= N + 1
        assert abs(w.sum() - 1.0) < 1e-12
        assert np.max(np.abs(sampled_V(samples, t, dt) - np.polyval(coef, t))) < 1e-11 * np.max(np.abs(samples))
    for n in range(N + 1):
        n0, w = window(n * dt, dt, N)
        assert n0 == n and list(w) == [1.0]


def _as_sampled(prob, fn):
    p = copy.copy(prob)
    p.V_kind = "sampled"
    p.V_samples = np.stack([fn(n * prob.dt) for n in range(prob.nsteps + 1)])
    p.V_fields, p.f_kind, p.f_params = [], [], []
    return p


@pytest.mark.parametrize("dim", [1, 2])
def test_sampled_separable_potential_matches_fields_form(dim):
    # V = (1 + a sin(w t)) V0(x) given as samples: the interpolated V at the
    # start-up sub-steps differs from the closed form by O((w dt)^8), far below
    # the bar at w dt = 0.05
    M = (64,) if dim == 1 else (32, 48)
    prob = periodic_problem_from_seed(60 + dim, dim, M, 0.1, 40)
    ref, _ = PeriodicOracle(prob).run()
    orc = PeriodicOracle(prob)
    samp = _as_sampled(prob, orc.V)
    u, _ = PeriodicOracle(samp).run()
    assert _rel(u, ref) < 1e-12


def test_sampled_free_space_potential_matches_fields_form():
    prob = free_problem_from_seed(62, 1, (48,), 0.05, 20, nu=(512,), eps=1e-11, q=10, panels=2)
    ref, _ = FreeSpaceOracle(prob).run()
    orc = FreeSpaceOracle(prob)
    samp = _as_sampled(prob, orc.V)
    u, _ = FreeSpaceOracle(samp).run()
    assert _rel(u, ref) < 1e-12


def test_sampled_moving_well_matches_closed_form():
    # Example 1's moving well (non-separable in x and t) given as samples
    # against the closed-form image sum: the difference is the interpolation
    # error at the start-up sub-steps only, eighth order in dt
    diffs = []
    for N in (200, 400):
        prob = moving_well_problem(c=(30.0,), M=(128,), nsteps=N)
        ref, _ = PeriodicOracle(prob).run()
        orc = PeriodicOracle(prob)
        u, _ = PeriodicOracle(_as_sampled(prob, orc.V)).run()
        diffs.append(_rel(u, ref))
    assert diffs[0] / diffs[1] > 150 and diffs[1] < 1e-6, diffs
    # with the samples shifted by half a step the difference is visible
    # (negative control: the samples are where the recipe puts them)
    bad = _as_sampled(prob, lambda t: orc.V(t + 0.5 * prob.dt))
    assert _rel(PeriodicOracle(bad).run()[0], ref) > 1e-3


@pytest.mark.parametrize("domain", ["periodic", "free"])
def test_sampled_recipe_converges_eighth_order(domain):
    # the general sampled potential of the recipe: self-convergence in dt at
    # about 2^8 per halving (the interpolation keeps the scheme's order)
    sols = {}
    Ns = (40, 80, 160, 640) if domain == "periodic" else (160, 320, 640, 2560)
    for N in Ns:
        if domain == "periodic":
            base = periodic_problem_from_seed(63, 1, (64,), 0.2, N)
            sols[N], _ = PeriodicOracle(sampled_potential_problem(base)).run()
        else:
            base = free_problem_from_seed(64, 1, (48,), 0.1, N, nu=(512,), eps=1e-12, q=10, panels=2)
            sols[N], _ = FreeSpaceOracle(sampled_potential_problem(base), H=2.0).run()
    ref = sols[Ns[-1]]
    e1, e2 = (np.linalg.norm(sols[N] - ref) for N in Ns[:2])
    assert e1 / e2 > 100, (e1, e2)
