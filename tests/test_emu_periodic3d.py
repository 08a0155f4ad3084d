"""CPU run of the 3D periodic path (the periodic scheme of Section 2 on an
M0 x M1 x M2 grid: row passes over the last axis, column passes over axis 0,
FFT-only passes over the middle axis) through the emulation harness, against
the oracle."""
import ctypes as C

import numpy as np
import pytest

from oracle.periodic import PeriodicOracle
from workloads import periodic_problem_from_seed


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _stepwise3(prob, seed):
    rng = np.random.default_rng(seed)
    t = (np.arange(prob.nsteps) + 0.5) / prob.nsteps
    base = rng.uniform(-3.0, 3.0, size=3)
    prob.A_kind = "stepwise"
    prob.A_steps = base[None, :] * np.sin(2 * np.pi * t)[:, None] + rng.uniform(-0.5, 0.5, size=(prob.nsteps, 3))
    prob.A_params = ()
    return prob


CASES = [
    dict(seed=40, M=(8, 8, 8), T=0.05, N=12, order=8),
    dict(seed=41, M=(16, 24, 8), T=0.06, N=14, order=8, stepwise=True),
    dict(seed=42, M=(24, 16, 8), T=0.04, N=9, order=6, stepwise=True),
    dict(seed=43, M=(32, 8, 16), T=0.05, N=4, order=8),                      # ends inside the start-up
    dict(seed=44, M=(8, 32, 24), T=0.05, N=7, order=2, stepwise=True),      # trapezoid steps only
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c['M']}-{c['N']}-o{c['order']}" for c in CASES])
def test_emulated_3d_matches_oracle(emu, case):
    from emu.emu_plan import EmuPlan

    prob = periodic_problem_from_seed(case["seed"], 3, case["M"], case["T"], case["N"], order=case["order"])
    if case.get("stepwise"):
        _stepwise3(prob, case["seed"])
    plan = EmuPlan(emu, prob)
    u = plan.run(prob.u0)
    ref, _ = PeriodicOracle(prob).run()
    assert _rel(u, ref) < 1e-12


def test_emulated_3d_steps_in_pieces(emu):
    from emu.emu_plan import EmuPlan

    prob = _stepwise3(periodic_problem_from_seed(45, 3, (16, 8, 24), 0.06, 16), 45)
    plan = EmuPlan(emu, prob)
    full = plan.run(prob.u0)
    plan.set_state(prob.u0)
    for k in (3, 5, 8):
        plan.step(k)
    out = np.zeros(prob.M, dtype=np.complex128)
    plan.call("tdse_get_state", C.c_void_p(out.ctypes.data), 1)
    assert np.array_equal(out, full)


SPLIT_CASES = [
    dict(seed=46, M=(8, 8, 8), T=0.05, N=12),
    dict(seed=51, M=(16, 24, 8), T=0.06, N=14, stepwise=True),
    dict(seed=52, M=(8, 16, 32), T=0.05, N=9),                   # two split steps after the start-up
]


@pytest.mark.parametrize("case", SPLIT_CASES, ids=[f"split-{c['M']}-{c['N']}" for c in SPLIT_CASES])
def test_emulated_3d_split_matches_oracle(emu, case):
    # FP32 transforms along all three axes, FP64 carried state: the split bar
    from emu.emu_plan import EmuPlan

    prob = periodic_problem_from_seed(case["seed"], 3, case["M"], case["T"], case["N"], precision="fp32split")
    if case.get("stepwise"):
        _stepwise3(prob, case["seed"])
    u = EmuPlan(emu, prob).run(prob.u0)
    ref, _ = PeriodicOracle(prob).run()
    r = _rel(u, ref)
    assert r < 1e-6, r
    assert r > 1e-12   # really ran in reduced precision
