"""CPU run of the HIP kernels and the C ABI through the emulation harness
(tests/emu): same sources, compiled for the host, against the oracle.  This
checks indexing, tiling, ragged tails and the step sequence without a GPU."""
import numpy as np
import pytest

from oracle.periodic import PeriodicOracle
from workloads import periodic_problem_from_seed


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [
    dict(seed=3, dim=2, M=(16, 24), T=0.05, N=12),
    dict(seed=3, dim=2, M=(96, 8), T=0.05, N=10),             # ragged row tiles
    dict(seed=4, dim=2, M=(8, 48), T=0.05, N=10, A_kind="stepwise"),
    dict(seed=3, dim=1, M=(384,), T=0.05, N=10),              # radix 3
    dict(seed=5, dim=2, M=(24, 16), T=0.05, N=9, order=4),
    dict(seed=6, dim=2, M=(16, 16), T=0.04, N=4, order=6),
    dict(seed=7, dim=1, M=(64,), T=0.02, N=2, order=2),
    dict(seed=8, dim=1, M=(32,), T=0.07, N=7),                # ends right after start-up
    dict(seed=9, dim=2, M=(8, 8), T=0.03, N=3, A_kind="none"),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c['M']}-{c['N']}-{c.get('order', 8)}" for c in CASES])
def test_emulated_kernels_match_oracle(emu, case):
    from emu.emu_plan import EmuPlan

    prob = periodic_problem_from_seed(case["seed"], case["dim"], case["M"], case["T"], case["N"],
                                      order=case.get("order", 8), A_kind=case.get("A_kind", "pulse_sin2"))
    u = EmuPlan(emu, prob).run(prob.u0)
    ref, _ = PeriodicOracle(prob).run()
    assert _rel(u, ref) < 1e-12


SPLIT_CASES = [
    dict(seed=11, dim=2, M=(16, 32), T=0.05, N=12),
    dict(seed=12, dim=1, M=(128,), T=0.05, N=10),
    dict(seed=13, dim=2, M=(24, 8), T=0.05, N=8, order=4),
]


@pytest.mark.parametrize("case", SPLIT_CASES, ids=[f"split-{c['M']}-{c['N']}" for c in SPLIT_CASES])
def test_emulated_split_precision_within_bar(emu, case):
    # complex64 transforms and history with FP64 carried state: within 1e-6
    from emu.emu_plan import EmuPlan

    prob = periodic_problem_from_seed(case["seed"], case["dim"], case["M"], case["T"], case["N"],
                                      order=case.get("order", 8), precision="fp32split")
    u = EmuPlan(emu, prob).run(prob.u0)
    ref, _ = PeriodicOracle(prob).run()
    r = _rel(u, ref)
    assert r < 1e-6, r
    assert r > 1e-12   # really ran in reduced precision


def test_emulated_split_long_run_high_potential(emu):
    # the 1D instance of the 64-instance workload with the largest |V| (about
    # 19) over its 500 steps: rounded history weights or a rounded potential
    # would perturb every step alike and push the error past 2e-6
    from emu.emu_plan import EmuPlan
    from workloads import batch_64_problems

    prob = batch_64_problems()[12]
    u = EmuPlan(emu, prob).run(prob.u0)
    ref, _ = PeriodicOracle(prob).run()
    assert _rel(u, ref) < 1e-6


WELL_CASES = [
    dict(M=(64,), c=(15.0,), N=30, precision="fp64", tol=1e-12),
    dict(M=(16, 24), c=(15.0, -7.5), N=20, precision="fp64", tol=1e-12),
    dict(M=(64,), c=(45.0,), N=30, precision="fp32split", tol=1e-6),
    dict(M=(16, 24), c=(15.0, -7.5), N=20, precision="fp64", tol=1e-12, beta=0.8),   # one image per side
]


@pytest.mark.parametrize("case", WELL_CASES, ids=[f"well-{c['M']}-{c['precision']}-b{c.get('beta', 0.2)}" for c in WELL_CASES])
def test_emulated_moving_well_matches_oracle(emu, case):
    # the moving periodic Gaussian well (Example 1), evaluated on the fly in
    # the column pass, against the oracle's image sum
    from emu.emu_plan import EmuPlan
    from workloads import moving_well_problem

    prob = moving_well_problem(c=case["c"], M=case["M"], T=0.05, nsteps=case["N"], precision=case["precision"],
                               beta=case.get("beta", 0.2))
    u = EmuPlan(emu, prob).run(prob.u0)
    ref, _ = PeriodicOracle(prob).run()
    assert _rel(u, ref) < case["tol"]
