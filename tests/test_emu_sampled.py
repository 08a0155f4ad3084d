"""CPU run of potentials given as samples at the step times (TDSE_V_SAMPLED:
a general non-separable V(x, t)) through the emulation harness, against the
oracle: periodic 1D/2D/3D, the FP32-split form, free space 1D/2D."""
import numpy as np
import pytest

from oracle.freespace import FreeSpaceOracle
from oracle.periodic import PeriodicOracle
from workloads import free_problem_from_seed, periodic_problem_from_seed, sampled_potential_problem


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [
    dict(domain="periodic", seed=70, M=(64,), T=0.05, N=14),
    dict(domain="periodic", seed=71, M=(32, 24), T=0.04, N=12),
    dict(domain="periodic", seed=72, M=(16, 8, 24), T=0.04, N=9),
    dict(domain="periodic", seed=73, M=(32,), T=0.05, N=5),        # fewer than eight samples
    dict(domain="free", seed=74, M=(48,), T=0.03, N=12, nu=(512,)),
    dict(domain="free", seed=75, M=(24, 32), T=0.03, N=9, nu=(256, 256)),
]


def _problem(c):
    if c["domain"] == "periodic":
        base = periodic_problem_from_seed(c["seed"], len(c["M"]), c["M"], c["T"], c["N"])
    else:
        base = free_problem_from_seed(c["seed"], len(c["M"]), c["M"], c["T"], c["N"], nu=c["nu"], eps=1e-11,
                                      q=10, panels=2)
    return sampled_potential_problem(base)


@pytest.mark.parametrize("case", CASES, ids=[f"{c['domain']}-{c['M']}-{c['N']}" for c in CASES])
def test_emulated_sampled_potential_matches_oracle(emu, case):
    from emu.emu_plan import EmuPlan

    prob = _problem(case)
    u = EmuPlan(emu, prob).run(prob.u0)
    orc = PeriodicOracle(prob) if case["domain"] == "periodic" else FreeSpaceOracle(prob)
    ref, _ = orc.run()
    assert _rel(u, ref) < 1e-12


def test_emulated_sampled_split_form(emu):
    from emu.emu_plan import EmuPlan

    prob = _problem(dict(domain="periodic", seed=76, M=(64, 64), T=0.04, N=12))
    prob.precision = "fp32split"
    u = EmuPlan(emu, prob).run(prob.u0)
    prob.precision = "fp64"
    ref, _ = PeriodicOracle(prob).run()
    assert _rel(u, ref) < 1e-6
