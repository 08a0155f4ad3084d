"""GPU parity of potentials given as samples at the step times
(TDSE_V_SAMPLED: a general non-separable V(x, t), interpolated in time at
the start-up sub-steps) through the C ABI, against the oracle: periodic
1D/2D/3D in FP64 and FP32-split, free space 1D/2D, and a Gaussian well moving
through free space.

Bar: relative L2 <= 1e-11 (FP64), 1e-6 (split) against the oracle."""
import os

import numpy as np
import pytest

from oracle.freespace import FreeSpaceOracle
from oracle.periodic import PeriodicOracle
from workloads import free_grid, free_problem_from_seed, periodic_problem_from_seed, sampled_potential_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2001_06113_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2001_06113_amd import build

        build.build()
    yield


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _run(prob):
    from paper_2001_06113_amd.tdse import Plan

    plan = Plan.from_problem(prob, device="cuda:0")
    u = plan.run(prob.u0).cpu().numpy()
    plan.close()
    return u


CASES = [
    dict(domain="periodic", seed=70, M=(64,), T=0.05, N=14),
    dict(domain="periodic", seed=71, M=(32, 24), T=0.04, N=12),
    dict(domain="periodic", seed=72, M=(16, 8, 24), T=0.04, N=9),
    dict(domain="periodic", seed=73, M=(32,), T=0.05, N=5),
    dict(domain="periodic", seed=77, M=(512, 512), T=0.2, N=200),
    dict(domain="periodic", seed=78, M=(64, 64, 64), T=0.05, N=24),
    dict(domain="free", seed=74, M=(48,), T=0.03, N=12, nu=(512,)),
    dict(domain="free", seed=75, M=(24, 32), T=0.03, N=9, nu=(256, 256)),
    dict(domain="free", seed=79, M=(128, 96), T=0.05, N=40, nu=(1024, 512)),
]


def _problem(c):
    if c["domain"] == "periodic":
        base = periodic_problem_from_seed(c["seed"], len(c["M"]), c["M"], c["T"], c["N"])
    else:
        base = free_problem_from_seed(c["seed"], len(c["M"]), c["M"], c["T"], c["N"], nu=c["nu"], eps=1e-11,
                                      q=10, panels=2)
    return sampled_potential_problem(base)


@pytest.mark.parametrize("case", CASES, ids=[f"{c['domain']}-{c['M']}-{c['N']}" for c in CASES])
def test_sampled_potential_matches_oracle(case):
    print(f"case sampled {case}", flush=True)
    prob = _problem(case)
    u = _run(prob)
    orc = PeriodicOracle(prob) if case["domain"] == "periodic" else FreeSpaceOracle(prob)
    ref, _ = orc.run()
    e = _rel(u, ref)
    print(f"  rel-L2 = {e:.3e}", flush=True)
    assert e < 1e-11


def test_sampled_split_form():
    prob = _problem(dict(domain="periodic", seed=76, M=(256, 256), T=0.1, N=60))
    prob.precision = "fp32split"
    u = _run(prob)
    prob.precision = "fp64"
    ref, _ = PeriodicOracle(prob).run()
    assert _rel(u, ref) < 1e-6


def test_gaussian_well_moving_through_free_space():
    # the moving well of Section 6, Example 1, taken to free space (no
    # periodic images): a Gaussian well crossing [-1, 1] at constant speed,
    # given by samples; the bound state is dragged along
    M, N, T = 128, 400, 0.4
    base = free_problem_from_seed(80, 1, (M,), T, N, nu=(1024,), eps=1e-11, q=10, panels=2, A_kind="none")
    x = free_grid(M)
    V0, beta, c, x0 = 400.0, 0.06, 1.0, -0.2
    base.V_kind = "sampled"
    base.V_samples = np.stack([-V0 * np.exp(-(x - x0 - c * n * base.dt) ** 2 / (2 * beta ** 2)) for n in range(N + 1)])
    base.V_fields, base.f_kind, base.f_params = [], [], []
    base.u0 = (np.exp(-(x - x0) ** 2 / (2 * 0.05 ** 2))).astype(complex)
    u = _run(base)
    ref, _ = FreeSpaceOracle(base).run()
    assert _rel(u, ref) < 1e-11
    # the density follows the well: its centre of mass moved by about c T
    com0 = np.sum(x * np.abs(base.u0) ** 2) / np.sum(np.abs(base.u0) ** 2)
    com = np.sum(x * np.abs(u) ** 2) / np.sum(np.abs(u) ** 2)
    assert abs((com - com0) - c * T) < 0.1, (com0, com)
