"""GPU parity of the free-space path with the C-type transforms through the
Chebyshev interpolant (Section 4.1, eqs. (expintrpm)/(expintrpp); the (C,E)
and (C,C) subsets of Section 4.2 in tensor order) through the C ABI: against
the oracle, which evaluates the interpolant in the paper's coefficient form,
and, for the long-time wave packet of Section 6, Example 2, against the exact
solution.

Bar: relative L2 <= 1e-11 against the oracle."""
import os

import numpy as np
import pytest

from oracle.freespace import FreeSpaceOracle
from workloads import example2_long_time_problem, free_problem_from_seed
from workloads import wavepacket as _wavepacket

pytestmark = pytest.mark.gpu

TOL = 1e-11


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
    from paper_2001_06113_amd.tdse import Q_FS_CHEB, Plan

    plan = Plan.from_problem(prob, device="cuda:0")
    nt = [int(plan.query(Q_FS_CHEB + a)) for a in range(prob.dim)]
    u = plan.run(prob.u0).cpu().numpy()
    plan.close()
    return u, nt


@pytest.mark.parametrize("nr", [1, 2, 3, 4, 5])
def test_example2_long_time(nr):
    # T = 1000, q = 16, n_r = 1..5, 1000 steps: the GPU run equals the oracle
    # at every depth, and at n_r = 5 both are the exact wave packet
    prob = example2_long_time_problem(nr, cheb=0, nsteps=1000)
    print(f"example 2 long time n_r={nr}", flush=True)
    orc = FreeSpaceOracle(prob)
    u, nt = _run(prob)
    assert nt == orc.NT and nt[0] > 0
    ref, _ = orc.run()
    e = _rel(u, ref)
    ex = _wavepacket(orc.xs[0] + orc.phi(prob.T)[0], prob.T, 0.1)
    print(f"  NT={nt[0]} rel vs oracle {e:.2e}, vs exact {_rel(u, ex):.2e}", flush=True)
    assert e < TOL
    if nr == 5:
        assert _rel(u, ex) < 1e-13


CASES = [
    dict(seed=30, dim=1, M=(64,), nu=(512,), T=0.04, N=10, q=16, panels=5, cheb=0),     # N_C = 160
    dict(seed=31, dim=1, M=(48,), nu=(256,), T=0.05, N=9, q=12, panels=2, cheb=30),     # forced NT
    dict(seed=35, dim=1, M=(256,), nu=(2048,), T=0.05, N=24, q=32, panels=8, cheb=0),   # N_C = 512
    dict(seed=32, dim=2, M=(32, 24), nu=(256, 256), T=0.04, N=9, q=16, panels=3, cheb=0),
    dict(seed=33, dim=2, M=(16, 40), nu=(256, 512), T=0.03, N=8, q=8, panels=4, cheb=0, order=6),
    dict(seed=36, dim=2, M=(128, 96), nu=(1024, 1024), T=0.03, N=14, q=16, panels=4, cheb=0),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c['M']}-q{c['q']}x{c['panels']}-cheb{c['cheb']}" for c in CASES])
def test_chebyshev_matches_oracle(case):
    print(f"chebyshev case {case}", flush=True)
    prob = free_problem_from_seed(case["seed"], case["dim"], case["M"], case["T"], case["N"], nu=case["nu"],
                                  order=case.get("order", 8), eps=1e-11, q=case["q"], panels=case["panels"])
    prob.cheb = case["cheb"]
    orc = FreeSpaceOracle(prob)
    u, nt = _run(prob)
    assert nt == orc.NT and all(nt)
    ref, _ = orc.run()
    assert _rel(u, ref) < TOL


def test_interpolant_and_direct_sums_agree():
    # the same plan with the C-type block both ways: equal to rounding
    prob = free_problem_from_seed(37, 2, (64, 64), 0.04, 12, nu=(512, 512), eps=1e-11, q=16, panels=3)
    prob.cheb = -1
    ud, nt = _run(prob)
    assert nt == [0, 0]
    prob.cheb = 0
    uc, nt = _run(prob)
    assert all(nt)
    assert _rel(uc, ud) < 1e-12
