"""GPU parity of the 3D free-space path (Section 4.3: the line transforms of
Section 4.1 along each of the three axes, the 125 node-type subsets in tensor
order) through the C ABI: against the oracle on small grids (order 2 and the
order-4 start-up), against the stored oracle samples of the 32^3, 100-step
order-8 workload, and step-in-pieces / graph replay bitwise.

Bar: relative L2 <= 1e-11 against the oracle."""
import os

import numpy as np
import pytest

from oracle.freespace import FreeSpaceOracle
from workloads import free_3d_32_problem, free_problem_from_seed
from workloads.golden import load_samples, sampled_error

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


def _plan(prob):
    from paper_2001_06113_amd.tdse import Plan

    return Plan.from_problem(prob, device="cuda:0")


CASES = [
    dict(seed=61, M=(8, 10, 8), nu=(256, 256, 256), N=2, order=2, q=4),
    dict(seed=64, M=(16, 12, 20), nu=(256, 512, 256), N=3, order=2, q=6),
    dict(seed=65, M=(12, 16, 8), nu=(256, 256, 256), N=4, order=4, q=4),   # start-up and one Adams step
    # N_C = 32 > NT = 24 on every axis: the C-type block through the interpolant
    dict(seed=67, M=(8, 8, 10), nu=(256, 256, 256), N=2, order=2, q=8, panels=2, nt=24),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c['M']}-{c['nu']}-o{c['order']}" for c in CASES])
def test_3d_free_space_matches_oracle(case):
    print(f"case 3d free {case}", flush=True)
    from paper_2001_06113_amd.tdse import Q_FS_AXIS2, Q_FS_CHEB

    prob = free_problem_from_seed(case["seed"], 3, case["M"], 0.02, case["N"], order=case["order"], nu=case["nu"],
                                  eps=1e-8, q=case["q"], panels=case.get("panels", 1))
    plan = _plan(prob)
    nt = [int(plan.query(Q_FS_CHEB + a if a < 2 else Q_FS_AXIS2 + 6)) for a in range(3)]
    u = plan.run(prob.u0).cpu().numpy()
    plan.close()
    orc = FreeSpaceOracle(prob)
    assert nt == orc.NT == [case.get("nt", 0)] * 3
    ref, _ = orc.run()
    e = _rel(u, ref)
    print(f"  rel-L2 = {e:.3e}", flush=True)
    assert e < TOL


def test_3d_free_space_field_on_every_axis_matches_oracle():
    # a stepwise field with components on all three axes: every axis' phase
    # increment (the row factor's axis-0 and middle-axis parts, the last axis)
    prob = free_problem_from_seed(69, 3, (8, 10, 12), 0.03, 5, order=4, nu=(256, 256, 256), eps=1e-8, q=4, panels=1)
    rng = np.random.default_rng(69)
    t = (np.arange(prob.nsteps) + 0.5) / prob.nsteps
    prob.A_kind = "stepwise"
    prob.A_steps = rng.uniform(-8.0, 8.0, size=3)[None, :] * np.sin(2 * np.pi * t)[:, None]
    prob.A_params = ()
    plan = _plan(prob)
    u = plan.run(prob.u0).cpu().numpy()
    plan.close()
    orc = FreeSpaceOracle(prob)
    assert all(abs(x) > 1e-4 for x in orc.phi(0.5 * prob.T))
    ref, _ = orc.run()
    assert _rel(u, ref) < TOL


def test_3d_free_space_sampled_potential_matches_oracle():
    # a general V(x, t) given by samples at the step times (the free-space
    # moving well of sampled_potential_problem) on a 3D plan
    from workloads import sampled_potential_problem

    base = free_problem_from_seed(68, 3, (10, 8, 8), 0.02, 3, order=2, nu=(256, 256, 256), eps=1e-8, q=4, panels=1)
    prob = sampled_potential_problem(base)
    plan = _plan(prob)
    u = plan.run(prob.u0).cpu().numpy()
    plan.close()
    ref, _ = FreeSpaceOracle(prob).run()
    assert _rel(u, ref) < TOL


def test_3d_free_space_pieces_and_graph_replay_bitwise():
    import torch

    prob = free_problem_from_seed(66, 3, (8, 12, 10), 0.03, 10, order=8, nu=(256, 256, 256), eps=1e-8, q=4)
    plan = _plan(prob)
    full = plan.run(prob.u0).cpu().numpy()
    plan.set_state(prob.u0)
    for k in (3, 4, 3):
        plan.step(k)
    assert np.array_equal(plan.get_state().cpu().numpy(), full)
    plan.use_graph(True)
    for _ in range(2):
        g = plan.run(prob.u0).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(g, full)
    plan.close()


def test_3d_free_32_full_run_against_stored_oracle_samples():
    # the benchmarked 32^3 workload, 100 order-8 steps, the plan's default H
    prob = free_3d_32_problem()
    print("case 3d free 32^3 100 steps", flush=True)
    plan = _plan(prob)
    plan.use_graph(True)
    u = plan.run(prob.u0).cpu().numpy()
    plan.close()
    e = sampled_error(u, load_samples("free_3d_32")[0])
    print(f"  sampled rel-L2 = {e['rel_l2']:.3e}, max-abs {e['max_abs_rel']:.3e}, norm {e['norm_rel']:.3e}", flush=True)
    assert e["rel_l2"] < TOL and e["max_abs_rel"] < TOL and e["norm_rel"] < TOL
