"""GPU parity of the 3D periodic FP64 path (the periodic scheme of Section 2
on an M0 x M1 x M2 grid) through the C ABI: against the oracle on small and
mid-size grids, against the stored oracle samples of the 128^3, 500-step
workload, and step-in-pieces / graph replay bitwise.

Bar: relative L2 <= 1e-11 against the oracle."""
import ctypes as C
import os

import numpy as np
import pytest

from oracle.periodic import PeriodicOracle
from workloads import periodic_3d_128_problem, periodic_problem_from_seed
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


def _stepwise3(prob, seed):
    rng = np.random.default_rng(seed)
    t = (np.arange(prob.nsteps) + 0.5) / prob.nsteps
    base = rng.uniform(-3.0, 3.0, size=3)
    prob.A_kind = "stepwise"
    prob.A_steps = base[None, :] * np.sin(2 * np.pi * t)[:, None] + rng.uniform(-0.5, 0.5, size=(prob.nsteps, 3))
    prob.A_params = ()
    return prob


def _plan(prob):
    from paper_2001_06113_amd.tdse import Plan

    return Plan.from_problem(prob, device="cuda:0")


CASES = [
    dict(seed=40, M=(8, 8, 8), T=0.05, N=12, order=8),
    dict(seed=41, M=(16, 24, 8), T=0.06, N=14, order=8, stepwise=True),
    dict(seed=42, M=(24, 16, 8), T=0.04, N=9, order=6, stepwise=True),
    dict(seed=43, M=(32, 8, 16), T=0.05, N=4, order=8),
    dict(seed=44, M=(8, 32, 24), T=0.05, N=7, order=2, stepwise=True),
    dict(seed=47, M=(64, 64, 64), T=0.05, N=20, order=8, stepwise=True),
    dict(seed=48, M=(32, 48, 128), T=0.04, N=16, order=8),
    dict(seed=49, M=(128, 16, 256), T=0.03, N=10, order=8, stepwise=True),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c['M']}-{c['N']}-o{c['order']}" for c in CASES])
def test_3d_matches_oracle(case):
    print(f"case 3d {case}", flush=True)
    prob = periodic_problem_from_seed(case["seed"], 3, case["M"], case["T"], case["N"], order=case["order"])
    if case.get("stepwise"):
        _stepwise3(prob, case["seed"])
    plan = _plan(prob)
    u = plan.run(prob.u0).cpu().numpy()
    plan.close()
    ref, _ = PeriodicOracle(prob).run()
    e = _rel(u, ref)
    print(f"  rel-L2 = {e:.3e}", flush=True)
    assert e < TOL


def test_3d_pieces_and_graph_replay_bitwise():
    import torch

    prob = _stepwise3(periodic_problem_from_seed(45, 3, (32, 16, 64), 0.06, 16), 45)
    plan = _plan(prob)
    full = plan.run(prob.u0).cpu().numpy()
    plan.set_state(prob.u0)
    for k in (3, 5, 8):
        plan.step(k)
    assert np.array_equal(plan.get_state().cpu().numpy(), full)
    plan.use_graph(True)
    for _ in range(2):
        g = plan.run(prob.u0).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(g, full)
    plan.close()


def test_3d_128_full_run_against_stored_oracle_samples():
    # the benchmarked 128^3 workload, 500 steps, exactly as the bench plans it
    prob = periodic_3d_128_problem()
    print("case 3d 128^3 500 steps", flush=True)
    plan = _plan(prob)
    plan.use_graph(True)
    u = plan.run(prob.u0).cpu().numpy()
    plan.close()
    e = sampled_error(u, load_samples("periodic_3d_128")[0])
    print(f"  sampled rel-L2 = {e['rel_l2']:.3e}, max-abs {e['max_abs_rel']:.3e}, norm {e['norm_rel']:.3e}", flush=True)
    assert e["rel_l2"] < TOL and e["max_abs_rel"] < TOL and e["norm_rel"] < TOL


SPLIT_CASES = [
    dict(seed=46, M=(8, 8, 8), T=0.05, N=12),
    dict(seed=51, M=(16, 24, 8), T=0.06, N=14, stepwise=True),
    dict(seed=52, M=(8, 16, 32), T=0.05, N=9),
    dict(seed=53, M=(64, 64, 64), T=0.05, N=20, stepwise=True),
    dict(seed=54, M=(128, 32, 48), T=0.04, N=16),
]


@pytest.mark.parametrize("case", SPLIT_CASES, ids=[f"split-{c['M']}-{c['N']}" for c in SPLIT_CASES])
def test_3d_split_matches_oracle(case):
    # FP32 transforms along all three axes, FP64 carried state: rel-L2 <= 1e-6
    print(f"case 3d split {case}", flush=True)
    prob = periodic_problem_from_seed(case["seed"], 3, case["M"], case["T"], case["N"], precision="fp32split")
    if case.get("stepwise"):
        _stepwise3(prob, case["seed"])
    plan = _plan(prob)
    u = plan.run(prob.u0).cpu().numpy()
    plan.close()
    ref, _ = PeriodicOracle(prob).run()
    e = _rel(u, ref)
    print(f"  rel-L2 = {e:.3e}", flush=True)
    assert 1e-12 < e < 1e-6


def test_3d_128_split_full_run_against_stored_oracle_samples():
    # the 128^3, 500-step workload with FP32 transforms, against the same
    # FP64 oracle samples, at the split bar
    prob = periodic_3d_128_problem()
    prob.precision = "fp32split"
    print("case 3d 128^3 split 500 steps", flush=True)
    plan = _plan(prob)
    plan.use_graph(True)
    u = plan.run(prob.u0).cpu().numpy()
    plan.close()
    e = sampled_error(u, load_samples("periodic_3d_128")[0])
    print(f"  sampled rel-L2 = {e['rel_l2']:.3e}, max-abs {e['max_abs_rel']:.3e}, norm {e['norm_rel']:.3e}", flush=True)
    assert e["rel_l2"] < 1e-6 and e["norm_rel"] < 1e-6
