"""GPU parity of the persistent 2D Adams steps (one co-resident grid per run
of a square 2D periodic FP64 plan) through the C ABI: against the oracle on
small and mid sizes, against the two-pass path at 512 x 512, and in pieces.
The full-length 512 x 512 run against the stored oracle samples is in
test_gpu_bench_configs.py (the persistent path is the default)."""
import os

import numpy as np
import pytest

from oracle.periodic import PeriodicOracle
from workloads import periodic_problem_from_seed

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


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _plan(prob):
    from paper_2001_06113_amd.tdse import Plan

    return Plan.from_problem(prob, device="cuda:0")


CASES = [
    dict(seed=40, M=32, T=0.05, N=14, order=8),
    dict(seed=41, M=64, T=0.04, N=30, order=8, dir2=True),
    dict(seed=44, M=128, T=0.05, N=25, order=6, A_kind="stepwise"),
    dict(seed=45, M=256, T=0.05, N=40, order=8),
    dict(seed=46, M=512, T=0.02, N=20, order=8, dir2=True),
]


def _problem(case):
    prob = periodic_problem_from_seed(case["seed"], 2, (case["M"], case["M"]), case["T"], case["N"],
                                      order=case["order"], A_kind=case.get("A_kind", "pulse_sin2"))
    if case.get("dir2"):
        E0, om, Tp = prob.A_params[:3]
        prob.A_params = (E0, om, Tp, 0.6, -0.8)
    if prob.A_kind == "stepwise":
        rng = np.random.default_rng(case["seed"])
        prob.A_steps = rng.uniform(-1, 1, size=(prob.nsteps, 2))
    return prob


@pytest.mark.parametrize("case", CASES, ids=[f"{c['M']}-{c['N']}-o{c['order']}" for c in CASES])
def test_persistent_matches_oracle(case):
    from paper_2001_06113_amd.tdse import Q_PATH, Q_PROF_N_PERSIST

    prob = _problem(case)
    print(f"case persistent 2D M={prob.M} steps={prob.nsteps} order={prob.order}", flush=True)
    plan = _plan(prob)
    assert plan.query(Q_PATH) == 2.0
    plan.profile(True)
    u = plan.run(prob.u0).cpu().numpy()
    launches = plan.query(Q_PROF_N_PERSIST)
    plan.close()
    r = rel(u, PeriodicOracle(prob).run()[0])
    print(f"  persistent launches {launches:.0f}, rel-L2 vs oracle {r:.3e}", flush=True)
    assert launches == 1.0
    assert r <= 1e-11


def test_persistent_equals_two_pass_512():
    import torch

    from paper_2001_06113_amd.tdse import CFG_PERSISTENT, Q_PATH

    prob = periodic_problem_from_seed(1, 2, (512, 512), 0.2, 200)
    print("case persistent vs two-pass 512^2, 200 steps", flush=True)
    plan = _plan(prob)
    plan.use_graph(True)
    a = plan.run(prob.u0).clone()
    b = plan.run(prob.u0).clone()
    plan.configure(CFG_PERSISTENT, 0)
    assert plan.query(Q_PATH) == 0.0
    c = plan.run(prob.u0).clone()
    torch.cuda.synchronize()
    plan.close()
    assert torch.equal(a, b)
    r = (torch.linalg.vector_norm(a - c) / torch.linalg.vector_norm(c)).item()
    print(f"  rel-L2 persistent vs two passes {r:.3e}", flush=True)
    assert r <= 1e-13


def test_persistent_in_pieces():
    prob = _problem(CASES[1])
    plan = _plan(prob)
    full = plan.run(prob.u0).cpu().numpy()
    traj = PeriodicOracle(prob).run(keep=True)[1]["us"]
    plan.set_state(prob.u0)
    done = 0
    for k in (2, 6, 1, 9, 12):
        print(f"case persistent pieces: step {k} from {done}", flush=True)
        plan.step(k)
        done += k
        got = plan.get_state().cpu().numpy()
        assert rel(got, traj[done]) <= 1e-11, done
    assert np.array_equal(got, full)
    plan.close()
