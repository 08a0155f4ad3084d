"""GPU parity of the batched form: many independent periodic instances of
uneven sizes marched by batched launches (one per pass and schedule family),
through the C ABI.  Bars: FP64 relative L2 <= 1e-11 against the oracle; the
FP32-split form within 1e-6 of the oracle and of the FP64 GPU path."""
import os

import numpy as np
import pytest

from oracle.periodic import PeriodicOracle
from workloads import batch_64_problems, periodic_problem_from_seed

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


def batch(probs):
    from paper_2001_06113_amd.tdse import BatchPlan

    return BatchPlan.from_problems(probs, device="cuda:0")


def _mixed(prec, T=0.05, N=24):
    return [periodic_problem_from_seed(50, 1, (64,), T, N, precision=prec, A_kind="stepwise"),
            periodic_problem_from_seed(51, 2, (64, 128), T, N, precision=prec),
            periodic_problem_from_seed(52, 2, (192, 64), 0.8 * T, N, precision=prec, A_kind="stepwise"),
            periodic_problem_from_seed(53, 1, (384,), 1.2 * T, N, precision=prec),
            periodic_problem_from_seed(54, 2, (1536, 96 * 2), T, N, precision=prec),
            periodic_problem_from_seed(55, 1, (2048,), T, N, precision=prec)]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32split", 1e-6)])
def test_mixed_batch_matches_oracle(prec, tol):
    probs = _mixed(prec)
    print(f"case mixed batch {prec}: {[p.M for p in probs]}", flush=True)
    b = batch(probs)
    outs = [u.cpu().numpy() for u in b.run_list([p.u0 for p in probs])]
    b.close()
    for p, u in zip(probs, outs):
        r = rel(u, PeriodicOracle(p).run()[0])
        print(f"  {p.M}: rel-L2 {r:.3e}", flush=True)
        assert r <= tol, (p.M, r)


def test_batch_64_fp64_against_oracle():
    # all 64 instances of the uneven batch in FP64 for 10 steps; one instance
    # of each size against the oracle
    probs = batch_64_problems(T=0.04, nsteps=10, precision="fp64")
    print("case 64-instance batch geometry, FP64, 10 steps", flush=True)
    b = batch(probs)
    outs = b.run_list([p.u0 for p in probs])
    for i in (0, 1, 2, 3, 32, 33, 34, 35):
        r = rel(outs[i].cpu().numpy(), PeriodicOracle(probs[i]).run()[0])
        print(f"  instance {i} {probs[i].M}: rel-L2 {r:.3e}", flush=True)
        assert r <= 1e-11, (i, r)
    b.close()


def test_batch_64_split_autotuned():
    # the benchmarked configuration: 64 instances, 500 steps, FP32-split,
    # autotuned schedules, whole-run graph replay; every instance within 1e-6
    # of the FP64 GPU path, the smallest 1D and 2D ones against the oracle
    import torch

    from paper_2001_06113_amd.tdse import Plan

    probs = batch_64_problems()
    print("case 64-instance batch, full split run", flush=True)
    b = batch(probs)
    chosen = b.autotune(5)
    print(f"  schedules {sorted(set(chosen))}", flush=True)
    b.use_graph(True)
    u0 = b.pack([p.u0 for p in probs])
    first = b.run(u0).clone()
    again = b.run(u0)
    torch.cuda.synchronize()
    assert torch.equal(first, again)
    outs = [u.cpu().numpy() for u in b.unpack(first)]
    b.close()
    worst = 0.0
    for i, p64 in enumerate(batch_64_problems(precision="fp64")):
        pl = Plan.from_problem(p64, device="cuda:0")
        ref = pl.run(p64.u0).cpu().numpy()
        pl.close()
        worst = max(worst, rel(outs[i], ref))
    print(f"  worst rel-L2 vs FP64 GPU path: {worst:.3e}", flush=True)
    assert worst <= 1e-6
    for i in (0, 32):
        r = rel(outs[i], PeriodicOracle(probs[i]).run()[0])
        print(f"  instance {i} {probs[i].M} vs oracle: {r:.3e}", flush=True)
        assert r <= 1e-6


def test_batch_pieces_instance_state_and_graph():
    import torch

    probs = _mixed("fp64", N=15)
    b = batch(probs)
    full = b.run([p.u0 for p in probs]).clone()
    for i, p in enumerate(probs):
        b.set_instance_state(i, p.u0)
    for k in (3, 4, 1, 7):
        b.step(k)
    assert torch.equal(b.get_state(), full)
    for i, p in enumerate(probs):
        assert torch.equal(b.get_instance_state(i), b.unpack(full)[i])
    b.use_graph(True)
    for _ in range(3):
        assert torch.equal(b.run([p.u0 for p in probs]), full)
        b.use_graph(False)
        assert torch.equal(b.run([p.u0 for p in probs]), full)
        b.use_graph(True)
    b.close()
