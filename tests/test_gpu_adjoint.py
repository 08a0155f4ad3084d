"""GPU parity of the adjoint (tdse_adjoint) through the C ABI and the torch
autograd Function: against the oracle's reverse sweep, finite differences of
the GPU forward and the exact dot-product test in u0."""
import os

import numpy as np
import pytest

from oracle.adjoint import adjoint, dipole, dipole_seed
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


def _plan(prob):
    from paper_2001_06113_amd.tdse import Plan

    return Plan.from_problem(prob, device="cuda:0")


CASES = [(1, (256,), 40, 0), (2, (64, 96), 30, 4), (2, (128, 32), 12, 1), (1, (512,), 5, 0)]


@pytest.mark.parametrize("dim,M,N,K", CASES)
def test_adjoint_matches_oracle(dim, M, N, K):
    prob = periodic_problem_from_seed(80, dim, M, 0.2, N, A_kind="stepwise")
    print(f"case adjoint {M} steps={N} K={K}", flush=True)
    u, _ = PeriodicOracle(prob).run()
    lam = dipole_seed(prob, u)
    gA, g0 = adjoint(prob, lam)
    plan = _plan(prob)
    eA, e0 = plan.adjoint(prob.u0, lam, K)
    e0 = e0.cpu().numpy()
    plan.close()
    rA = np.max(np.abs(eA - gA)) / np.max(np.abs(gA))
    r0 = np.linalg.norm(e0 - g0) / np.linalg.norm(g0)
    print(f"  dJ/dA rel {rA:.2e}, dJ/du0 rel {r0:.2e}", flush=True)
    assert rA <= 1e-10 and r0 <= 1e-10


def test_autograd_function_dipole_gradient():
    import torch

    from paper_2001_06113_amd.tdse import TDSEFunction

    prob = periodic_problem_from_seed(81, 2, (64, 64), 0.2, 25, A_kind="stepwise")
    plan = _plan(prob)
    A = torch.tensor(np.asarray(prob.A_steps), dtype=torch.float64, requires_grad=True)
    u0 = torch.as_tensor(prob.u0).to("cuda:0")
    uT = TDSEFunction.apply(A, plan, u0)
    x = torch.as_tensor(-np.pi + 2 * np.pi * np.arange(64) / 64, device="cuda:0").reshape(64, 1)
    w = (2 * np.pi / 64) ** 2
    J = w * torch.sum(x * torch.abs(uT) ** 2)
    J.backward()
    gA, _ = adjoint(prob, dipole_seed(prob, PeriodicOracle(prob).run()[0]))
    assert abs(J.item() - dipole(prob, PeriodicOracle(prob).run()[0])) < 1e-12
    r = np.max(np.abs(A.grad.numpy() - gA)) / np.max(np.abs(gA))
    print(f"case autograd 64^2: rel {r:.2e}", flush=True)
    assert r <= 1e-10
    plan.close()


def test_autograd_function_keeps_its_own_field():
    # two applications on one plan with different fields: backpropagating the
    # first output must use the first field, not the one the plan holds last
    import copy

    import torch

    from paper_2001_06113_amd.tdse import TDSEFunction

    prob = periodic_problem_from_seed(82, 1, (128,), 0.2, 30, A_kind="stepwise")
    other = copy.deepcopy(prob)
    other.A_steps = np.asarray(prob.A_steps)[::-1].copy() * -1.5
    plan = _plan(prob)
    u0 = torch.as_tensor(prob.u0).to("cuda:0")
    A1 = torch.tensor(np.asarray(prob.A_steps), dtype=torch.float64, requires_grad=True)
    A2 = torch.tensor(np.asarray(other.A_steps), dtype=torch.float64, requires_grad=True)
    x = torch.as_tensor(-np.pi + 2 * np.pi * np.arange(128) / 128, device="cuda:0")
    w = 2 * np.pi / 128
    u1 = TDSEFunction.apply(A1, plan, u0)
    u2 = TDSEFunction.apply(A2, plan, u0)
    J1 = w * torch.sum(x * torch.abs(u1) ** 2)
    J1.backward()
    gA, _ = adjoint(prob, dipole_seed(prob, PeriodicOracle(prob).run()[0]))
    r = np.max(np.abs(A1.grad.numpy() - gA)) / np.max(np.abs(gA))
    print(f"case autograd twice on one plan: first field's gradient rel {r:.2e}", flush=True)
    assert r <= 1e-10
    J2 = w * torch.sum(x * torch.abs(u2) ** 2)
    J2.backward()
    gB, _ = adjoint(other, dipole_seed(other, PeriodicOracle(other).run()[0]))
    r2 = np.max(np.abs(A2.grad.numpy() - gB)) / np.max(np.abs(gB))
    print(f"  second field's gradient rel {r2:.2e}", flush=True)
    assert r2 <= 1e-10
    plan.close()


def test_batch_adjoint_streams_agree():
    # a batch's adjoints from 8 host threads on 8 streams (more instances than
    # workers) equal the one-stream run bit for bit: each instance's arithmetic
    # is the same on any stream and workspace slice
    from paper_2001_06113_amd.tdse import BatchPlan

    shapes = [(1, (64,)), (2, (64, 64)), (1, (256,)), (2, (128, 64)), (1, (2048,)), (2, (192, 256)),
              (1, (384,)), (2, (64, 128)), (1, (128,))]
    probs = [periodic_problem_from_seed(90 + i, d, M, 0.1, 30, A_kind="stepwise") for i, (d, M) in enumerate(shapes)]
    lams = [dipole_seed(p, PeriodicOracle(p).run()[0], axis=p.dim - 1) for p in probs]
    print("case batch adjoint on 1 and 8 streams", flush=True)
    b = BatchPlan.from_problems(probs, device="cuda:0")
    b.adjoint_streams(1)
    gA1, g01 = b.adjoint([p.u0 for p in probs], lams)
    g01 = g01.cpu().numpy()
    b.adjoint_streams(8)
    gA8, g08 = b.adjoint([p.u0 for p in probs], lams)
    g08 = g08.cpu().numpy()
    b.close()
    for x, y in zip(gA1, gA8):
        assert np.array_equal(x, y)
    assert np.array_equal(g01, g08)
    gA, _ = adjoint(probs[1], lams[1])
    r = np.max(np.abs(gA8[1] - gA)) / np.max(np.abs(gA))
    print(f"  instance 1 {probs[1].M}: vs oracle {r:.2e}", flush=True)
    assert r <= 1e-10


def test_batch_64_adjoint():
    # the 64-instance batch (FP32-split forward plans, 500 steps): the FP64
    # derivative of each instance's <x_1>(T) with respect to its 500 samples
    import torch

    from paper_2001_06113_amd.tdse import BatchPlan, Plan

    probs = batch_64_problems()
    p64s = batch_64_problems(precision="fp64")
    print("case 64-instance batch adjoint", flush=True)
    # seeds from the FP64 forward of every instance
    lams, uTs = [], []
    for p in p64s:
        pl = Plan.from_problem(p, device="cuda:0")
        uT = pl.run(p.u0).cpu().numpy()
        pl.close()
        uTs.append(uT)
        lams.append(dipole_seed(p, uT))
    b = BatchPlan.from_problems(probs, device="cuda:0")
    gAs, g0 = b.adjoint([p.u0 for p in probs], lams)
    g0s = [g.cpu().numpy() for g in b.unpack(g0)]
    b.close()
    assert len(gAs) == 64 and all(g.shape == (500, p.dim) for g, p in zip(gAs, probs))
    # the smallest 1D and 2D instances against the oracle's reverse sweep
    for i in (0, 32):
        gA, _ = adjoint(p64s[i], dipole_seed(p64s[i], PeriodicOracle(p64s[i]).run()[0]))
        r = np.max(np.abs(gAs[i] - gA)) / np.max(np.abs(gA))
        print(f"  instance {i} {probs[i].M}: vs oracle {r:.2e}", flush=True)
        assert r <= 1e-9
    # a 512 x 512 instance: central differences of the FP64 GPU forward, and the
    # dot-product test in u0 (J is quadratic in u0)
    i = 35
    p = p64s[i]
    pl = Plan.from_problem(p, device="cuda:0")

    def J(A=None, u0=None):
        if A is not None:
            pl.set_field(A)
        out = pl.run(p.u0 if u0 is None else u0).cpu().numpy()
        return dipole(p, out)

    scale = np.max(np.abs(gAs[i]))
    for m in (0, 3, 250, 499):
        h = 1e-4
        Ap = np.array(p.A_steps, dtype=float)
        Am = Ap.copy()
        Ap[m, 0] += h
        Am[m, 0] -= h
        fd = (J(A=Ap) - J(A=Am)) / (2 * h)
        print(f"  instance {i} A[{m}]: adjoint {gAs[i][m, 0]:.10e} FD {fd:.10e}", flush=True)
        assert abs(fd - gAs[i][m, 0]) <= 1e-6 * scale
    pl.set_field(np.asarray(p.A_steps, dtype=float))
    rng = np.random.default_rng(2)
    d = rng.standard_normal(p.u0.shape) + 1j * rng.standard_normal(p.u0.shape)
    fd = (J(u0=p.u0 + 1e-2 * d) - J(u0=p.u0 - 1e-2 * d)) / 2e-2
    dot = float(np.real(np.vdot(g0s[i], d)))
    print(f"  instance {i} u0 dot test: {fd:.12e} vs {dot:.12e}", flush=True)
    assert abs(fd - dot) <= 1e-9 * abs(fd)
    pl.close()
