"""GPU check of tdse_far_eval_noalloc, the allocation-free variant of
tdse_far_eval (workspace in the library's own device array): through the C
ABI, its output equals tdse_far_eval's on the same plan and points, for two
calls in a row, the second with fewer points; sizes past the array's limit are
refused before any device work."""
import os

import numpy as np
import pytest

from workloads import free_problem_from_seed

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


@pytest.mark.parametrize("dim,M,nu", [(2, (48, 96), (256, 1024)), (1, (256,), (2048,))])
def test_noalloc_far_eval_matches_workspace_entry_point(dim, M, nu):
    import torch

    from paper_2001_06113_amd.tdse import Plan

    prob = free_problem_from_seed(23, dim, M, 0.03, 10, nu=nu, eps=1e-11, q=10, panels=1)
    plan = Plan.from_problem(prob, device="cuda:0")
    plan.run(prob.u0)
    rng = np.random.default_rng(7)
    for call, (nx, ny) in enumerate([(131, 197), (29, 45)]):
        print(f"case noalloc far-eval dim={dim} M={M} call {call}: {nx} x {ny} points", flush=True)
        px, py = np.sort(rng.uniform(-2, 2, nx)), np.sort(rng.uniform(-2, 2, ny))
        xs = px if dim == 2 else None
        ref = plan.far_eval(py, xs).clone()
        got = plan.far_eval_noalloc(py, xs)
        torch.cuda.synchronize()
        diff = (got - ref).abs().max().item()
        scale = ref.abs().max().item()
        print(f"  max |noalloc - workspace| = {diff:.3e} (max |u| {scale:.3e})", flush=True)
        assert scale > 0
        assert diff <= 1e-11 * scale
    plan.close()


def test_noalloc_far_eval_refuses_sizes_past_its_array():
    import torch

    from paper_2001_06113_amd.tdse import Plan, TDSEError

    prob = free_problem_from_seed(23, 2, (48, 96), 0.03, 10, nu=(256, 1024), eps=1e-11, q=10, panels=1)
    plan = Plan.from_problem(prob, device="cuda:0")
    plan.run(prob.u0)
    big = np.linspace(-2, 2, 40000)
    with pytest.raises(TDSEError, match="library array"):
        plan.far_eval_noalloc(big, big[:200])
    torch.cuda.synchronize()
    plan.close()
