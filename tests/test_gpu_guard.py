"""GPU checks of the failure guard (TDSE_CFG_GUARD: a device-side scan of the
state for non-finite entries every K steps, TDSE_ENONFINITE through
tdse_step and tdse_run) on every marching path, and of the history residual
(TDSE_Q_RESIDUAL) of the FP64 and split forms."""
import os

import numpy as np
import pytest

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


# 1D one-workgroup run, 2D persistent, 2D two passes (384 is not persistent), split
PATHS = [((256,), "fp64", 1.0), ((64, 64), "fp64", 2.0), ((384, 64), "fp64", 0.0), ((128, 96), "fp32split", 0.0)]


@pytest.mark.parametrize("M,prec,path", PATHS)
def test_guard_reports_a_non_finite_state(M, prec, path):
    from paper_2001_06113_amd.tdse import CFG_GUARD, Q_PATH, Q_STATE_NORM, Plan, TDSEError

    prob = periodic_problem_from_seed(70, len(M), M, 0.05, 20, precision=prec)
    print(f"case guard M={M} {prec}", flush=True)
    plan = Plan.from_problem(prob, device="cuda:0")
    assert plan.query(Q_PATH) == path
    plan.configure(CFG_GUARD, 7)
    u = plan.run(prob.u0).cpu().numpy()
    assert plan.query(Q_STATE_NORM) == pytest.approx(np.linalg.norm(u), rel=1e-12)
    bad = np.array(prob.u0, dtype=np.complex128)
    bad.flat[11] = np.nan
    with pytest.raises(TDSEError, match="not finite") as ei:
        plan.run(bad)
    assert ei.value.status == -5
    plan.use_graph(True)
    with pytest.raises(TDSEError, match="not finite"):
        plan.run(bad)
    good = plan.run(prob.u0).cpu().numpy()
    assert np.array_equal(good, u)
    plan.close()


@pytest.mark.parametrize("M,prec,lo,hi", [((512, 512), "fp64", 0.0, 1e-14), ((1024, 1024), "fp32split", 1e-9, 1e-5),
                                          ((256,), "fp64", 0.0, 1e-14)])
def test_history_residual(M, prec, lo, hi):
    from paper_2001_06113_amd.tdse import Q_RESIDUAL, Plan

    prob = periodic_problem_from_seed(71, len(M), M, 0.05, 30, precision=prec)
    plan = Plan.from_problem(prob, device="cuda:0")
    plan.set_state(prob.u0)
    plan.step(25)
    r = plan.query(Q_RESIDUAL)
    print(f"case residual M={M} {prec}: {r:.3e}", flush=True)
    assert lo <= r <= hi
    plan.close()
