"""CPU checks (emulation harness) of the failure guard, the history residual
and the free-space parameter queries of the C ABI."""
import ctypes as C

import numpy as np
import pytest

from workloads import free_problem_from_seed, periodic_problem_from_seed

ENONFINITE, ESTATE = -5, -6
CFG_GUARD, Q_RESIDUAL, Q_STATE_NORM = 1, 29, 30


def test_guard_stops_a_non_finite_run(emu):
    from emu.emu_plan import EmuPlan

    for M in ((64,), (16, 24)):
        prob = periodic_problem_from_seed(60, len(M), M, 0.05, 12)
        plan = EmuPlan(emu, prob)
        plan.call("tdse_configure", CFG_GUARD, 4)
        u = plan.run(prob.u0)                           # a finite run passes every check
        assert plan.query(Q_STATE_NORM) == pytest.approx(np.linalg.norm(u), rel=1e-12)
        bad = np.array(prob.u0, dtype=np.complex128).copy()
        bad.flat[3] = np.nan
        plan.set_state(bad)
        st = emu.tdse_step(plan.h, 5)
        assert st == ENONFINITE, st
        assert "not finite" in emu.tdse_last_error().decode()
        plan.call("tdse_configure", CFG_GUARD, 0)       # unguarded, the NaN runs through silently
        plan.set_state(bad)
        assert emu.tdse_step(plan.h, 5) == 0


def test_guard_on_a_batch(emu):
    from emu.emu_plan import EmuBatchPlan

    probs = [periodic_problem_from_seed(61 + i, d, M, 0.05, 9) for i, (d, M) in enumerate([(1, (64,)), (2, (64, 64))])]
    b = EmuBatchPlan(emu, probs)
    b.call("tdse_configure", CFG_GUARD, 3)
    outs = b.run([p.u0 for p in probs])
    assert np.isfinite(b.query(Q_STATE_NORM))
    bad = [np.array(p.u0, dtype=np.complex128) for p in probs]
    bad[1].flat[7] = np.inf
    with pytest.raises(RuntimeError, match="not finite"):
        b.run(bad)
    assert all(np.all(np.isfinite(u)) for u in outs)


@pytest.mark.parametrize("prec,lo,hi", [("fp64", 0.0, 1e-14), ("fp32split", 1e-9, 1e-5)])
def test_history_residual(emu, prec, lo, hi):
    from emu.emu_plan import EmuPlan

    for M in ((128,), (32, 48)):
        prob = periodic_problem_from_seed(62, len(M), M, 0.05, 12, precision=prec)
        plan = EmuPlan(emu, prob)
        plan.set_state(prob.u0)
        v = C.c_double()
        assert emu.tdse_query(plan.h, Q_RESIDUAL, C.byref(v)) == ESTATE   # before the Adams start
        plan.step(9)
        r = plan.query(Q_RESIDUAL)
        assert lo <= r <= hi, (M, prec, r)
        plan.step(3)
        assert emu.tdse_query(plan.h, Q_RESIDUAL, C.byref(v)) == ESTATE   # at T


def test_free_space_parameter_queries(emu):
    from emu.emu_plan import EmuPlan

    prob = free_problem_from_seed(5, 2, (24, 32), 0.04, 9, nu=(256, 512), eps=1e-11, q=6, panels=2)
    plan = EmuPlan(emu, prob)
    for a, (M, nu) in enumerate(zip(prob.M, prob.nu)):
        h = plan.query(128 + a)
        assert h == pytest.approx(np.pi * M / nu, rel=1e-15)
        assert plan.query(130 + a) == nu
        NE, H = plan.query(83 + a), plan.query(86 + a)
        assert NE == nu // 2 - 13
        assert plan.query(132 + a) == pytest.approx(H + (14 + NE - 1) * h, rel=1e-15)
