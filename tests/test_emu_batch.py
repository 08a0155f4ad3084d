"""CPU run of the batched passes (one launch per pass and schedule family
over many instances) through the emulation harness: every instance of a
mixed batch against the oracle, stepping in pieces, per-instance state
access, the autotuner's bookkeeping and the planner's validation."""
import ctypes as C

import numpy as np
import pytest

from oracle.periodic import PeriodicOracle
from workloads import periodic_problem_from_seed


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _mixed(prec, T=0.05, N=10):
    return [periodic_problem_from_seed(50, 1, (64,), T, N, precision=prec, A_kind="stepwise"),
            periodic_problem_from_seed(51, 2, (64, 128), T, N, precision=prec),
            periodic_problem_from_seed(52, 2, (192, 64), 0.8 * T, N, precision=prec, A_kind="stepwise"),
            periodic_problem_from_seed(53, 1, (384,), 1.2 * T, N, precision=prec)]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32split", 1e-6)])
def test_emulated_batch_matches_oracle(emu, prec, tol):
    from emu.emu_plan import EmuBatchPlan

    probs = _mixed(prec)
    outs = EmuBatchPlan(emu, probs).run([p.u0 for p in probs])
    for p, u in zip(probs, outs):
        ref, _ = PeriodicOracle(p).run()
        assert _rel(u, ref) < tol, p.M


def test_emulated_batch_pieces_instances_and_autotune(emu):
    from emu.emu_plan import EmuBatchPlan

    probs = _mixed("fp64", N=9)
    b = EmuBatchPlan(emu, probs)
    full = b.run([p.u0 for p in probs])
    assert b.query(4) == 4.0
    assert b.query(0) == sum(int(np.prod(p.M)) for p in probs)
    # per-instance set, stepping in pieces that end inside start-up and Adams phases
    for i, p in enumerate(probs):
        u0 = np.ascontiguousarray(p.u0, dtype=np.complex128)
        b.call("tdse_set_instance_state", i, C.c_void_p(u0.ctypes.data), 1)
    for k in (2, 5, 1, 1):
        b.call("tdse_step", k)
    for i, p in enumerate(probs):
        u = np.zeros(p.M, dtype=np.complex128)
        b.call("tdse_get_instance_state", i, C.c_void_p(u.ctypes.data), 1)
        assert np.array_equal(u, full[i]), i
    # the autotuner keeps a compiled schedule per instance and leaves the plan runnable
    b.call("tdse_autotune", 2)
    for i, p in enumerate(probs):
        col = b.query(8192 + i)
        row = b.query(12288 + i)
        assert (p.M[0] if p.dim == 2 else 1) % col == 0 and p.M[-1] % row == 0
    again = b.run([p.u0 for p in probs])
    for p, u, f in zip(probs, again, full):
        assert _rel(u, f) < 1e-13


def test_batch_planner_validation(emu):
    from emu.emu_plan import EmuBatchPlan

    a = periodic_problem_from_seed(60, 1, (64,), 0.05, 10)
    with pytest.raises(RuntimeError, match="share"):
        EmuBatchPlan(emu, [a, periodic_problem_from_seed(61, 1, (64,), 0.05, 12)])      # nsteps differ
    with pytest.raises(RuntimeError, match="share"):
        EmuBatchPlan(emu, [a, periodic_problem_from_seed(61, 1, (64,), 0.05, 10, order=6)])
    with pytest.raises(RuntimeError, match="batched line lengths"):
        EmuBatchPlan(emu, [a, periodic_problem_from_seed(62, 2, (32, 64), 0.05, 10)])    # 32 not compiled
