"""CPU run of the library's adjoint (tdse_adjoint: checkpointed forward
recomputation, reverse Adams recurrence, reversed start-up sub-steps, phase
gradient reductions) through the emulation harness, against the oracle's
reverse sweep."""
import numpy as np
import pytest

from oracle.adjoint import adjoint, dipole_seed
from oracle.periodic import PeriodicOracle
from workloads import periodic_problem_from_seed

CASES = [
    dict(dim=1, M=(64,), N=12, order=8, K=0),
    dict(dim=1, M=(64,), N=12, order=8, K=2),
    dict(dim=2, M=(16, 24), N=14, order=8, K=3),
    dict(dim=1, M=(32,), N=4, order=8, K=0),       # ends inside the start-up
    dict(dim=1, M=(48,), N=7, order=8, K=0),       # one Adams step
    dict(dim=2, M=(16, 16), N=9, order=4, K=2),
    dict(dim=2, M=(24, 8), N=11, order=6, K=1),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c['M']}-{c['N']}-o{c['order']}-K{c['K']}" for c in CASES])
def test_emulated_adjoint_matches_oracle(emu, case):
    from emu.emu_plan import EmuPlan, emu_adjoint

    prob = periodic_problem_from_seed(70, case["dim"], case["M"], 0.1, case["N"], order=case["order"],
                                      A_kind="stepwise")
    u, _ = PeriodicOracle(prob).run()
    lam = dipole_seed(prob, u, axis=case["dim"] - 1)
    gA, g0 = adjoint(prob, lam)
    eA, e0 = emu_adjoint(EmuPlan(emu, prob), prob.u0, lam, case["K"])
    assert np.max(np.abs(eA - gA)) <= 1e-12 * np.max(np.abs(gA))
    assert np.linalg.norm(e0 - g0) <= 1e-12 * np.linalg.norm(g0)


def test_emulated_adjoint_of_split_plan_is_the_fp64_derivative(emu):
    from emu.emu_plan import EmuPlan, emu_adjoint

    p64 = periodic_problem_from_seed(73, 2, (16, 32), 0.1, 12, A_kind="stepwise")
    psp = periodic_problem_from_seed(73, 2, (16, 32), 0.1, 12, A_kind="stepwise", precision="fp32split")
    lam = dipole_seed(p64, PeriodicOracle(p64).run()[0])
    a64, _ = emu_adjoint(EmuPlan(emu, p64), p64.u0, lam)
    asp, _ = emu_adjoint(EmuPlan(emu, psp), psp.u0, lam)
    assert np.max(np.abs(asp - a64)) <= 1e-13 * np.max(np.abs(a64))


def test_adjoint_rejects_other_fields(emu):
    from emu.emu_plan import EmuPlan, emu_adjoint

    prob = periodic_problem_from_seed(74, 1, (32,), 0.1, 8)        # smooth pulse, not stepwise
    with pytest.raises(RuntimeError, match="stepwise"):
        emu_adjoint(EmuPlan(emu, prob), prob.u0, prob.u0)


def test_emulated_batch_adjoint_on_several_streams(emu):
    # a batch's adjoints run from several host threads, each on a stream and a
    # workspace slice of its own: every instance's result is the same whichever
    # worker computed it, and matches the oracle's reverse sweep
    from emu.emu_plan import EmuBatchPlan, emu_batch_adjoint

    shapes = [(1, (64,)), (2, (64, 64)), (1, (128,)), (1, (256,))]
    probs = [periodic_problem_from_seed(80 + i, d, M, 0.1, 10, A_kind="stepwise") for i, (d, M) in enumerate(shapes)]
    lams = [dipole_seed(p, PeriodicOracle(p).run()[0], axis=p.dim - 1) for p in probs]
    b = EmuBatchPlan(emu, probs)
    res, sizes = {}, {}
    for streams in (1, 3, 4):
        assert emu.tdse_adjoint_streams(b.h, streams) == 0
        res[streams] = emu_batch_adjoint(b, [p.u0 for p in probs], lams)
        import ctypes as C
        sz = C.c_size_t()
        assert emu.tdse_adjoint_workspace_size(b.h, 0, C.byref(sz)) == 0
        sizes[streams] = sz.value
    assert sizes[3] == 3 * sizes[1] and sizes[4] == 4 * sizes[1]
    for streams in (3, 4):
        for x, y in zip(res[1][0] + res[1][1], res[streams][0] + res[streams][1]):
            assert np.array_equal(x, y)
    for i, p in enumerate(probs):
        gA, g0 = adjoint(p, lams[i])
        assert np.max(np.abs(res[4][0][i] - gA)) <= 1e-12 * np.max(np.abs(gA))
        assert np.linalg.norm(res[4][1][i] - g0) <= 1e-12 * np.linalg.norm(g0)
    assert emu.tdse_adjoint_streams(b.h, 0) != 0
    assert emu.tdse_adjoint_streams(b.h, 17) != 0


def test_adjoint_rejects_the_moving_well(emu):
    # the adjoint's point kernels take the potential from stored fields
    from emu.emu_plan import EmuPlan, emu_adjoint
    from workloads import moving_well_problem

    prob = moving_well_problem(c=(15.0,), M=(64,), T=0.05, nsteps=8)
    with pytest.raises(RuntimeError, match="stored fields"):
        emu_adjoint(EmuPlan(emu, prob), prob.u0, prob.u0)
