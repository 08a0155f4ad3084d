"""CPU run of the one-workgroup 1D path (run1d_kernels.hip: the start-up and
the implicit Adams steps of a 1D periodic FP64 plan in one launch) through the
emulation harness, against the oracle, and its step-in-pieces contract."""
import numpy as np
import pytest

from oracle.periodic import PeriodicOracle
from workloads import moving_well_problem, periodic_problem_from_seed


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [
    dict(seed=20, M=(64,), T=0.06, N=24, order=8),                       # pulse field, Adams phase
    dict(seed=21, M=(128,), T=0.05, N=16, order=4, A_kind="stepwise"),
    dict(seed=22, M=(256,), T=0.04, N=12, order=6, A_kind="none"),
    dict(seed=23, M=(8,), T=0.05, N=10, order=8),                        # shortest line
    dict(seed=24, M=(512,), T=0.03, N=9, order=8),                       # longest line of the path
    dict(seed=25, M=(32,), T=0.05, N=4, order=8),                        # ends inside the start-up
    dict(seed=26, M=(64,), T=0.05, N=11, order=8, n_start=8),            # longer start-up
    dict(seed=27, M=(16,), T=0.05, N=6, order=2),                        # no start-up, trapezoid steps
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c['M']}-{c['N']}-o{c['order']}" for c in CASES])
def test_run1d_matches_oracle(emu, case):
    from emu.emu_plan import EmuPlan

    prob = periodic_problem_from_seed(case["seed"], 1, case["M"], case["T"], case["N"], order=case["order"],
                                      A_kind=case.get("A_kind", "pulse_sin2"))
    prob.n_start = case.get("n_start")
    plan = EmuPlan(emu, prob)
    plan.call("tdse_profile", 1)
    u = plan.run(prob.u0)
    assert plan.query(25) == 1.0    # the whole run was one launch of the one-workgroup kernel
    assert plan.query(11) == 0.0    # and no row pass
    ref, _ = PeriodicOracle(prob).run()
    assert _rel(u, ref) < 1e-12


def test_run1d_two_fields_and_moving_well(emu):
    from emu.emu_plan import EmuPlan

    prob = periodic_problem_from_seed(30, 1, (64,), 0.05, 14)
    prob.V_fields = [prob.V_fields[0], 0.5 * np.cos(2 * prob.grid(0))]
    prob.f_kind = ["sin", "sin"]
    prob.f_params = [prob.f_params[0], (0.3, 7.0)]
    u = EmuPlan(emu, prob).run(prob.u0)
    assert _rel(u, PeriodicOracle(prob).run()[0]) < 1e-12
    well = moving_well_problem(c=(30.0,), M=(128,), T=0.05, nsteps=20)
    u = EmuPlan(emu, well).run(well.u0)
    assert _rel(u, PeriodicOracle(well).run()[0]) < 1e-12


@pytest.mark.parametrize("pieces", [(3, 4, 1, 12), (1, 1, 1, 1, 1, 1, 14), (7, 13)])
def test_run1d_steps_in_pieces(emu, pieces):
    # any split of the run into tdse_step calls gives the whole run's u(T)
    # bit for bit, and the state after each piece is the oracle's u at that time
    from emu.emu_plan import EmuPlan

    prob = periodic_problem_from_seed(31, 1, (128,), 0.06, 20)
    plan = EmuPlan(emu, prob)
    full = plan.run(prob.u0)
    plan.set_state(prob.u0)
    done = 0
    traj = PeriodicOracle(prob).run(keep=True)[1]["us"]
    for k in pieces:
        plan.step(k)
        done += k
        out = np.zeros(prob.M, dtype=np.complex128)
        import ctypes as C

        plan.call("tdse_get_state", C.c_void_p(out.ctypes.data), 1)
        assert _rel(out, traj[done]) < 1e-12, done
    assert np.array_equal(out, full)
