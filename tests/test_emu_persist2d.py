"""CPU run of the persistent 2D Adams steps (persist2d_kernels.hip: one
co-resident grid, grid barriers between the transform directions, the
multistep state on chip) through the emulation harness, whose cooperative
launches run every workgroup's threads as fibers of one scheduler: against
the oracle, against the two-pass path, and in pieces."""
import numpy as np
import pytest

from oracle.periodic import PeriodicOracle
from workloads import periodic_problem_from_seed


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [
    dict(seed=40, M=32, T=0.05, N=14, order=8),
    dict(seed=41, M=64, T=0.04, N=11, order=8, dir2=True),      # field with an axis-1 component
    dict(seed=42, M=32, T=0.05, N=12, order=4, A_kind="stepwise"),
    dict(seed=43, M=32, T=0.03, N=9, order=6, A_kind="none"),
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
def test_persistent_steps_match_oracle_and_passes(emu, case):
    from emu.emu_plan import EmuPlan

    prob = _problem(case)
    plan = EmuPlan(emu, prob)
    assert plan.query(28) == 2.0
    plan.call("tdse_profile", 1)
    u = plan.run(prob.u0)
    assert plan.query(27) == 1.0        # one persistent launch for the Adams steps
    ref, _ = PeriodicOracle(prob).run()
    assert _rel(u, ref) < 1e-12
    plan.call("tdse_configure", 0, 0)
    assert plan.query(28) == 0.0
    two = plan.run(prob.u0)
    assert _rel(u, two) < 1e-13


def test_persistent_steps_in_pieces(emu):
    import ctypes as C

    from emu.emu_plan import EmuPlan

    prob = _problem(CASES[0])
    plan = EmuPlan(emu, prob)
    full = plan.run(prob.u0)
    plan.set_state(prob.u0)
    traj = PeriodicOracle(prob).run(keep=True)[1]["us"]
    done = 0
    for k in (2, 6, 1, 5):   # ends inside the start-up, at the Adams start, then persistent pieces
        plan.step(k)
        done += k
        out = np.zeros(prob.M, dtype=np.complex128)
        plan.call("tdse_get_state", C.c_void_p(out.ctypes.data), 1)
        assert _rel(out, traj[done]) < 1e-12, done
    assert np.array_equal(out, full)
