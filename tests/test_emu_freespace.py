"""CPU run of the free-space HIP kernels and C ABI through the emulation
harness (tests/emu) against the free-space oracle: the contour transforms
(shifted FFTs of the equispaced rays and the dense Alpert/Gauss block), the
Richardson start-up on u and uhat, and the implicit Adams steps
(Sections 3.3-3.4, 4.1)."""
import copy

import numpy as np
import pytest

from oracle.freespace import FreeSpaceOracle
from workloads import free_problem_from_seed


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [
    dict(seed=5, dim=1, M=(32,), nu=(256,), T=0.05, N=12, q=8, panels=1),
    dict(seed=6, dim=1, M=(96,), nu=(512,), T=0.03, N=7, q=10, panels=3),     # ends right after start-up
    dict(seed=7, dim=1, M=(64,), nu=(256,), T=0.04, N=9, q=6, panels=2, order=4),
    dict(seed=8, dim=1, M=(40,), nu=(256,), T=0.02, N=3, q=5, panels=1, A_kind="none"),
    dict(seed=9, dim=2, M=(24, 32), nu=(256, 256), T=0.04, N=9, q=6, panels=2),
    dict(seed=10, dim=2, M=(40, 16), nu=(512, 256), T=0.04, N=8, q=4, panels=1),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c['M']}-{c['nu']}-{c['N']}" for c in CASES])
def test_emulated_free_space_matches_oracle(emu, case):
    from emu.emu_plan import EmuPlan

    prob = free_problem_from_seed(case["seed"], case["dim"], case["M"], case["T"], case["N"], nu=case["nu"],
                                  order=case.get("order", 8), eps=1e-11, q=case["q"], panels=case["panels"],
                                  A_kind=case.get("A_kind", "pulse_sin2"))
    u = EmuPlan(emu, prob).run(prob.u0)
    ref, _ = FreeSpaceOracle(prob).run()
    assert _rel(u, ref) < 1e-12


def test_emulated_free_space_given_H_and_partial_runs(emu):
    # a caller-supplied H overrides the rule; every prefix of the run matches
    from emu.emu_plan import EmuPlan

    prob = free_problem_from_seed(12, 1, (48,), 0.05, 10, nu=(256,), eps=1e-11, q=8, panels=2)
    for N in (1, 5, 6, 8):
        pr = copy.copy(prob)
        pr.nsteps, pr.T = N, prob.dt * N
        plan = EmuPlan(emu, pr, H=1.75)
        assert plan.query(80) == 1.75
        ref, _ = FreeSpaceOracle(pr, H=1.75).run()
        assert _rel(plan.run(pr.u0), ref) < 1e-12


FAR_CASES = [
    dict(seed=5, dim=1, M=(32,), nu=(256,), T=0.05, N=12, q=8, panels=1),
    dict(seed=6, dim=1, M=(96,), nu=(512,), T=0.03, N=7, q=10, panels=3),     # T reached in the start-up
    dict(seed=9, dim=2, M=(24, 32), nu=(256, 256), T=0.04, N=9, q=6, panels=2),
    dict(seed=10, dim=2, M=(40, 16), nu=(512, 256), T=0.04, N=8, q=4, panels=1),
]


@pytest.mark.parametrize("case", FAR_CASES, ids=[f"{c['M']}-{c['nu']}-{c['N']}" for c in FAR_CASES])
def test_emulated_far_evaluation_matches_oracle(emu, case):
    # tdse_far_eval at t = 0, after a start-up step and at T, on points inside
    # and outside [-1,1]^d (Remark on evaluation outside [-1,1]), against the
    # oracle's discrete representation of its own uhat
    from emu.emu_plan import EmuPlan

    prob = free_problem_from_seed(case["seed"], case["dim"], case["M"], case["T"], case["N"], nu=case["nu"],
                                  eps=1e-11, q=case["q"], panels=case["panels"])
    rng = np.random.default_rng(1)
    pts = [np.sort(rng.uniform(-2, 2, 37 + 4 * a)) for a in range(prob.dim)]
    for stop in (0, 2, case["N"]):
        plan = EmuPlan(emu, prob)
        plan.set_state(prob.u0)
        plan.step(stop)
        got = plan.far_eval(pts[-1], pts[0] if prob.dim == 2 else None)
        orc = FreeSpaceOracle(prob)
        _, info = orc.run(stop)
        ref = orc.evaluate(info["uhat"], pts)
        assert got.shape == ref.shape
        assert _rel(got, ref) < 1e-11, stop


def test_emulated_far_evaluation_without_allocation(emu):
    # tdse_far_eval_noalloc (workspace in the library's own array) equals
    # tdse_far_eval, twice in a row with a smaller second call
    import ctypes as C

    from emu.emu_plan import EmuPlan

    prob = free_problem_from_seed(9, 2, (24, 32), 0.04, 9, nu=(256, 256), eps=1e-11, q=6, panels=2)
    plan = EmuPlan(emu, prob)
    plan.set_state(prob.u0)
    plan.step(prob.nsteps)
    rng = np.random.default_rng(3)
    for nx, ny in ((21, 33), (5, 7)):
        px, py = np.sort(rng.uniform(-2, 2, nx)), np.sort(rng.uniform(-2, 2, ny))
        ref = plan.far_eval(py, px)
        out = np.zeros((nx, ny), dtype=np.complex128)
        plan.call("tdse_far_eval_noalloc", C.c_void_p(px.ctypes.data), nx, C.c_void_p(py.ctypes.data), ny,
                  C.c_void_p(out.ctypes.data))
        assert np.array_equal(out, ref)
    big = np.zeros(1 << 20)
    with pytest.raises(RuntimeError, match="library array"):
        plan.call("tdse_far_eval_noalloc", C.c_void_p(big.ctypes.data), 64, C.c_void_p(big.ctypes.data), 1 << 20,
                  C.c_void_p(big.ctypes.data))


def test_emulated_far_evaluation_errors(emu):
    from emu.emu_plan import EmuPlan
    from workloads import periodic_problem_from_seed

    prob = free_problem_from_seed(5, 1, (32,), 0.05, 12, nu=(256,), eps=1e-11, q=8, panels=1)
    plan = EmuPlan(emu, prob)
    ys = np.linspace(-1.5, 1.5, 7)
    with pytest.raises(RuntimeError, match="no state"):
        plan.far_eval(ys)
    plan.set_state(prob.u0)
    plan.step(prob.nsteps - 2)    # past the start-up, before T: no mode state kept
    with pytest.raises(RuntimeError, match="mode state"):
        plan.far_eval(ys)
    with pytest.raises(RuntimeError, match="nx = 1"):
        plan.far_eval(ys, xs=np.zeros(3))
    per = EmuPlan(emu, periodic_problem_from_seed(3, 1, (32,), 0.05, 10))
    per.set_state(np.ones(32, dtype=complex))
    with pytest.raises(RuntimeError, match="free-space"):
        per.far_eval(ys)


def test_emulated_cosine_pulse_ionization_setup(emu):
    # the Example 3 set-up (ground state of the Gaussian well, cosine pulse of
    # eq. (apulse)) on a short interval, against the oracle
    from emu.emu_plan import EmuPlan
    from workloads import ionization_1d_problem

    prob = ionization_1d_problem(100.0, nu=256, T=0.01, nsteps=12)
    u = EmuPlan(emu, prob).run(prob.u0)
    ref, _ = FreeSpaceOracle(prob).run()
    assert _rel(u, ref) < 1e-12


# C-type transforms through the Chebyshev interpolant (Section 4.1): the
# automatic choice, forced term counts, Gamma_2 blocks larger than the direct
# path's dense limit, and both axes of a 2D plan
CHEB_CASES = [
    dict(seed=30, dim=1, M=(64,), nu=(512,), T=0.04, N=10, q=16, panels=5, cheb=0),     # N_C = 160
    dict(seed=31, dim=1, M=(48,), nu=(256,), T=0.05, N=9, q=12, panels=2, cheb=-1),     # direct, same nodes
    dict(seed=31, dim=1, M=(48,), nu=(256,), T=0.05, N=9, q=12, panels=2, cheb=30),     # forced NT
    dict(seed=32, dim=2, M=(32, 24), nu=(256, 256), T=0.04, N=9, q=16, panels=3, cheb=0),
    dict(seed=33, dim=2, M=(16, 40), nu=(256, 512), T=0.03, N=8, q=8, panels=4, cheb=0, order=6),
]


@pytest.mark.parametrize("case", CHEB_CASES, ids=[f"{c['M']}-q{c['q']}x{c['panels']}-cheb{c['cheb']}" for c in CHEB_CASES])
def test_emulated_chebyshev_c_type_matches_oracle(emu, case):
    from emu.emu_plan import EmuPlan

    prob = free_problem_from_seed(case["seed"], case["dim"], case["M"], case["T"], case["N"], nu=case["nu"],
                                  order=case.get("order", 8), eps=1e-11, q=case["q"], panels=case["panels"])
    prob.cheb = case["cheb"]
    plan = EmuPlan(emu, prob)
    orc = FreeSpaceOracle(prob)
    for a in range(case["dim"]):
        assert plan.query(134 + a) == orc.NT[a], (a, plan.query(134 + a), orc.NT)
    if case["cheb"] != -1:
        assert all(orc.NT)
    u = plan.run(prob.u0)
    ref, _ = orc.run()
    assert _rel(u, ref) < 1e-12


def test_emulated_example2_long_time(emu):
    # Section 6, Example 2's long-time run (T = 1000, q = 16, n_r = 5) through
    # the interpolant: the oracle's u(T) and the exact wave packet
    from emu.emu_plan import EmuPlan
    from workloads import example2_long_time_problem
    from workloads import wavepacket as _wavepacket

    prob = example2_long_time_problem(5, cheb=0, nsteps=40)
    orc = FreeSpaceOracle(prob)
    plan = EmuPlan(emu, prob)
    assert plan.query(134) == orc.NT[0] > 0
    u = plan.run(prob.u0)
    ref, _ = orc.run()
    assert _rel(u, ref) < 1e-12
    ex = _wavepacket(orc.xs[0] + orc.phi(prob.T)[0], prob.T, 0.1)
    assert _rel(u, ex) < 1e-13


def test_plan_rejects_bad_chebyshev_settings(emu):
    from emu.emu_plan import EmuPlan

    prob = free_problem_from_seed(34, 1, (32,), 0.05, 4, nu=(256,), eps=1e-11, q=8, panels=1)
    for bad in (-2, 1, 65):
        prob.cheb = bad
        with pytest.raises(Exception):
            EmuPlan(emu, prob)
    # more direct-sum rows than half the FFT line: refused, accepted through the interpolant
    prob = free_problem_from_seed(34, 1, (32,), 0.05, 4, nu=(256,), eps=1e-11, q=32, panels=4)
    prob.cheb = -1
    with pytest.raises(Exception):
        EmuPlan(emu, prob)
    prob.cheb = 0
    EmuPlan(emu, prob)
