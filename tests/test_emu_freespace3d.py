"""CPU run of the 3D free-space path (the line transforms of Section 4.1 along
each axis: the column pass over axis 0, middle-axis passes around it, the row
pass over the last axis with the recurrence) through the emulation harness,
against the oracle."""
import numpy as np

from oracle.freespace import FreeSpaceOracle
from workloads import free_problem_from_seed


def test_emulated_3d_free_space_matches_oracle(emu):
    from emu.emu_plan import EmuPlan

    # uneven axes (8, 10, 8) so that a transposed axis cannot pass
    prob = free_problem_from_seed(61, 3, (8, 10, 8), 0.02, 2, order=2, nu=(256, 256, 256), eps=1e-8, q=4, panels=1)
    u = EmuPlan(emu, prob).run(prob.u0)
    ref, _ = FreeSpaceOracle(prob).run()
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < 1e-12
