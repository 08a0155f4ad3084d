"""Write free_2d_256_oracle_sample.txt: sampled values of the free-space oracle on the
2D free-space workload (seed 2, 256 x 256 points on [-1,1)^2, FFT size 2048
per axis, eps = 1e-10, p = 8, q = 10, one Gauss panel per side, 1000 steps to
T = 1; Sections 3.3-3.4).

Two runs with the contour parameter H of the full 1000-step run: the first 8
steps (six Richardson start-up steps and two Adams steps) and all 1000 steps.
Every 8th grid point per axis is written, as "case i j Re(u) Im(u)", with the
grid 2-norm of each result.  Calls only oracle/ and workloads/.

    python tests/golden/make_free_2d_256_oracle.py      (about 20-40 min on 8 cores)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.freespace import FreeSpaceOracle  # noqa: E402
from workloads import free_2d_256_problem  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "free_2d_256_oracle_sample.txt")
STRIDE = 8


def main():
    full = free_2d_256_problem()
    H = FreeSpaceOracle(full).H
    lines = [f"# free-space oracle on the 2D free-space workload (seed 2, 256^2, nu 2048, eps 1e-10, p 8, q 10, 1 panel)",
             f"# H {H!r}", f"# stride {STRIDE}"]
    for steps in (8, 1000):
        prob = free_2d_256_problem()
        prob.nsteps = steps
        prob.T = full.dt * steps
        t = time.time()
        u, _ = FreeSpaceOracle(prob, H=H).run()
        print(f"{steps} steps: {time.time() - t:.1f} s", flush=True)
        lines.append(f"# case {steps} norm {float(np.linalg.norm(u))!r}")
        for i in range(0, u.shape[0], STRIDE):
            for j in range(0, u.shape[1], STRIDE):
                lines.append(f"{steps} {i} {j} {float(u[i, j].real)!r} {float(u[i, j].imag)!r}")
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(OUT)


if __name__ == "__main__":
    main()
