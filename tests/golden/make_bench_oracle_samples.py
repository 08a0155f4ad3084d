"""Write the stored oracle values of the benchmarked workloads: the FP64 oracle
run to the final time on exactly the inputs and plan parameters the benchmark
times, sampled on a regular sub-grid (Section 6's err(T) is then evaluated
on those points).  Calls only oracle/ and workloads/.

Cases (one file each, tests/golden/<case>_oracle_sample.txt):
  periodic_1d_256    1D periodic, M = 256, 100 steps to T = 1 (seed 0), every point
  periodic_2d_512    2D periodic, 512^2, 2000 steps to T = 2 (seed 1), every 8th point per axis
  periodic_2d_1024   2D periodic, 1024^2, 2000 steps to T = 2 (seed 3), every 16th point per axis
  free_2d_256_default_h
                     2D free space, 256^2, nu = 2048, eps = 1e-10, 1000 steps to T = 1 (seed 2),
                     the contour parameter of each axis from the Remark's rule (the plan's
                     default), every 8th point per axis
  moving_well_2d_512 the moving well (V0 = 300, beta = 0.2, c = (30, 15)) on 512^2, 2000 steps
                     to T = 2 pi / 15, every 8th point per axis
  batch_64           the 64 uneven periodic instances (seeds 4000 + i), 500 steps to T = 2,
                     stepwise field; 1D every (M/64)-th point, 2D every (M/16)-th point per axis
  periodic_3d_128    3D periodic, 128^3, 500 steps to T = 0.5 (seed 50), every 8th point per axis
  sampled_2d_512     2D periodic, 512^2 (seed 1), the potential replaced by the general sampled
                     V(x, t) of sampled_potential_problem, 500 steps to T = 0.5, every 8th point
  free_3d_32         3D free space, 32^3, nu = 256 per axis, eps = 1e-8, q = 8, 100 steps to
                     T = 0.1 (seed 62), the plan's default H per axis, every 4th point per axis
  example2_long_time_nr5
                     Section 6, Example 2's long-time wave packet: 1D free space, M = 128,
                     nu = 1024, q = 16, n_r = 5, 1000 steps to T = 1000, the C-type block
                     through the interpolant (automatic choice); every point

File format: "# key value" header lines (the case, the full-grid 2-norm of the
oracle's u(T) per instance, the sampling strides, free space: H per axis), then
one line per sample "inst i j Re(u) Im(u)" (1D: j = 0 and i the grid index;
3D: "inst i j k Re(u) Im(u)").

    python tests/golden/make_bench_oracle_samples.py CASE [CASE ...]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.freespace import FreeSpaceOracle  # noqa: E402
from oracle.periodic import PeriodicOracle  # noqa: E402
from workloads import (batch_64_problems, example2_long_time_problem, free_2d_256_problem,  # noqa: E402
                       free_3d_32_problem,
                       moving_well_problem, periodic_1d_256_problem, periodic_2d_512_problem,
                       periodic_2d_1024_problem, periodic_3d_128_problem, sampled_2d_512_problem)

HERE = os.path.dirname(os.path.abspath(__file__))


def _sample_lines(inst, u, stride):
    out = []
    if u.ndim == 1:
        for i in range(0, u.shape[0], stride):
            out.append(f"{inst} {i} 0 {float(u[i].real)!r} {float(u[i].imag)!r}")
    elif u.ndim == 3:
        for i in range(0, u.shape[0], stride):
            for j in range(0, u.shape[1], stride):
                for k in range(0, u.shape[2], stride):
                    v = u[i, j, k]
                    out.append(f"{inst} {i} {j} {k} {float(v.real)!r} {float(v.imag)!r}")
    else:
        for i in range(0, u.shape[0], stride):
            for j in range(0, u.shape[1], stride):
                out.append(f"{inst} {i} {j} {float(u[i, j].real)!r} {float(u[i, j].imag)!r}")
    return out


def cases():
    return {
        "periodic_1d_256": lambda: [("periodic", periodic_1d_256_problem(), 1, 1)],
        "periodic_2d_512": lambda: [("periodic", periodic_2d_512_problem(), 8, 8)],
        "periodic_2d_1024": lambda: [("periodic", periodic_2d_1024_problem(precision="fp64"), 16, 16)],
        "free_2d_256_default_h": lambda: [("free", free_2d_256_problem(), 8, 8)],
        "moving_well_2d_512": lambda: [("periodic", moving_well_problem(c=(30.0, 15.0), M=(512, 512), nsteps=2000),
                                        8, 8)],
        "batch_64": lambda: [("periodic", p, p.M[0] // 16, p.M[0] // 64)
                             for p in batch_64_problems(precision="fp64")],
        "example2_long_time_nr5": lambda: [("free", example2_long_time_problem(5), 1, 1)],
        "periodic_3d_128": lambda: [("periodic", periodic_3d_128_problem(), 8, 8)],
        "sampled_2d_512": lambda: [("periodic", sampled_2d_512_problem(), 8, 8)],
        "free_3d_32": lambda: [("free", free_3d_32_problem(), 4, 4)],
    }


def main(names):
    table = cases()
    for name in names:
        lines = [f"# case {name}"]
        body = []
        t0 = time.time()
        for inst, (kind, prob, s2, s1) in enumerate(table[name]()):
            stride = s2 if prob.dim == 2 else s1
            if kind == "free":
                orc = FreeSpaceOracle(prob)
                lines.append(f"# H {inst} " + " ".join(repr(float(h)) for h in orc.Hs))
            else:
                orc = PeriodicOracle(prob)
            u, _ = orc.run()
            lines.append(f"# norm {inst} {float(np.linalg.norm(u))!r}")
            lines.append(f"# stride {inst} {stride}")
            lines.append(f"# shape {inst} " + " ".join(str(m) for m in prob.M))
            body += _sample_lines(inst, u, stride)
            print(f"{name}[{inst}] {prob.M} {prob.nsteps} steps: {time.time() - t0:.1f} s", flush=True)
        path = os.path.join(HERE, f"{name}_oracle_sample.txt")
        with open(path, "w") as f:
            f.write("\n".join(lines + body) + "\n")
        print(path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(cases()))
