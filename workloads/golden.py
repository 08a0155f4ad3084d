"""Reader of the stored oracle samples under tests/golden/ (text files written
by tests/golden/make_bench_oracle_samples.py, which calls only the oracle),
and the sampled error of a computed u(T) against them.

The error is Section 6's err(T) (relative L2 on the grid, eq. (l2err))
restricted to the stored sub-grid, beside the largest pointwise deviation
relative to the largest stored |u|.  Parsing and norms only: nothing here
takes part in the scheme.
"""
from __future__ import annotations

import os
from typing import Dict

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden")


def load_samples(case: str) -> Dict[int, dict]:
    """{instance: {"idx": int [n, 2] (3D: [n, 3]), "val": complex [n], "norm": float,
    "stride": int, "shape": tuple, "H": list (free space)}} of one case file."""
    path = os.path.join(GOLDEN, f"{case}_oracle_sample.txt")
    inst: Dict[int, dict] = {}
    rows: Dict[int, list] = {}
    with open(path) as f:
        for line in f:
            parts = line.split()
            if not parts:
                continue
            if parts[0] == "#":
                key = parts[1]
                if key in ("norm", "stride", "shape", "H"):
                    d = inst.setdefault(int(parts[2]), {})
                    vals = parts[3:]
                    if key == "norm":
                        d["norm"] = float(vals[0])
                    elif key == "stride":
                        d["stride"] = int(vals[0])
                    elif key == "shape":
                        d["shape"] = tuple(int(v) for v in vals)
                    else:
                        d["H"] = [float(v) for v in vals]
                continue
            rows.setdefault(int(parts[0]), []).append(parts[1:])
    for i, r in rows.items():
        arr = np.array(r, dtype=object)
        nd = arr.shape[1] - 2   # 1D and 2D files carry two indices, 3D files three
        inst[i]["idx"] = arr[:, :nd].astype(np.int64)
        inst[i]["val"] = arr[:, nd].astype(np.float64) + 1j * arr[:, nd + 1].astype(np.float64)
    return inst


def sampled_error(u: np.ndarray, ref: dict) -> dict:
    """Relative L2 error and max-abs error (relative to max |u_ref|) of u on
    the stored points, and the relative deviation of the full-grid norm."""
    u = np.asarray(u)
    idx = ref["idx"]
    got = u[idx[:, 0]] if u.ndim == 1 else u[tuple(idx[:, a] for a in range(u.ndim))]
    want = ref["val"]
    return {"rel_l2": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
            "max_abs_rel": float(np.max(np.abs(got - want)) / np.max(np.abs(want))),
            "norm_rel": float(abs(np.linalg.norm(u) - ref["norm"]) / ref["norm"]),
            "points": int(len(want))}
