"""Benchmark: mode-updates/s of the 2D periodic FP64 marcher on one MI355X.

Workload: 2D periodic TDSE, 512 x 512 grid, T = 2, 2000 steps of the 8th-order
implicit Adams scheme (6 Richardson start-up steps), four-well potential with
sinusoidal modulation and a sin^2 pulse, seed 1, complex128 (synthetic inputs).
One benchmark "step" is one whole run [0, T] on inputs already resident in
device memory: start-up plus 1994 Adams steps (the library's default path:
the start-up replayed from a captured graph, the Adams steps in one
persistent launch; the two-pass path is timed beside it).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--workload periodic-2d-512|periodic-2d-1024-fp64]

Prints one JSON line.  value = modes x time steps / wall time of the K timed
runs (whole job).  roofline: algorithmic bytes of the dominant kernel (the
persistent Adams launch: 216 B per mode and step times the steps it takes)
per launch / its mean duration measured with HIP events on the library's
stream in eager runs of the same workload.  Every leg reports its error
against the stored oracle samples.  cpu_baseline: the FP64 oracle on the host
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFS = 78.6     # MI355X dense FP64 matrix-core peak


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=100, help="Adams steps in the oracle sample (after the start-up)")
    ap.add_argument("--workload", default="periodic-2d-512", choices=["periodic-2d-512", "periodic-2d-1024-fp64"])
    ap.add_argument("--prof-runs", type=int, default=3, help="eager runs timed per kernel with HIP events")
    ap.add_argument("--no-split", action="store_true", help="skip the FP32-split 1024x1024 leg")
    ap.add_argument("--split-steps", type=int, default=3)
    ap.add_argument("--no-free", action="store_true", help="skip the free-space 256x256 leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance batched leg")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="batched leg without its adjoint (which launches from several host threads)")
    ap.add_argument("--no-well", action="store_true", help="skip the moving-well (potential on the fly) leg")
    ap.add_argument("--no-ionization", action="store_true", help="skip the 1D ionization (Example 3) leg")
    ap.add_argument("--no-1d", action="store_true", help="skip the 1D periodic M = 256 leg")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D periodic 128^3 leg")
    ap.add_argument("--no-sampled", action="store_true", help="skip the sampled-potential 512^2 leg")
    ap.add_argument("--no-free-3d", action="store_true", help="skip the 3D free-space 32^3 leg")
    ap.add_argument("--runs-3d", type=int, default=3)
    ap.add_argument("--no-long-time", action="store_true",
                    help="skip the long-time free-space leg (Chebyshev-interpolated C-type block)")
    ap.add_argument("--batch-runs", type=int, default=3)
    ap.add_argument("--free-runs", type=int, default=2)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run device copies of 256 MiB (to scale HBM byte counters) and exit")
    return ap.parse_args()


def calibrate_copy():
    import torch

    n = 256 * 1024 * 1024 // 16
    a = torch.ones(n, dtype=torch.complex128, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": a.numel() * 16, "copy_bytes_written": b.numel() * 16, "copies": 5}))


def device_copy_gbps(dev, mib: int = 512, reps: int = 10) -> float:
    """Bandwidth of a plain device-to-device copy (bytes read + written per
    second), timed with events on the current stream.  At 512 MiB the copy
    streams from HBM: the practical HBM ceiling.  At 32 MiB source and
    destination together (64 MiB) stay in the 256 MB last-level cache (MALL)
    between repetitions: the ceiling of a working set that fits there, as the
    512 x 512 and 1024 x 1024 periodic runs do."""
    import torch

    n = mib * (1 << 20) // 16
    a = torch.ones(n, dtype=torch.complex128, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * n * 16 / (ms * 1e-3) / 1e9


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, adams_steps: int) -> dict:
    """Time the FP64 oracle (as written) on the host: the Richardson start-up
    alone, then start-up plus `adams_steps` implicit Adams steps, one thread
    (numpy's FFT is single-threaded).  End to end = modes x steps / time of
    the second run; steady state = modes x adams_steps / (difference of the
    two).  Beside it, for context only, the same oracle with its transforms
    taken by scipy.fft on all available cores."""
    from threadpoolctl import threadpool_limits

    from oracle.periodic import PeriodicOracle

    ns = prob.start_steps
    modes = float(prob.u0.size)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        PeriodicOracle(prob).run(nsteps=ns)
        t_start = time.perf_counter() - t0
        t0 = time.perf_counter()
        PeriodicOracle(prob).run(nsteps=ns + adams_steps)
        t_full = time.perf_counter() - t0
    out = {
        "value": modes * (ns + adams_steps) / t_full,
        "unit": "mode-updates/s",
        "cores": 1,
        "kind": "oracle",
        "steady_state_value": modes * adams_steps / max(t_full - t_start, 1e-9),
        "cpu_model": cpu_model(),
        "host_cores_available": len(os.sched_getaffinity(0)),
        "sample": f"{prob.name} at full size ({'x'.join(map(str, prob.M))}): the {ns} Richardson start-up steps "
                  f"({t_start:.1f} s), then start-up + {adams_steps} Adams steps ({t_full:.1f} s) of {prob.nsteps}, "
                  f"numpy/pocketfft single thread",
    }
    try:
        import scipy.fft as sfft

        cores = len(os.sched_getaffinity(0))

        class AllCores(PeriodicOracle):
            def F(self, f):
                return sfft.fftn(f, workers=cores) / f.size

            def Finv(self, g):
                return sfft.ifftn(g, workers=cores) * g.size

        t0 = time.perf_counter()
        AllCores(prob).run(nsteps=ns + adams_steps)
        t_all = time.perf_counter() - t0
        out["all_cores_scipy_fft"] = {"value": modes * (ns + adams_steps) / t_all, "cores": cores,
                                      "note": "the oracle with scipy.fft transforms on all cores (context)"}
    except ImportError:
        pass
    return out


def oracle_error(case: str, u, inst: int = 0, bar: float = 1e-11) -> dict:
    """Error of a computed u(T) against the stored oracle samples of the same
    workload (tests/golden/<case>_oracle_sample.txt): Section 6's err(T) on
    the stored sub-grid."""
    from workloads.golden import load_samples, sampled_error

    e = sampled_error(u.detach().cpu().numpy() if hasattr(u, "detach") else u, load_samples(case)[inst])
    return {"rel_l2_vs_oracle": e["rel_l2"], "max_abs_rel_vs_oracle": e["max_abs_rel"],
            "sampled_points": e["points"], "bar": bar, "pass": e["rel_l2"] <= bar}


def end_to_end(bytes_per_step: float, nsteps: int, seconds: float, copies: dict) -> dict:
    """Algorithmic bytes of every nominal time step over the whole-run wall
    time, against the datasheet HBM peak and the measured copy ceilings."""
    gbps = bytes_per_step * nsteps / seconds / 1e9
    out = {"algorithmic_bytes_per_step": bytes_per_step, "GBps": gbps, "frac_of_peak": gbps / HBM_PEAK_GBS}
    for k, v in copies.items():
        out[f"frac_of_copy_{k}"] = gbps / v
    return out


KERNEL_SOURCES = ("paper_2001_06113_amd/csrc/periodic_kernels.hip", "paper_2001_06113_amd/csrc/periodic_body.h",
                  "paper_2001_06113_amd/csrc/fft_lds.h")


P2_KERNEL_SOURCES = ("paper_2001_06113_amd/csrc/persist2d_kernels.hip", "paper_2001_06113_amd/csrc/fft_lds.h")


FS_KERNEL_SOURCES = ("paper_2001_06113_amd/csrc/freespace_kernels.hip", "paper_2001_06113_amd/csrc/fft_lds.h")


def measured_traffic(name: str, sources=KERNEL_SOURCES):
    """HBM bytes per launch of a kernel from the committed FETCH_SIZE/WRITE_SIZE
    summary, or None if the kernel sources changed since those counters were
    taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = dict(l.split(": ", 1) for l in open(path).read().splitlines() if ": " in l and not l.startswith("#"))
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if kv.get("source_sha256", "").strip() != h.hexdigest():
        return None
    return float(kv["traffic_bytes"])


def split_leg(steps: int, copies: dict) -> dict:
    """FP32-split form on the 1024 x 1024 workload (seed 3): throughput of
    graph-replayed runs, rel-L2 of u(T) against the FP64 GPU path, and both
    runs against the stored oracle samples."""
    import torch

    from paper_2001_06113_amd.tdse import Q_BYTES_PER_STEP, Q_RESIDUAL, Plan
    from workloads import periodic_2d_1024_problem

    dev = torch.device("cuda:0")
    res, outs, walls, e2e, err = {}, {}, {}, {}, {}
    for prec in ("fp32split", "fp64"):
        prob = periodic_2d_1024_problem(precision=prec)
        plan = Plan.from_problem(prob, device=dev)
        plan.use_graph(True)
        u0 = torch.as_tensor(prob.u0).to(dev)
        out = torch.empty_like(u0)
        plan.run(u0, out)
        torch.cuda.synchronize()
        n = steps
        t0 = time.perf_counter()
        for _ in range(n):
            plan.run(u0, out)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / n
        outs[prec] = out.clone()
        walls[prec] = wall
        res[prec] = u0.numel() * prob.nsteps / wall
        e2e[prec] = end_to_end(plan.query(Q_BYTES_PER_STEP), prob.nsteps, wall, copies)
        err[prec] = oracle_error("periodic_2d_1024", out, bar=1e-6 if prec == "fp32split" else 1e-11)
        # the history residual of the last Adams step before T (FP64 recomputation)
        plan.use_graph(False)
        plan.set_state(u0)
        plan.step(prob.nsteps - 1)
        err[prec]["history_residual_step_N-1"] = plan.query(Q_RESIDUAL)
        plan.close()
    rel = (torch.linalg.vector_norm(outs["fp32split"] - outs["fp64"]) / torch.linalg.vector_norm(outs["fp64"])).item()
    return {"workload": "2D periodic TDSE 1024x1024, T=2, 2000 steps AM8, FP32-split",
            "value": res["fp32split"], "unit": "mode-updates/s", "ms_per_run": walls["fp32split"] * 1e3,
            "end_to_end": e2e["fp32split"], "error": err["fp32split"],
            "fp64_value": res["fp64"], "fp64_ms_per_run": walls["fp64"] * 1e3, "fp64_end_to_end": e2e["fp64"],
            "fp64_error": err["fp64"],
            "speedup_vs_fp64": res["fp32split"] / res["fp64"], "rel_l2_vs_fp64": rel, "bar": 1e-6}


def moving_well_leg(runs: int = 5) -> dict:
    """Potential evaluated on the fly: Example 1 of Section 6 at its own size
    (1D, M = 256, moving Gaussian well V0 = 300, beta = 0.2, c = 30, T = 2 pi/15,
    400 steps), and the same well moving at (30, 15) on the 512 x 512 grid
    with 2000 steps, where the column pass computes V instead of reading it."""
    import torch

    from paper_2001_06113_amd.tdse import Q_PROF_MS_COL, Q_PROF_N_COL, Plan
    from workloads import moving_well_problem

    dev = torch.device("cuda:0")
    out = {}
    for key, prob in (("example1_1d", moving_well_problem(c=(30.0,), M=(256,), nsteps=400)),
                      ("grid_512x512", moving_well_problem(c=(30.0, 15.0), M=(512, 512), nsteps=2000))):
        plan = Plan.from_problem(prob, device=dev)
        u0 = torch.as_tensor(prob.u0).to(dev)
        res = torch.empty_like(u0)
        plan.use_graph(True)
        plan.run(u0, res)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(runs):
            plan.run(u0, res)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / runs
        plan.use_graph(False)
        plan.profile(True)
        plan.run(u0, res)
        col_us = plan.query(Q_PROF_MS_COL) * 1e3 / max(plan.query(Q_PROF_N_COL), 1)
        run1d_us = plan.query(24) * 1e3 / max(plan.query(25), 1)
        plan.profile(False)
        plan.close()
        out[key] = {"ms_per_run": wall * 1e3, "value": u0.numel() * prob.nsteps / wall, "unit": "mode-updates/s",
                    "us_per_time_step": wall * 1e6 / prob.nsteps,
                    "finite": bool(torch.isfinite(torch.view_as_real(res)).all().item())}
        if prob.dim == 1:
            out[key]["one_workgroup_run_kernel_us"] = run1d_us
        else:
            out[key]["col_pass_us"] = col_us
        if key == "grid_512x512":
            out[key]["error"] = oracle_error("moving_well_2d_512", res)
    return {"workload": "moving periodic Gaussian well (V0=300, beta=0.2), potential on the fly: "
                        "1D M=256 c=30 400 steps; 2D 512x512 c=(30,15) 2000 steps, FP64", **out}


def free_space_leg(runs: int, copies: dict) -> dict:
    """Free-space FP64 form on the 256 x 256 workload (seed 2, nu = 2048 per
    axis, eps = 1e-10, 1000 steps): graph-replayed whole runs, and the
    per-pass durations of one eager run from dispatch-recorded HIP events."""
    import torch

    from paper_2001_06113_amd.tdse import (Q_BYTES_COL, Q_BYTES_ROW, Q_PROF_MS_COL, Q_PROF_MS_ROW,
                                           Q_PROF_N_COL, Q_PROF_N_ROW, Plan)
    from workloads import free_2d_256_problem

    dev = torch.device("cuda:0")
    prob = free_2d_256_problem()
    plan = Plan.from_problem(prob, device=dev)
    u0 = torch.as_tensor(prob.u0).to(dev)
    out = torch.empty_like(u0)
    plan.use_graph(True)
    plan.run(u0, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(runs):
        plan.run(u0, out)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / runs
    err = oracle_error("free_2d_256_default_h", out)
    plan.use_graph(False)
    plan.profile(True)
    plan.run(u0, out)
    row_us = plan.query(Q_PROF_MS_ROW) * 1e3 / max(plan.query(Q_PROF_N_ROW), 1)
    col_us = plan.query(Q_PROF_MS_COL) * 1e3 / max(plan.query(Q_PROF_N_COL), 1)
    plan.profile(False)
    n_modes = plan.query(81) * plan.query(82)
    row_b, col_b = plan.query(Q_BYTES_ROW), plan.query(Q_BYTES_COL)
    plan_H = [plan.query(86), plan.query(87)]
    ach = row_b / (row_us * 1e-6) / 1e9
    far = far_field_eval(plan, dev)
    plan.close()
    return {"workload": "2D free-space TDSE 256x256, nu=2048 per axis, eps=1e-10, p=8, q=10, 1 panel, "
                        "T=1, 1000 steps AM8",
            "value": n_modes * prob.nsteps / wall, "unit": "mode-updates/s",
            "modes": int(n_modes), "grid_points": int(u0.numel()),
            "grid_point_updates_per_s": u0.numel() * prob.nsteps / wall, "ms_per_run": wall * 1e3,
            "contour_H": [plan_H[0], plan_H[1]], "error": err,
            "end_to_end": end_to_end(row_b + col_b, prob.nsteps, wall, copies),
            "roofline": {"bound": "hbm", "kernel": "free-space Adams row pass (k_fs_row)", "achieved": ach,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                         "traffic": measured_traffic("k_fs_row_2048_traffic.txt", FS_KERNEL_SOURCES),
                         "bytes_per_launch": row_b, "mean_launch_us": row_us, "row_pass_us": row_us,
                         "col_pass_us": col_us, "col_bytes_per_launch": col_b},
            "far_field": far}


def far_field_eval(plan, dev, n: int = 512, box: float = 2.0, reps: int = 5) -> dict:
    """u(T) of a free-space plan on an n x n grid of [-box, box]^2 from its
    complex-frequency representation (tdse_far_eval): wall time per call, and
    the first product (the contraction over the last axis, 8 N1 N2 n flops)
    timed by dispatch-recorded HIP events against the FP64 matrix-core peak."""
    import torch

    from paper_2001_06113_amd.tdse import Q_PROF_MS_FAR, Q_PROF_N_FAR

    pts = torch.linspace(-box, box, n, dtype=torch.float64, device=dev)
    out = plan.far_eval(pts, pts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = plan.far_eval(pts, pts)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    plan.profile(True)
    for _ in range(reps):
        plan.far_eval(pts, pts)
    g_us = plan.query(Q_PROF_MS_FAR) * 1e3 / max(plan.query(Q_PROF_N_FAR), 1)
    plan.profile(False)
    N1, N2 = plan.query(81), plan.query(82)
    flops = 8.0 * N1 * N2 * n
    ach = flops / (g_us * 1e-6) / 1e12
    return {"points": [n, n], "box": [-box, box], "ms_per_eval": wall * 1e3,
            "finite": bool(torch.isfinite(torch.view_as_real(out)).all().item()),
            "roofline": {"bound": "mfma", "kernel": "far-field product over the last axis (k_far_gemm, FP64 MFMA)",
                         "achieved": ach, "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s",
                         "frac": ach / FP64_MFMA_PEAK_TFS, "flops_per_launch": flops, "mean_launch_us": g_us}}


def ionization_leg(runs: int = 3, nsteps: int = 4000) -> dict:
    """Section 6, Example 3: 1D ionization from the ground state of a Gaussian
    well (V0 = 1400, beta = 0.1) by the cosine pulse A0 = 100, omega = 50, 100,
    200, free space, M = 100, nu = 1024 (h = 0.31), eps = 1e-10, q = 10,
    T = 0.5: graph-replayed whole runs, time steps per second, and the
    ionization fractions 1 - int_{-1}^{1} |u(T)|^2."""
    import torch

    from paper_2001_06113_amd.tdse import Plan
    from workloads import ionization_1d_problem

    dev = torch.device("cuda:0")
    out = {"workload": f"Example 3 ionization, 1D free space M=100, nu=1024, eps=1e-10, q=10, T=0.5, {nsteps} steps AM8",
           "cases": []}
    for om in (50.0, 100.0, 200.0):
        prob = ionization_1d_problem(om, nsteps=nsteps)
        plan = Plan.from_problem(prob, device=dev)
        u0 = torch.as_tensor(prob.u0).to(dev)
        u = torch.empty_like(u0)
        plan.use_graph(True)
        plan.run(u0, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(runs):
            plan.run(u0, u)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / runs
        ion = 100.0 * (1.0 - float(torch.sum(torch.abs(u) ** 2)) * 2.0 / prob.M[0])
        plan.close()
        out["cases"].append({"omega": om, "ionization_percent": ion, "ms_per_run": wall * 1e3,
                             "time_steps_per_s": nsteps / wall})
    # Example 4 (2D, field along x), omega = 100, the paper's two accuracy settings
    from workloads import ionization_2d_problem

    out["cases_2d"] = []
    for label, nu, eps, n2 in (("eps=1e-10, h1=0.31, h2=0.61", (1024, 512), 1e-10, 8000),
                               ("eps=1e-5, h=1.23 both axes", (256, 256), 1e-5, 4000)):
        prob = ionization_2d_problem(100.0, nu=nu, eps=eps, nsteps=n2)
        plan = Plan.from_problem(prob, device=dev)
        u0 = torch.as_tensor(prob.u0).to(dev)
        u = torch.empty_like(u0)
        plan.use_graph(True)
        plan.run(u0, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(runs):
            plan.run(u0, u)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / runs
        ion = 100.0 * (1.0 - float(torch.sum(torch.abs(u) ** 2)) * (2.0 / prob.M[0]) ** 2)
        modes = plan.query(81) * plan.query(82)
        plan.close()
        out["cases_2d"].append({"setting": label, "omega": 100.0, "nu": list(nu), "time_steps": n2,
                                "modes": int(modes), "ionization_percent": ion, "ms_per_run": wall * 1e3,
                                "time_steps_per_s": n2 / wall})
    return out


def periodic_1d_leg(runs: int = 20) -> dict:
    """The 1D periodic workload (M = 256, seed 0, T = 1, 100 steps, FP64):
    graph-replayed whole runs and the error against the stored oracle values
    (every grid point)."""
    import torch

    from paper_2001_06113_amd.tdse import Plan
    from workloads import periodic_1d_256_problem

    dev = torch.device("cuda:0")
    prob = periodic_1d_256_problem()
    plan = Plan.from_problem(prob, device=dev)
    u0 = torch.as_tensor(prob.u0).to(dev)
    out = torch.empty_like(u0)
    plan.use_graph(True)
    plan.run(u0, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(runs):
        plan.run(u0, out)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / runs
    err = oracle_error("periodic_1d_256", out)
    plan.use_graph(False)
    plan.profile(True)
    plan.run(u0, out)
    k_us = plan.query(24) * 1e3 / max(plan.query(25), 1)
    plan.profile(False)
    plan.close()
    return {"workload": "1D periodic TDSE M=256, V=-a cos x, T=1, 100 steps AM8 (6 Richardson start-up steps), FP64",
            "value": u0.numel() * prob.nsteps / wall, "unit": "mode-updates/s", "ms_per_run": wall * 1e3,
            "us_per_time_step": wall * 1e6 / prob.nsteps, "one_workgroup_run_kernel_us": k_us, "error": err}


def periodic_3d_leg(runs: int, copies: dict) -> dict:
    """3D periodic on the 128^3 workload (seed 50, 500 steps to T = 0.5), in
    FP64 and in the FP32-split form: graph-replayed whole runs, the error
    against the stored oracle values, and the per-pass durations of one eager
    run (dispatch-recorded HIP events): row pass (last axis, recurrence),
    column pass (axis 0, solve) and the two middle-axis FFT passes."""
    out = _periodic_3d_run(runs, copies, "fp64")
    out["split"] = _periodic_3d_run(runs, copies, "fp32split")
    return out


def _periodic_3d_run(runs: int, copies: dict, precision: str) -> dict:
    import torch

    from paper_2001_06113_amd.tdse import (Q_BYTES_COL, Q_BYTES_MID, Q_BYTES_PER_STEP, Q_BYTES_ROW, Q_PROF_MS_COL,
                                           Q_PROF_MS_MID, Q_PROF_MS_ROW, Q_PROF_N_COL, Q_PROF_N_MID, Q_PROF_N_ROW,
                                           Plan)
    from workloads import periodic_3d_128_problem

    dev = torch.device("cuda:0")
    prob = periodic_3d_128_problem()
    prob.precision = precision
    plan = Plan.from_problem(prob, device=dev)
    u0 = torch.as_tensor(prob.u0).to(dev)
    out = torch.empty_like(u0)
    plan.use_graph(True)
    plan.run(u0, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(runs):
        plan.run(u0, out)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / runs
    err = oracle_error("periodic_3d_128", out, bar=1e-11 if precision == "fp64" else 1e-6)
    plan.use_graph(False)
    plan.profile(True)
    plan.run(u0, out)
    row = plan.query(Q_PROF_MS_ROW) * 1e3 / max(plan.query(Q_PROF_N_ROW), 1)
    col = plan.query(Q_PROF_MS_COL) * 1e3 / max(plan.query(Q_PROF_N_COL), 1)
    mid = plan.query(Q_PROF_MS_MID) * 1e3 / max(plan.query(Q_PROF_N_MID), 1)
    plan.profile(False)
    row_b, col_b, mid_b = plan.query(Q_BYTES_ROW), plan.query(Q_BYTES_COL), plan.query(Q_BYTES_MID)
    step_b = plan.query(Q_BYTES_PER_STEP)
    plan.close()
    modes = u0.numel()

    def rf(b, us):
        a = b / (us * 1e-6) / 1e9
        return {"us": us, "bytes_per_launch": b, "GBps": a, "frac": a / HBM_PEAK_GBS}

    form = "FP64" if precision == "fp64" else "FP32 transforms, FP64 state"
    return {"workload": f"3D periodic TDSE 128^3, T=0.5, 500 steps AM8, {form}",
            "value": modes * prob.nsteps / wall, "unit": "mode-updates/s", "ms_per_run": wall * 1e3,
            "us_per_time_step": wall * 1e6 / prob.nsteps, "error": err,
            "end_to_end": end_to_end(step_b, prob.nsteps, wall, copies),
            "row_pass": rf(row_b, row), "col_pass": rf(col_b, col), "mid_pass": rf(mid_b, mid),
            "adams_step_us_eager": row + col + 2 * mid}


def free_space_3d_leg(runs: int, copies: dict) -> dict:
    """3D free space on the 32^3 workload (seed 62, nu = 256 per axis, eps =
    1e-8, q = 8, 100 order-8 steps to T = 0.1, the plan's default H per axis):
    graph-replayed whole runs, the error against the stored oracle values,
    and the per-pass durations of one eager run: row pass (last axis,
    recurrence), column pass (axis 0, solve) and the middle-axis transforms."""
    import torch

    from paper_2001_06113_amd.tdse import (Q_BYTES_COL, Q_BYTES_MID, Q_BYTES_PER_STEP, Q_BYTES_ROW, Q_FS_AXIS2,
                                           Q_FS_MODES, Q_PROF_MS_COL, Q_PROF_MS_MID, Q_PROF_MS_ROW, Q_PROF_N_COL,
                                           Q_PROF_N_MID, Q_PROF_N_ROW, Plan)
    from workloads import free_3d_32_problem

    dev = torch.device("cuda:0")
    prob = free_3d_32_problem()
    plan = Plan.from_problem(prob, device=dev)
    modes = 1
    for a in range(3):
        modes *= int(plan.query(Q_FS_MODES + a if a < 2 else Q_FS_AXIS2))
    u0 = torch.as_tensor(prob.u0).to(dev)
    out = torch.empty_like(u0)
    plan.use_graph(True)
    plan.run(u0, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(runs):
        plan.run(u0, out)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / runs
    err = oracle_error("free_3d_32", out)
    plan.use_graph(False)
    plan.profile(True)
    plan.run(u0, out)
    row = plan.query(Q_PROF_MS_ROW) * 1e3 / max(plan.query(Q_PROF_N_ROW), 1)
    col = plan.query(Q_PROF_MS_COL) * 1e3 / max(plan.query(Q_PROF_N_COL), 1)
    mid = plan.query(Q_PROF_MS_MID) * 1e3 / max(plan.query(Q_PROF_N_MID), 1)
    plan.profile(False)
    row_b, col_b, mid_b = plan.query(Q_BYTES_ROW), plan.query(Q_BYTES_COL), plan.query(Q_BYTES_MID)
    step_b = plan.query(Q_BYTES_PER_STEP)
    plan.close()

    def rf(b, us):
        a = b / (us * 1e-6) / 1e9
        return {"us": us, "bytes_per_launch": b, "GBps": a, "frac": a / HBM_PEAK_GBS}

    return {"workload": "3D free-space TDSE 32^3, nu=256 per axis, eps=1e-8, q=8, T=0.1, 100 steps AM8, FP64",
            "value": modes * prob.nsteps / wall, "unit": "mode-updates/s", "modes": modes,
            "grid_point_updates_per_s": u0.numel() * prob.nsteps / wall, "ms_per_run": wall * 1e3,
            "us_per_time_step": wall * 1e6 / prob.nsteps, "error": err,
            "end_to_end": end_to_end(step_b, prob.nsteps, wall, copies),
            "row_pass": rf(row_b, row), "col_pass": rf(col_b, col), "mid_pass": rf(mid_b, mid),
            "adams_step_us_eager": row + col + 2 * mid}


def sampled_leg(runs: int, copies: dict) -> dict:
    """A general non-separable potential given as samples at the step times
    (TDSE_V_SAMPLED) on the 512^2 grid (seed 1, 500 steps, dt = 1e-3):
    graph-replayed whole runs (two passes per step: the persistent launch
    takes stored fields only), the error against the stored oracle values,
    and the per-pass durations of one eager run."""
    import torch

    from paper_2001_06113_amd.tdse import (Q_BYTES_COL, Q_BYTES_PER_STEP, Q_BYTES_ROW, Q_PROF_MS_COL, Q_PROF_MS_ROW,
                                           Q_PROF_N_COL, Q_PROF_N_ROW, Plan)
    from workloads import sampled_2d_512_problem

    dev = torch.device("cuda:0")
    prob = sampled_2d_512_problem()
    plan = Plan.from_problem(prob, device=dev)
    u0 = torch.as_tensor(prob.u0).to(dev)
    out = torch.empty_like(u0)
    plan.use_graph(True)
    plan.run(u0, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(runs):
        plan.run(u0, out)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / runs
    err = oracle_error("sampled_2d_512", out)
    plan.use_graph(False)
    plan.profile(True)
    plan.run(u0, out)
    row = plan.query(Q_PROF_MS_ROW) * 1e3 / max(plan.query(Q_PROF_N_ROW), 1)
    col = plan.query(Q_PROF_MS_COL) * 1e3 / max(plan.query(Q_PROF_N_COL), 1)
    plan.profile(False)
    step_b, row_b, col_b = plan.query(Q_BYTES_PER_STEP), plan.query(Q_BYTES_ROW), plan.query(Q_BYTES_COL)
    plan.close()
    samples_gb = prob.V_samples.nbytes / 1e9
    return {"workload": "2D periodic 512x512, general non-separable V(x,t) given by 501 samples in time "
                        "(4 Gaussian wells modulated + a breathing well circling the origin), 500 steps, FP64",
            "value": u0.numel() * prob.nsteps / wall, "unit": "mode-updates/s", "ms_per_run": wall * 1e3,
            "us_per_time_step": wall * 1e6 / prob.nsteps, "samples_GB_in_HBM": samples_gb, "error": err,
            "end_to_end": end_to_end(step_b, prob.nsteps, wall, copies),
            "row_pass_us": row, "col_pass_us": col, "row_bytes_per_launch": row_b, "col_bytes_per_launch": col_b}


def long_time_leg(runs: int = 5) -> dict:
    """The C-type block on Gamma_2 through the Chebyshev interpolant against
    direct sums (Section 4.1): Section 6, Example 2's long-time wave packet
    (1D, M = 128, nu = 1024, q = 16, n_r = 5, 1000 steps to T = 1000; error
    against the stored oracle values and the exact packet), and the 256^2,
    nu = 2048 free-space grid with q = 16, n_r = 5 (N_C = 160 per axis, 200
    steps of dt = 1e-3): time per step and per row and column pass."""
    import numpy as np
    import torch

    from paper_2001_06113_amd.tdse import (Q_FS_CHEB, Q_PHI, Q_PROF_MS_COL, Q_PROF_MS_ROW, Q_PROF_N_COL,
                                           Q_PROF_N_ROW, Plan)
    from workloads import example2_long_time_problem, free_grid, free_problem_from_seed, wavepacket

    dev = torch.device("cuda:0")

    def timed(prob, reps):
        plan = Plan.from_problem(prob, device=dev)
        u0 = torch.as_tensor(prob.u0).to(dev)
        out = torch.empty_like(u0)
        plan.use_graph(True)
        plan.run(u0, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.run(u0, out)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        plan.use_graph(False)
        plan.profile(True)
        plan.run(u0, out)
        row = plan.query(Q_PROF_MS_ROW) * 1e3 / max(plan.query(Q_PROF_N_ROW), 1)
        col = plan.query(Q_PROF_MS_COL) * 1e3 / max(plan.query(Q_PROF_N_COL), 1)
        plan.profile(False)
        nt = [int(plan.query(Q_FS_CHEB + a)) for a in range(prob.dim)]
        phi = [plan.query(Q_PHI + a) for a in range(prob.dim)]
        plan.close()
        return out.cpu().numpy(), wall, row, col, nt, phi

    res = {"workload": "C-type block through the Chebyshev interpolant vs direct sums: Example 2 long-time "
                       "wave packet (1D M=128, nu=1024, q=16, n_r=5, T=1000, 1000 steps) and 2D 256x256, "
                       "nu=2048, q=16, n_r=5 (200 steps)"}
    for cheb, key in ((0, "example2_interpolant"), (-1, "example2_direct")):
        prob = example2_long_time_problem(5, cheb=cheb)
        u, wall, row, col, nt, phi = timed(prob, runs)
        ex = wavepacket(free_grid(prob.M[0]) + phi[0], prob.T, 0.1)
        res[key] = {"NT": nt[0], "ms_per_run": wall * 1e3, "us_per_time_step": wall * 1e6 / prob.nsteps,
                    "row_pass_us": row, "error": oracle_error("example2_long_time_nr5", u),
                    "rel_l2_vs_exact": float(np.linalg.norm(u - ex) / np.linalg.norm(ex))}
    grid = {}
    for cheb, key in ((0, "interpolant"), (-1, "direct")):
        prob = free_problem_from_seed(2, 2, (256, 256), 0.2, 200, nu=(2048, 2048), eps=1e-10, q=16, panels=5)
        prob.cheb = cheb
        u, wall, row, col, nt, _ = timed(prob, 2)
        grid[key] = {"NT": nt, "us_per_time_step": wall * 1e6 / prob.nsteps, "row_pass_us": row, "col_pass_us": col,
                     "u": u}
    ud, uc = grid["direct"].pop("u"), grid["interpolant"].pop("u")
    grid["rel_l2_interpolant_vs_direct"] = float(np.linalg.norm(uc - ud) / np.linalg.norm(ud))
    res["grid_256_nr5"] = grid
    return res


def batch_leg(runs: int, copies: dict, adjoint: bool = True) -> dict:
    """Batched form on the 64-instance workload (seed 4000 + i; 32 1D with
    M in {256..2048}, 32 2D with M in {128..512}^2; 500 steps, FP32-split,
    stepwise field): autotuned schedules, graph-replayed whole runs, against
    the same instances run one plan at a time; and the adjoint of every
    instance's <x_1>(T) with respect to its 500 field samples."""
    import numpy as np
    import torch

    from paper_2001_06113_amd.tdse import Q_BYTES_PER_STEP, BatchPlan, Plan
    from workloads import batch_64_problems

    dev = torch.device("cuda:0")
    probs = batch_64_problems()
    b = BatchPlan.from_problems(probs, device=dev)
    t0 = time.perf_counter()
    chosen = b.autotune(5)
    tune_s = time.perf_counter() - t0
    b.use_graph(True)
    u0 = b.pack([p.u0 for p in probs])
    out = b.run(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(runs):
        out = b.run(u0, out)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / runs
    nsteps = probs[0].nsteps
    value = b.total * nsteps / wall
    bytes_step = b.query(Q_BYTES_PER_STEP)
    errs = [oracle_error("batch_64", u, inst=i, bar=1e-6) for i, u in enumerate(b.unpack(out))]
    worst = max(errs, key=lambda e: e["rel_l2_vs_oracle"])
    # the same work one plan after another (each replayed from its own graph)
    seq = 0.0
    for p in probs:
        pl = Plan.from_problem(p, device=dev)
        pl.use_graph(True)
        ui = torch.as_tensor(p.u0).to(dev)
        oi = pl.run(ui)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pl.run(ui, oi)
        torch.cuda.synchronize()
        seq += time.perf_counter() - t1
        pl.close()
    # adjoint of <x_1>(T) for every instance, seeded from the batch output
    adj = {}
    lams = [] if adjoint else None
    if adjoint:
        for p, uT in zip(probs, b.unpack(out)):
            x = torch.as_tensor(-np.pi + 2 * np.pi * np.arange(p.M[0]) / p.M[0], device=dev)
            w = float(np.prod([2 * np.pi / m for m in p.M]))
            lams.append(2.0 * w * (x.reshape(-1, *([1] * (p.dim - 1)))) * uT)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gAs, _ = b.adjoint(u0, lams)
        torch.cuda.synchronize()
        adj_first_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        gAs, _ = b.adjoint(u0, lams)
        torch.cuda.synchronize()
        adj_s = time.perf_counter() - t0
        adj = {"adjoint_s_all_instances": adj_s, "adjoint_first_call_s": adj_first_s,
               "adjoint_vs_forward_run": adj_s / wall, "adjoint_samples": int(sum(g.size for g in gAs))}
    b.close()
    return {"workload": "64 periodic instances (32 1D M=256..2048, 32 2D M=128^2..512^2), T=2, 500 steps AM8, "
                        "FP32-split, stepwise A",
            "value": value, "unit": "mode-updates/s", "ms_per_run": wall * 1e3, "modes": int(b.total),
            "end_to_end": end_to_end(bytes_step, nsteps, wall, copies),
            "error": {"worst_instance": errs.index(worst), **worst,
                      "all_pass": all(e["pass"] for e in errs)},
            "one_plan_at_a_time_value": b.total * nsteps / seq, "speedup_vs_one_plan_at_a_time": seq / wall,
            "autotune_s": tune_s, "schedules_col_row": sorted(set(chosen)), **adj}


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU (no sharding across GPUs); --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2001_06113_amd import _lib
    from paper_2001_06113_amd.tdse import (CFG_PERSISTENT, Q_BYTES_COL, Q_BYTES_PER_STEP, Q_BYTES_ROW, Q_PATH,
                                           Q_PROF_MS_COL, Q_PROF_MS_PERSIST, Q_PROF_MS_ROW, Q_PROF_N_COL,
                                           Q_PROF_N_PERSIST, Q_PROF_N_ROW, Plan)
    from workloads import periodic_2d_512_problem, periodic_problem_from_seed

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2001_06113_amd import build

        build.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.workload == "periodic-2d-512":
        prob = periodic_2d_512_problem()
        wname = "2D periodic TDSE 512x512, T=2, 2000 steps AM8, FP64"
    else:
        prob = periodic_problem_from_seed(3, 2, (1024, 1024), 2.0, 2000, name="periodic-2d-1024-fp64")
        wname = "2D periodic TDSE 1024x1024, T=2, 2000 steps AM8, FP64"
    copy_gbps = device_copy_gbps(dev)
    copy_mall_gbps = device_copy_gbps(dev, mib=32, reps=200)
    copies = {"512MiB": copy_gbps, "32MiB_in_MALL": copy_mall_gbps}
    # The batched leg runs first: in a process that has made a cooperative
    # launch (the persistent 2D path below), kernels launched for the first
    # time afterwards from several streams at once run about 3x slower (the
    # eight-stream adjoint: 3.3 s instead of 1.06 s).
    batch = batch_leg(args.batch_runs, copies, not args.no_adjoint) if not args.no_batch else None
    plan = Plan.from_problem(prob, device=dev)
    u0 = torch.as_tensor(prob.u0).to(dev)
    out = torch.empty_like(u0)
    modes = float(u0.numel())

    # timed region: whole runs replayed from one captured hipGraph
    plan.use_graph(True)
    for _ in range(max(args.warmup, 1)):
        plan.run(u0, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.run(u0, out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ok = bool(torch.isfinite(torch.view_as_real(out)).all().item())

    # per-kernel durations: the same runs launched eagerly, every Adams
    # launch bracketed by HIP events on the library's stream
    path = plan.query(Q_PATH)
    plan.profile(True)
    for _ in range(args.prof_runs):
        plan.run(u0, out)
    p_ms, p_n = plan.query(Q_PROF_MS_PERSIST), plan.query(Q_PROF_N_PERSIST)
    plan.profile(False)
    ms_per_run = wall * 1e3 / args.steps
    value = modes * prob.nsteps * args.steps / wall
    err = oracle_error("periodic_2d_512" if args.workload == "periodic-2d-512" else "periodic_2d_1024", out)
    bytes_step = plan.query(Q_BYTES_PER_STEP)
    adams_steps = prob.nsteps - prob.start_steps - 1   # the Adams steps after the first (inside the persistent launch)

    # the same workload on the two-pass path (one column and one row launch per step)
    plan.configure(CFG_PERSISTENT, 0)
    plan.run(u0, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.run(u0, out)
    torch.cuda.synchronize()
    wall2 = (time.perf_counter() - t0) / args.steps
    err2 = oracle_error("periodic_2d_512" if args.workload == "periodic-2d-512" else "periodic_2d_1024", out)
    plan.profile(True)
    for _ in range(args.prof_runs):
        plan.run(u0, out)
    row_ms, col_ms = plan.query(Q_PROF_MS_ROW), plan.query(Q_PROF_MS_COL)
    n_row, n_col = plan.query(Q_PROF_N_ROW), plan.query(Q_PROF_N_COL)
    plan.profile(False)
    plan.configure(CFG_PERSISTENT, 1)

    row_us, col_us = row_ms * 1e3 / max(n_row, 1), col_ms * 1e3 / max(n_col, 1)
    row_b, col_b = plan.query(Q_BYTES_ROW), plan.query(Q_BYTES_COL)
    row_ach = row_b / (row_us * 1e-6) / 1e9 if row_us > 0 else None
    if path == 2.0 and p_n > 0:
        dom_us = p_ms * 1e3 / p_n
        dom_b = bytes_step * adams_steps
        kernel = f"persistent Adams launch (k_persist2d, {adams_steps} steps per launch)"
        traffic = measured_traffic("k_persist2d_512_traffic.txt", P2_KERNEL_SOURCES)
    else:
        dom_us, dom_b, kernel = row_us, row_b, "Adams row pass (k_row)"
        traffic = measured_traffic("k_row_512_fp64_traffic.txt")
    achieved = dom_b / (dom_us * 1e-6) / 1e9 if dom_us > 0 else None
    res = {
        "metric": "mode-updates/s",
        "value": value,
        "unit": "mode-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_run,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wname, "grid": list(prob.M), "time_steps": prob.nsteps,
                   "order": prob.order, "modes": int(modes), "seed": 1 if args.workload == "periodic-2d-512" else 3,
                   "finite": ok, "path": {0.0: "two passes per step", 2.0: "persistent Adams launch"}.get(path)},
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": traffic,
            "kernel": kernel,
            "bytes_per_launch": dom_b,
            "mean_launch_us": dom_us,
            "device_copy_GBps": copy_gbps,
            "frac_of_device_copy": achieved / copy_gbps if achieved else None,
            "device_copy_32MiB_in_MALL_GBps": copy_mall_gbps,
            "frac_of_device_copy_in_MALL": achieved / copy_mall_gbps if achieved else None,
        },
        "error": err,
        "end_to_end": end_to_end(bytes_step, prob.nsteps, wall / args.steps, copies),
        "graph_us_per_time_step": wall * 1e6 / (args.steps * prob.nsteps),
        "two_pass": {
            "value": modes * prob.nsteps / wall2, "ms_per_run": wall2 * 1e3,
            "us_per_time_step": wall2 * 1e6 / prob.nsteps, "error": err2,
            "end_to_end": end_to_end(bytes_step, prob.nsteps, wall2, copies),
            "row_pass_us": row_us, "col_pass_us": col_us, "row_bytes_per_launch": row_b,
            "col_bytes_per_launch": col_b,
            "row_pass_roofline": {"achieved": row_ach, "frac": row_ach / HBM_PEAK_GBS if row_ach else None,
                                  "traffic": measured_traffic("k_row_512_fp64_traffic.txt")},
            "adams_step_us_eager": row_us + col_us,
        },
    }
    if not args.no_1d:
        res["periodic_1d"] = periodic_1d_leg()
    if not args.no_split:
        res["split"] = split_leg(args.split_steps, copies)
    if not args.no_free:
        res["free_space"] = free_space_leg(args.free_runs, copies)
    if not args.no_well:
        res["moving_well"] = moving_well_leg()
    if not args.no_ionization:
        res["ionization"] = ionization_leg()
    if not args.no_long_time:
        res["long_time"] = long_time_leg()
    if not args.no_3d:
        res["periodic_3d"] = periodic_3d_leg(args.runs_3d, copies)
    if not args.no_sampled:
        res["sampled"] = sampled_leg(3, copies)
    if not args.no_free_3d:
        res["free_space_3d"] = free_space_3d_leg(3, copies)
    if batch is not None:
        res["batch"] = batch
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(prob, args.cpu_steps)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
