"""Python binding of libtdse.so: a Plan owns a device workspace (torch) and
forwards every call to the C ABI of include/tdse.h.  No arithmetic on the
solution happens here; torch supplies device memory and the stream."""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib

PERIODIC, FREE = 0, 1
FP64, FP32_SPLIT = 0, 1
F_KINDS = {"const": 0, "sin": 1, "callback": 2}
A_KINDS = {"none": 0, "pulse_sin2": 1, "callback": 2, "stepwise": 3, "pulse_cos2": 4}
Q_MODES, Q_STEPS_DONE, Q_DT, Q_BYTES_PER_STEP = 0, 1, 2, 3
Q_PROF_MS_COL, Q_PROF_MS_ROW, Q_PROF_N_COL, Q_PROF_N_ROW = 8, 9, 10, 11
Q_BYTES_COL, Q_BYTES_ROW = 12, 13
Q_PROF_MS_MID, Q_PROF_N_MID, Q_BYTES_MID = 5, 6, 7
Q_PROF_MS_FAR, Q_PROF_N_FAR = 14, 15
Q_MU, Q_RICHARDSON, Q_PHI = 16, 32, 64
Q_INSTANCES, Q_INST_OFFSET, Q_INST_EPT_COL, Q_INST_EPT_ROW = 4, 4096, 8192, 12288
Q_PROF_MS_RUN1D, Q_PROF_N_RUN1D, Q_PROF_MS_PERSIST, Q_PROF_N_PERSIST, Q_PATH = 24, 25, 26, 27, 28
Q_RESIDUAL, Q_STATE_NORM = 29, 30
Q_FS_H, Q_FS_MODES, Q_FS_NE = 80, 81, 83
Q_FS_H_AXIS, Q_FS_HSTEP, Q_FS_NU, Q_FS_K, Q_FS_CHEB, Q_FS_AXIS2 = 86, 128, 130, 132, 134, 136
CFG_PERSISTENT, CFG_GUARD = 0, 1


class TDSEError(RuntimeError):
    def __init__(self, status: int, call: str):
        lib = _lib.load()
        super().__init__(f"{call}: {lib.tdse_status_string(status).decode()} ({lib.tdse_last_error().decode()})")
        self.status = status


def _check(status: int, call: str) -> None:
    if status != 0:
        raise TDSEError(status, call)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def problem_struct(*, dim: int, M: Sequence[int], T: float, nsteps: int, V_fields, order: int = 8,
                   n_start: int = -1, precision: str = "fp64", f_kind: str = "const", f_params=None,
                   A_kind: str = "none", A_params=None, A_steps=None, domain: str = "periodic",
                   eps: float = 1e-10, p: int = 8, q: int = 10, panels: int = 1, nu: Sequence[int] = (),
                   H: float = 0.0, V_kind: str = "fields", V_params: Sequence[float] = (), cheb: int = 0):
    """Fill a tdse_problem_t; returns it with the arrays it points into (keep them alive).
    V_kind "moving_well" takes V_params = (V0, beta, c_0[, c_1]) and no fields;
    V_kind "sampled" takes V_fields = the samples V(x, t_n), n = 0..nsteps."""
    M = tuple(int(m) for m in M)
    well = V_kind == "moving_well"
    if V_kind not in ("fields", "moving_well", "sampled"):
        raise ValueError(f"unknown V_kind {V_kind!r}")
    V = None if well else np.ascontiguousarray(np.asarray(V_fields, dtype=np.float64).reshape(-1, *M))
    prob = _lib.Problem()
    prob.dim = dim
    prob.domain = PERIODIC if domain == "periodic" else FREE
    for a in range(dim):
        prob.M[a] = M[a]
    prob.T = float(T)
    prob.nsteps = int(nsteps)
    prob.order = int(order)
    prob.n_start = int(n_start)
    prob.precision = FP64 if precision == "fp64" else FP32_SPLIT
    keep = []
    if well:
        prob.nV = 0
        prob.V_kind = 1
        for k, v in enumerate(tuple(V_params) + (0.0,) * (4 - len(V_params))):
            prob.V_params[k] = float(v)
    else:
        if V_kind == "sampled":
            if V.shape[0] != int(nsteps) + 1:
                raise ValueError("sampled V needs nsteps + 1 samples")
            prob.nV = 0
            prob.V_kind = 2
        else:
            prob.nV = V.shape[0]
        keep.append(V)
        prob.V_fields = _dptr(V)
    prob.f_kind = F_KINDS[f_kind]
    if f_params is not None:
        fp = np.ascontiguousarray(np.asarray(f_params, dtype=np.float64).ravel())
        keep.append(fp)
        prob.f_params = _dptr(fp)
    prob.A_kind = A_KINDS[A_kind]
    if A_params is not None:
        ap = np.ascontiguousarray(np.asarray(A_params, dtype=np.float64).ravel())
        keep.append(ap)
        prob.A_params = _dptr(ap)
    if A_steps is not None:
        st = np.ascontiguousarray(np.asarray(A_steps, dtype=np.float64).ravel())
        keep.append(st)
        prob.A_steps = _dptr(st)
    # free space: contour tolerance, Alpert order, Gauss panels, FFT sizes
    prob.eps = float(eps)
    prob.p = int(p)
    prob.q = int(q)
    prob.panels = int(panels)
    for a, n in enumerate(nu):
        prob.nu[a] = int(n)
    prob.H = float(H)
    prob.cheb = int(cheb)
    return prob, keep


def problem_kwargs(prob) -> dict:
    """Keyword arguments of problem_struct / Plan for a workloads.Problem
    (duck-typed: the plain problem fields)."""
    # one time-factor kind for all fields: constant fields get amplitude 0
    sin = any(k == "sin" for k in prob.f_kind)
    f_params = None
    if sin:
        f_params = [tuple(fp) if k == "sin" else (0.0, 0.0) for fp, k in zip(prob.f_params, prob.f_kind)]
    kind = getattr(prob, "V_kind", "fields")
    well = kind == "moving_well"
    if kind == "sampled":
        fields = np.asarray(prob.V_samples)
    else:
        fields = None if well else np.stack(prob.V_fields)
    return dict(dim=prob.dim, M=prob.M, T=prob.T, nsteps=prob.nsteps,
                V_fields=fields, V_kind=kind, V_params=tuple(prob.V_well) if well else (),
                order=prob.order, n_start=-1 if prob.n_start is None else prob.n_start,
                precision=prob.precision, f_kind="sin" if sin else "const", f_params=f_params,
                A_kind=prob.A_kind, A_params=prob.A_params if prob.A_kind in ("pulse_sin2", "pulse_cos2") else None,
                A_steps=prob.A_steps if prob.A_kind == "stepwise" else None,
                domain=prob.domain, eps=prob.eps, p=prob.p, q=prob.q, panels=prob.panels, nu=prob.nu,
                cheb=getattr(prob, "cheb", 0))


class Plan:
    """One TDSE instance planned and bound to a device workspace.

    Arguments follow the problem statement: grid M, final time T, number of
    steps, implicit Adams order, potential fields V_r(x) with time factors
    f_r(t) and the vector potential A(t).
    """

    def __init__(self, *, device=None, stream=None, **problem):
        self.lib = _lib.load()
        self.dim = problem["dim"]
        self.nsteps = int(problem["nsteps"])
        self.M = tuple(int(m) for m in problem["M"])
        self.shape = self.M
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        prob, keep = problem_struct(**problem)
        handle = C.c_void_p()
        _check(self.lib.tdse_plan(C.byref(prob), C.byref(handle)), "tdse_plan")
        self.handle = handle
        size = C.c_size_t()
        _check(self.lib.tdse_workspace_size(handle, C.byref(size)), "tdse_workspace_size")
        self.ws_bytes = size.value
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        # the plan's own stream (default priority); calls order it after the
        # caller's current stream and the caller's stream after it
        self.stream = torch.cuda.Stream(self.device) if stream is None else stream
        _check(self.lib.tdse_bind(handle, C.c_void_p(self.workspace.data_ptr()), self.ws_bytes,
                                  C.c_void_p(self.stream.cuda_stream)), "tdse_bind")
        self.graph = False

    @classmethod
    def from_problem(cls, prob, **kw) -> "Plan":
        """Plan a workloads.Problem (duck-typed: the plain problem fields)."""
        return cls(**{**problem_kwargs(prob), **kw})

    # -------------------------------------------------------------- calls
    def _as_device(self, u) -> torch.Tensor:
        t = torch.as_tensor(u)
        return t.to(device=self.device, dtype=torch.complex128).contiguous().reshape(self.shape)

    def _enter(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def set_state(self, u0) -> None:
        self._u0 = self._as_device(u0)
        self._enter()
        _check(self.lib.tdse_set_state(self.handle, C.c_void_p(self._u0.data_ptr()), 1), "tdse_set_state")

    def step(self, k: int) -> None:
        self._enter()
        _check(self.lib.tdse_step(self.handle, int(k)), "tdse_step")
        self._leave()

    def get_state(self) -> torch.Tensor:
        out = torch.empty(self.shape, dtype=torch.complex128, device=self.device)
        self._enter()
        _check(self.lib.tdse_get_state(self.handle, C.c_void_p(out.data_ptr()), 1), "tdse_get_state")
        self._leave()
        return out

    def use_graph(self, enable: bool = True) -> None:
        """Replay the whole run from one captured hipGraph (tdse_graph)."""
        _check(self.lib.tdse_graph(self.handle, 1 if enable else 0), "tdse_graph")
        self.graph = bool(enable)

    def run(self, u0, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        u0d = self._as_device(u0)
        self._u0 = u0d
        if out is None:
            out = torch.empty(self.shape, dtype=torch.complex128, device=self.device)
        self._enter()
        _check(self.lib.tdse_run(self.handle, C.c_void_p(u0d.data_ptr()), C.c_void_p(out.data_ptr()), 1), "tdse_run")
        self._leave()
        return out

    def query(self, key: int) -> float:
        v = C.c_double()
        _check(self.lib.tdse_query(self.handle, int(key), C.byref(v)), "tdse_query")
        return v.value

    def set_field(self, A_steps) -> None:
        """New stepwise field samples [nsteps, dim] (tdse_set_field)."""
        a = np.ascontiguousarray(np.asarray(A_steps, dtype=np.float64).ravel())
        _check(self.lib.tdse_set_field(self.handle, _dptr(a)), "tdse_set_field")

    def adjoint(self, u0, lam, checkpoint_every: int = 0):
        """dJ/dA [nsteps, dim] (numpy) and dJ/du0 (device tensor) for dJ = Re <lam, du(T)>
        (tdse_adjoint); the plan's state is overwritten."""
        u0d = self._as_device(u0)
        lamd = self._as_device(lam)
        size = C.c_size_t()
        _check(self.lib.tdse_adjoint_workspace_size(self.handle, int(checkpoint_every), C.byref(size)),
               "tdse_adjoint_workspace_size")
        if getattr(self, "_adj_ws", None) is None or self._adj_ws.numel() < size.value:
            self._adj_ws = torch.empty(size.value, dtype=torch.uint8, device=self.device)
        n_out = int(sum(self._field_shape()))
        gA = np.zeros(n_out, dtype=np.float64)
        g0 = torch.empty_like(u0d)
        self._enter()
        _check(self.lib.tdse_adjoint(self.handle, C.c_void_p(self._adj_ws.data_ptr()), size.value,
                                     int(checkpoint_every), C.c_void_p(u0d.data_ptr()), C.c_void_p(lamd.data_ptr()),
                                     1, _dptr(gA), C.c_void_p(g0.data_ptr())), "tdse_adjoint")
        self._leave()
        return self._split_field(gA), g0

    def far_eval(self, ys, xs=None) -> torch.Tensor:
        """u at the tensor grid xs x ys (1D: ys only) from the free-space mode
        state at the current time (tdse_far_eval); complex128 [nx, ny] (2D) or [ny]."""
        yd = torch.as_tensor(ys, dtype=torch.float64).to(self.device).contiguous().reshape(-1)
        xd = None if xs is None else torch.as_tensor(xs, dtype=torch.float64).to(self.device).contiguous().reshape(-1)
        nx = 1 if xd is None else xd.numel()
        ny = yd.numel()
        size = C.c_size_t()
        _check(self.lib.tdse_far_workspace_size(self.handle, nx, ny, C.byref(size)), "tdse_far_workspace_size")
        if getattr(self, "_far_ws", None) is None or self._far_ws.numel() < size.value:
            self._far_ws = torch.empty(max(size.value, 1), dtype=torch.uint8, device=self.device)
        out = torch.empty((nx, ny), dtype=torch.complex128, device=self.device)
        self._enter()
        _check(self.lib.tdse_far_eval(self.handle, None if xd is None else C.c_void_p(xd.data_ptr()), nx,
                                      C.c_void_p(yd.data_ptr()), ny, C.c_void_p(out.data_ptr()),
                                      C.c_void_p(self._far_ws.data_ptr()), self._far_ws.numel()), "tdse_far_eval")
        self._leave()
        self._far_keep = (xd, yd)   # inputs stay alive until the stream has used them
        return out if self.dim == 2 else out.reshape(ny)

    def far_eval_noalloc(self, ys, xs=None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """far_eval through the allocation-free entry point (tdse_far_eval_noalloc):
        the library's own device array is the workspace; `out` may be given."""
        yd = torch.as_tensor(ys, dtype=torch.float64).to(self.device).contiguous().reshape(-1)
        xd = None if xs is None else torch.as_tensor(xs, dtype=torch.float64).to(self.device).contiguous().reshape(-1)
        nx = 1 if xd is None else xd.numel()
        ny = yd.numel()
        if out is None:
            out = torch.empty((nx, ny), dtype=torch.complex128, device=self.device)
        self._enter()
        _check(self.lib.tdse_far_eval_noalloc(self.handle, None if xd is None else C.c_void_p(xd.data_ptr()), nx,
                                              C.c_void_p(yd.data_ptr()), ny, C.c_void_p(out.data_ptr())),
               "tdse_far_eval_noalloc")
        self._leave()
        self._far_keep = (xd, yd)
        return out if self.dim == 2 else out.reshape(ny)

    def adjoint_streams(self, streams: int) -> None:
        """Host threads / streams of a batch adjoint (tdse_adjoint_streams; 1 = one instance at a time)."""
        _check(self.lib.tdse_adjoint_streams(self.handle, int(streams)), "tdse_adjoint_streams")

    def _field_shape(self):
        return [self.nsteps * self.dim]

    def _split_field(self, flat):
        return flat.reshape(self.nsteps, self.dim)

    def configure(self, key: int, value: int) -> None:
        """Plan option (tdse_configure), e.g. CFG_PERSISTENT."""
        _check(self.lib.tdse_configure(self.handle, int(key), int(value)), "tdse_configure")

    def profile(self, enable: bool) -> None:
        _check(self.lib.tdse_profile(self.handle, 1 if enable else 0), "tdse_profile")

    def close(self) -> None:
        if getattr(self, "handle", None):
            self.lib.tdse_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan(Plan):
    """Many independent periodic instances marched together (tdse_plan_batch):
    one workspace, one stream, batched launches per pass.  States are lists of
    per-instance arrays (or one packed complex128 tensor)."""

    def __init__(self, problems: Sequence[dict], *, device=None, stream=None):
        self.lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        structs, keep = [], []
        for kw in problems:
            pr, k = problem_struct(**kw)
            structs.append(pr)
            keep += k
        arr = (_lib.Problem * len(structs))(*structs)
        self.shapes = [tuple(int(m) for m in kw["M"]) for kw in problems]
        self.field_shapes = [(int(kw["nsteps"]), int(kw["dim"])) for kw in problems]
        self.count = len(structs)
        handle = C.c_void_p()
        _check(self.lib.tdse_plan_batch(arr, len(structs), C.byref(handle)), "tdse_plan_batch")
        self.handle = handle
        size = C.c_size_t()
        _check(self.lib.tdse_workspace_size(handle, C.byref(size)), "tdse_workspace_size")
        self.ws_bytes = size.value
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(self.device) if stream is None else stream
        _check(self.lib.tdse_bind(handle, C.c_void_p(self.workspace.data_ptr()), self.ws_bytes,
                                  C.c_void_p(self.stream.cuda_stream)), "tdse_bind")
        self.graph = False
        self.offsets = [int(self.query(Q_INST_OFFSET + i)) for i in range(self.count)]
        self.total = int(self.query(Q_MODES))
        self.shape = (self.total,)

    @classmethod
    def from_problems(cls, probs, **kw) -> "BatchPlan":
        return cls([problem_kwargs(p) for p in probs], **kw)

    def pack(self, states) -> torch.Tensor:
        if isinstance(states, torch.Tensor) and states.dim() == 1:
            return states.to(device=self.device, dtype=torch.complex128).contiguous()
        parts = [torch.as_tensor(u).to(device=self.device, dtype=torch.complex128).reshape(-1) for u in states]
        return torch.cat(parts).contiguous()

    def unpack(self, packed: torch.Tensor):
        return [packed[o:o + int(np.prod(s))].reshape(s) for o, s in zip(self.offsets, self.shapes)]

    def _as_device(self, u) -> torch.Tensor:
        return self.pack(u)

    def autotune(self, reps: int = 20) -> list:
        """Time the compiled schedules per line length (tdse_autotune); the
        state is lost.  Returns the chosen (column, row) elements per thread."""
        self._enter()
        _check(self.lib.tdse_autotune(self.handle, int(reps)), "tdse_autotune")
        self._leave()
        return [(int(self.query(Q_INST_EPT_COL + i)), int(self.query(Q_INST_EPT_ROW + i))) for i in range(self.count)]

    def set_instance_state(self, i: int, u0) -> None:
        u = torch.as_tensor(u0).to(device=self.device, dtype=torch.complex128).contiguous()
        self._keep_states = getattr(self, "_keep_states", {})
        self._keep_states[i] = u
        self._enter()
        _check(self.lib.tdse_set_instance_state(self.handle, int(i), C.c_void_p(u.data_ptr()), 1),
               "tdse_set_instance_state")

    def get_instance_state(self, i: int) -> torch.Tensor:
        out = torch.empty(self.shapes[i], dtype=torch.complex128, device=self.device)
        self._enter()
        _check(self.lib.tdse_get_instance_state(self.handle, int(i), C.c_void_p(out.data_ptr()), 1),
               "tdse_get_instance_state")
        self._leave()
        return out

    def _field_shape(self):
        return [n * d for n, d in self.field_shapes]

    def _split_field(self, flat):
        out, o = [], 0
        for n, d in self.field_shapes:
            out.append(flat[o:o + n * d].reshape(n, d))
            o += n * d
        return out

    def run_list(self, u0s):
        return self.unpack(self.run(u0s))


class TDSEFunction(torch.autograd.Function):
    """u(T) as a differentiable function of the stepwise field samples (and of
    u0) of a planned periodic problem: forward sets the samples and runs the
    plan; backward is the library's adjoint (tdse_adjoint), seeded with the
    incoming gradient of u(T) (torch's convention dJ = Re <grad, du>).

        uT = TDSEFunction.apply(A_steps, plan, u0)        # A_steps [nsteps, dim] float64
    """

    @staticmethod
    def forward(ctx, A_steps, plan, u0, checkpoint_every=0):
        # the field this output was computed with: backward restores it, since
        # the plan may have been given another field (or run again) meanwhile
        A_host = np.array(A_steps.detach().cpu().numpy(), dtype=np.float64, copy=True)
        plan.set_field(A_host)
        u0d = plan._as_device(u0.detach() if isinstance(u0, torch.Tensor) else u0).clone()
        out = plan.run(u0d)
        ctx.plan, ctx.u0, ctx.k, ctx.A_host = plan, u0d, int(checkpoint_every), A_host
        ctx.A_meta = (A_steps.dtype, A_steps.device)
        ctx.u0_is_tensor = isinstance(u0, torch.Tensor)
        return out

    @staticmethod
    def backward(ctx, grad_uT):
        ctx.plan.set_field(ctx.A_host)
        gA, g0 = ctx.plan.adjoint(ctx.u0, grad_uT.detach().contiguous(), ctx.k)
        dtype, device = ctx.A_meta
        gA_t = torch.as_tensor(np.asarray(gA), dtype=dtype, device=device)
        return gA_t, None, (g0 if ctx.u0_is_tensor else None), None
