"""Run the emulated library (libtdse_emu.so) on host memory through the same
C ABI as the GPU build."""
import ctypes as C
import os

import numpy as np

from paper_2001_06113_amd import _lib

HERE = os.path.dirname(os.path.abspath(__file__))


def load(rebuild: bool = False):
    path = os.path.join(HERE, "libtdse_emu.so")
    if rebuild or not os.path.exists(path):
        from . import build_emu

        build_emu.build()
    saved = _lib.LIB_PATH, _lib._lib
    try:
        _lib.LIB_PATH, _lib._lib = path, None
        lib = _lib.load()
    finally:
        _lib.LIB_PATH, _lib._lib = saved
    return lib


class EmuPlan:
    """Plan of a workloads.Problem on the emulated library."""

    def __init__(self, lib, prob, H: float = 0.0):
        self.lib = lib
        p = _lib.Problem()
        p.dim = prob.dim
        p.domain = 0 if prob.domain == "periodic" else 1
        for a in range(prob.dim):
            p.M[a] = prob.M[a]
        p.T = prob.T
        p.nsteps = prob.nsteps
        p.order = prob.order
        p.n_start = -1 if prob.n_start is None else prob.n_start
        p.precision = 0 if prob.precision == "fp64" else 1
        self._keep = []
        if getattr(prob, "V_kind", "fields") == "moving_well":
            p.nV = 0
            p.V_kind = 1
            for k, v in enumerate(tuple(prob.V_well) + (0.0,) * (4 - len(prob.V_well))):
                p.V_params[k] = v
        elif getattr(prob, "V_kind", "fields") == "sampled":
            V = np.ascontiguousarray(np.asarray(prob.V_samples, dtype=np.float64))
            self._keep.append(V)
            p.nV = 0
            p.V_kind = 2
            p.V_fields = V.ctypes.data_as(C.POINTER(C.c_double))
        else:
            V = np.ascontiguousarray(np.stack(prob.V_fields).astype(np.float64))
            self._keep.append(V)
            p.nV = V.shape[0]
            p.V_fields = V.ctypes.data_as(C.POINTER(C.c_double))
        if any(k == "sin" for k in prob.f_kind):
            fp = np.array([tuple(f) if k == "sin" else (0.0, 0.0) for f, k in zip(prob.f_params, prob.f_kind)],
                          dtype=np.float64).ravel()
            self._keep.append(fp)
            p.f_kind = 1
            p.f_params = fp.ctypes.data_as(C.POINTER(C.c_double))
        kinds = {"none": 0, "pulse_sin2": 1, "stepwise": 3, "pulse_cos2": 4}
        p.A_kind = kinds[prob.A_kind]
        if prob.A_kind in ("pulse_sin2", "pulse_cos2"):
            ap = np.asarray(prob.A_params, dtype=np.float64)
            self._keep.append(ap)
            p.A_params = ap.ctypes.data_as(C.POINTER(C.c_double))
        if prob.A_kind == "stepwise":
            st = np.ascontiguousarray(np.asarray(prob.A_steps, dtype=np.float64).ravel())
            self._keep.append(st)
            p.A_steps = st.ctypes.data_as(C.POINTER(C.c_double))
        p.eps = prob.eps
        p.p = prob.p
        p.q = prob.q
        p.panels = prob.panels
        for a, n in enumerate(prob.nu):
            p.nu[a] = n
        p.H = H
        p.cheb = int(getattr(prob, "cheb", 0))
        self.prob = p
        h = C.c_void_p()
        st = lib.tdse_plan(C.byref(p), C.byref(h))
        if st:
            raise RuntimeError(lib.tdse_last_error().decode())
        self.h = h
        sz = C.c_size_t()
        lib.tdse_workspace_size(h, C.byref(sz))
        raw = np.zeros(sz.value + 512, dtype=np.uint8)
        off = (-raw.ctypes.data) % 256
        self.ws = raw[off:off + sz.value]
        self._raw = raw
        st = lib.tdse_bind(h, C.c_void_p(self.ws.ctypes.data), sz.value, None)
        if st:
            raise RuntimeError(lib.tdse_last_error().decode())
        self.shape = tuple(prob.M)

    def query(self, key: int) -> float:
        v = C.c_double()
        st = self.lib.tdse_query(self.h, key, C.byref(v))
        if st:
            raise RuntimeError(self.lib.tdse_last_error().decode())
        return v.value

    def run(self, u0):
        u0 = np.ascontiguousarray(np.asarray(u0, dtype=np.complex128))
        out = np.zeros(self.shape, dtype=np.complex128)
        st = self.lib.tdse_run(self.h, C.c_void_p(u0.ctypes.data), C.c_void_p(out.ctypes.data), 1)
        if st:
            raise RuntimeError(self.lib.tdse_last_error().decode())
        return out

    def call(self, name, *args):
        st = getattr(self.lib, name)(self.h, *args)
        if st:
            raise RuntimeError(self.lib.tdse_last_error().decode())

    def set_state(self, u0):
        self._u0 = np.ascontiguousarray(np.asarray(u0, dtype=np.complex128))
        self.call("tdse_set_state", C.c_void_p(self._u0.ctypes.data), 1)

    def step(self, k):
        self.call("tdse_step", int(k))

    def far_eval(self, ys, xs=None):
        """tdse_far_eval on the tensor grid xs x ys (1D: ys only)."""
        yd = np.ascontiguousarray(ys, dtype=np.float64)
        xd = None if xs is None else np.ascontiguousarray(xs, dtype=np.float64)
        nx, ny = (1 if xd is None else xd.size), yd.size
        sz = C.c_size_t()
        self.call("tdse_far_workspace_size", nx, ny, C.byref(sz))
        raw = np.zeros(sz.value + 512, dtype=np.uint8)
        off = (-raw.ctypes.data) % 256
        out = np.zeros((nx, ny), dtype=np.complex128)
        self.call("tdse_far_eval", None if xd is None else C.c_void_p(xd.ctypes.data), nx, C.c_void_p(yd.ctypes.data),
                  ny, C.c_void_p(out.ctypes.data), C.c_void_p(raw.ctypes.data + off), sz.value)
        return out if xd is not None else out.reshape(ny)

    def __del__(self):
        try:
            self.lib.tdse_destroy(self.h)
        except Exception:
            pass


class EmuBatchPlan:
    """Batch plan of several workloads.Problem on the emulated library; states packed in instance order."""

    def __init__(self, lib, probs):
        from paper_2001_06113_amd.tdse import problem_kwargs, problem_struct

        self.lib = lib
        structs, self._keep = [], []
        for pr in probs:
            s, k = problem_struct(**problem_kwargs(pr))
            structs.append(s)
            self._keep += k
        arr = (_lib.Problem * len(structs))(*structs)
        h = C.c_void_p()
        st = lib.tdse_plan_batch(arr, len(structs), C.byref(h))
        if st:
            raise RuntimeError(lib.tdse_last_error().decode())
        self.h = h
        sz = C.c_size_t()
        lib.tdse_workspace_size(h, C.byref(sz))
        raw = np.zeros(sz.value + 512, dtype=np.uint8)
        off = (-raw.ctypes.data) % 256
        self.ws = raw[off:off + sz.value]
        self._raw = raw
        st = lib.tdse_bind(h, C.c_void_p(self.ws.ctypes.data), sz.value, None)
        if st:
            raise RuntimeError(lib.tdse_last_error().decode())
        self.shapes = [tuple(pr.M) for pr in probs]
        self.fields = [(pr.nsteps, pr.dim) for pr in probs]
        self.offsets = [int(self.query(4096 + i)) for i in range(len(probs))]

    def query(self, key: int) -> float:
        v = C.c_double()
        st = self.lib.tdse_query(self.h, key, C.byref(v))
        if st:
            raise RuntimeError(self.lib.tdse_last_error().decode())
        return v.value

    def call(self, name, *args):
        st = getattr(self.lib, name)(self.h, *args)
        if st:
            raise RuntimeError(f"{name}: {self.lib.tdse_last_error().decode()}")

    def run(self, u0s):
        packed = np.ascontiguousarray(np.concatenate([np.asarray(u, dtype=np.complex128).ravel() for u in u0s]))
        out = np.zeros_like(packed)
        self.call("tdse_run", C.c_void_p(packed.ctypes.data), C.c_void_p(out.ctypes.data), 1)
        return [out[o:o + int(np.prod(s))].reshape(s) for o, s in zip(self.offsets, self.shapes)]

    def __del__(self):
        try:
            self.lib.tdse_destroy(self.h)
        except Exception:
            pass


def emu_adjoint(plan, u0, lam, checkpoint_every=0):
    """tdse_adjoint on an EmuPlan: (dJ/dA [nsteps, dim], dJ/du0)."""
    lib, h = plan.lib, plan.h
    sz = C.c_size_t()
    lib.tdse_adjoint_workspace_size(h, checkpoint_every, C.byref(sz))
    raw = np.zeros(sz.value + 512, dtype=np.uint8)
    off = (-raw.ctypes.data) % 256
    ws = raw[off:off + sz.value]
    u0 = np.ascontiguousarray(u0, dtype=np.complex128)
    lam = np.ascontiguousarray(lam, dtype=np.complex128)
    nsteps, dim = plan.prob.nsteps, plan.prob.dim
    gA = np.zeros((nsteps, dim))
    g0 = np.zeros_like(u0)
    st = lib.tdse_adjoint(h, C.c_void_p(ws.ctypes.data), sz.value, checkpoint_every, C.c_void_p(u0.ctypes.data),
                          C.c_void_p(lam.ctypes.data), 1, gA.ctypes.data_as(C.POINTER(C.c_double)),
                          C.c_void_p(g0.ctypes.data))
    if st:
        raise RuntimeError(lib.tdse_last_error().decode())
    return gA, g0


def emu_batch_adjoint(bplan, u0s, lams, checkpoint_every=0):
    """tdse_adjoint on an EmuBatchPlan: per-instance (dJ/dA [nsteps, dim], dJ/du0) lists."""
    lib, h = bplan.lib, bplan.h
    sz = C.c_size_t()
    st = lib.tdse_adjoint_workspace_size(h, checkpoint_every, C.byref(sz))
    if st:
        raise RuntimeError(lib.tdse_last_error().decode())
    raw = np.zeros(sz.value + 512, dtype=np.uint8)
    off = (-raw.ctypes.data) % 256
    ws = raw[off:off + sz.value]
    pack = lambda xs: np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.complex128).ravel() for x in xs]))
    u0 = pack(u0s)
    lam = pack(lams)
    sizes = [(nsteps, dim) for nsteps, dim in bplan.fields]
    gA = np.zeros(sum(n * d for n, d in sizes))
    g0 = np.zeros_like(u0)
    st = lib.tdse_adjoint(h, C.c_void_p(ws.ctypes.data), sz.value, checkpoint_every, C.c_void_p(u0.ctypes.data),
                          C.c_void_p(lam.ctypes.data), 1, gA.ctypes.data_as(C.POINTER(C.c_double)),
                          C.c_void_p(g0.ctypes.data))
    if st:
        raise RuntimeError(lib.tdse_last_error().decode())
    gAs, a = [], 0
    for n, d in sizes:
        gAs.append(gA[a:a + n * d].reshape(n, d))
        a += n * d
    g0s = [g0[o:o + int(np.prod(s))].reshape(s) for o, s in zip(bplan.offsets, bplan.shapes)]
    return gAs, g0s
