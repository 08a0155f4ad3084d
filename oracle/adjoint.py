"""Reverse-mode (adjoint) derivative of the periodic scheme, FP64 oracle.

Test infrastructure only (see the package docstring).

The discrete scheme of ``periodic.PeriodicOracle`` (Richardson start-up of
order-2 sub-steps, eq. (utrapk); implicit Adams steps, eq. (uadamsk)) is a
linear map u0 -> u_N for a fixed vector potential; the field enters only
through the phase factors of Lemma 1,
    P = exp(-i |k|^2 tau + i k . (phi(t_b) - phi(t_a))),  phi(t) = int_0^t A,
so with a piecewise-constant A (one sample A_m per step [t_m, t_{m+1}))
    d phi(t_b) - phi(t_a) / d A_m = |[t_a, t_b] n [t_m, t_{m+1}]|  (per axis).

For a real objective J(u_N) with dJ = Re <lam, du_N> (lam = "lam_T", e.g.
2 w x1 u_N for J = <x1> = w sum_j x1_j |u_N,j|^2, w the cell volume), this
module forms every forward array, then walks the steps backwards applying the
conjugate transpose of each linear operation:
    F = fftn / M^d         ->  F^H g    = ifftn(g)
    F^-1 = ifftn * M^d     ->  F^-H g   = fftn(g)
    y = P x                ->  g_x = conj(P) g_y,
                               dJ/dtheta_k = Re(conj(g_y,k) i P_k x_k)
    y = x / (1 + i c V)    ->  g_x = g_y / (1 - i c V)
and dJ/d(k . dphi) is summed over modes with the weight k_a for axis a.
Returns dJ/dA (shape [nsteps, dim]) and dJ/du0 (dJ = Re <g, du0>).
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np

from .adams import richardson_weights_exact
from .periodic import PeriodicOracle


def dipole(prob, u: np.ndarray, axis: int = 0) -> float:
    """<x_axis> = w sum_j x_j |u_j|^2 on the periodic grid x_j = -pi + 2 pi j / M."""
    x = -np.pi + 2.0 * np.pi * np.arange(prob.M[axis]) / prob.M[axis]
    shape = [1] * prob.dim
    shape[axis] = prob.M[axis]
    w = float(np.prod([2.0 * np.pi / m for m in prob.M]))
    return float(w * np.sum(x.reshape(shape) * np.abs(u) ** 2))


def dipole_seed(prob, u: np.ndarray, axis: int = 0) -> np.ndarray:
    """lam with d<x_axis> = Re <lam, du>:  lam = 2 w x u."""
    x = -np.pi + 2.0 * np.pi * np.arange(prob.M[axis]) / prob.M[axis]
    shape = [1] * prob.dim
    shape[axis] = prob.M[axis]
    w = float(np.prod([2.0 * np.pi / m for m in prob.M]))
    return 2.0 * w * x.reshape(shape) * u


class _Grad:
    """Accumulates dJ/dA from dJ/d(dphi) of each phase application."""

    def __init__(self, prob):
        self.dt = prob.dt
        self.N = prob.nsteps
        self.g = np.zeros((prob.nsteps, prob.dim))

    def add(self, t_a: float, t_b: float, dphi_grad: np.ndarray):
        m0 = int(np.floor(t_a / self.dt + 1e-9))
        m1 = int(np.ceil(t_b / self.dt - 1e-9))
        for m in range(max(m0, 0), min(m1, self.N)):
            lo, hi = max(t_a, m * self.dt), min(t_b, (m + 1) * self.dt)
            if hi > lo:
                self.g[m] += (hi - lo) * dphi_grad


def _phase_grad(orc: PeriodicOracle, g_y: np.ndarray, P: np.ndarray, x: np.ndarray) -> np.ndarray:
    """dJ/d(dphi_a) for y = P x:  sum_k k_a Re(conj(g_y) i P x)."""
    core = np.real(np.conj(g_y) * 1j * P * x)
    return np.array([np.sum(orc.K[a] * core) for a in range(orc.d)])


def adjoint(prob, lam_T: np.ndarray):
    """(dJ/dA [nsteps, dim], dJ/du0) for dJ = Re <lam_T, du_N> (stepwise A)."""
    assert prob.A_kind == "stepwise"
    orc = PeriodicOracle(prob)
    dt = prob.dt
    N = prob.nsteps
    n = prob.order
    ns = min(prob.start_steps, N)
    levels = n // 2
    mu = orc.mu
    rw = [float(r) for r in richardson_weights_exact(levels)]
    grad = _Grad(prob)
    F, Finv = orc.F, orc.Finv

    def Fh(g):            # F^H
        return np.fft.ifftn(g)

    def Finvh(g):         # (F^-1)^H
        return np.fft.fftn(g)

    # ---------------- forward, keeping what the reverse sweep reads
    u0 = np.asarray(prob.u0, dtype=np.complex128).copy()
    us = [u0]
    subs = {}             # (m, l) -> list of (u_in, g = F((1 - i d/2 V) u_in), t, d)
    for m in range(1, ns + 1):
        t = (m - 1) * dt
        results = []
        for l in range(levels):
            nsub = 2 ** l
            d = dt / nsub
            v = us[-1]
            rec = []
            for s in range(nsub):
                ts = t + s * d
                g = F((1.0 - 0.5j * d * orc.V(ts)) * v)
                rec.append((v, g, ts, d))
                w = Finv(orc.prop(ts + d, d) * g)
                v = w / (1.0 + 0.5j * d * orc.V(ts + d))
            subs[(m, l)] = rec
            results.append(v)
        us.append(sum(r * x for r, x in zip(rw, results)))
    if N > ns:
        uhat = {ns: F(us[ns])}
        W = {m: F(orc.V(m * dt) * us[m]) for m in range(max(0, ns - (n - 2)), ns + 1)}
        B = {}
        u = None
        for step in range(ns + 1, N + 1):
            tn = step * dt
            Bn = orc.prop(tn, dt) * uhat[step - 1]
            for j in range(1, n):
                Bn = Bn - 1j * dt * mu[j] * orc.prop(tn, j * dt) * W[step - j]
            B[step] = Bn
            u = Finv(Bn) / (1.0 + 1j * mu[0] * dt * orc.V(tn))
            W[step] = F(orc.V(tn) * u)
            uhat[step] = Bn - 1j * mu[0] * dt * W[step]

    # ---------------- reverse sweep
    g_u = defaultdict(lambda: 0.0)
    g_W = defaultdict(lambda: 0.0)
    g_u[N] = np.asarray(lam_T, dtype=np.complex128)
    if N > ns:
        g_uhat = 0.0
        for step in range(N, ns, -1):
            tn = step * dt
            Vn = orc.V(tn)
            # uhat_step = B - i mu0 dt W_step
            gB = g_uhat + 0.0
            g_W[step] = g_W[step] + 1j * mu[0] * dt * g_uhat
            # W_step = F(V u_step)
            g_u[step] = g_u[step] + Vn * Fh(g_W[step])
            # u_step = F^-1 B / (1 + i mu0 dt V)
            gB = gB + Finvh(g_u[step] / (1.0 - 1j * mu[0] * dt * Vn))
            # B = P1 uhat_{step-1} - i dt sum_j mu_j P_j W_{step-j}
            P1 = orc.prop(tn, dt)
            grad.add(tn - dt, tn, _phase_grad(orc, gB, P1, uhat[step - 1]))
            g_uhat = np.conj(P1) * gB
            for j in range(1, n):
                Pj = orc.prop(tn, j * dt)
                x = -1j * dt * mu[j] * W[step - j]
                grad.add(tn - j * dt, tn, _phase_grad(orc, gB, Pj, x))
                g_W[step - j] = g_W[step - j] + 1j * dt * mu[j] * np.conj(Pj) * gB
        # uhat_ns = F u_ns;  W_m = F(V u_m), m <= ns
        g_u[ns] = g_u[ns] + Fh(g_uhat)
        for m in range(max(0, ns - (n - 2)), ns + 1):
            g_u[m] = g_u[m] + orc.V(m * dt) * Fh(g_W[m])
    # start-up, newest step first
    for m in range(ns, 0, -1):
        for l in range(levels):
            gv = rw[l] * g_u[m]
            for (v_in, g, ts, d) in reversed(subs[(m, l)]):
                # v = F^-1(P g) / (1 + i d/2 V(ts + d))
                gw = gv / (1.0 - 0.5j * d * orc.V(ts + d))
                gy = Finvh(gw)
                P = orc.prop(ts + d, d)
                grad.add(ts, ts + d, _phase_grad(orc, gy, P, g))
                gg = np.conj(P) * gy
                # g = F((1 - i d/2 V(ts)) v_in)
                gv = (1.0 + 0.5j * d * orc.V(ts)) * Fh(gg)
            g_u[m - 1] = g_u[m - 1] + gv
    return grad.g, np.asarray(g_u[0], dtype=np.complex128)
