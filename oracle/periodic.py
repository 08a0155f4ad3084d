"""FP64 oracle of the periodic marching scheme (Sections 2.1 and 2.2).

Test infrastructure only (see the package docstring).

Discretization (Section 2.1, eqs. (ftperdisc) and (utrapkdisc)):
  grid x_j = -pi + 2 pi j / M, modes k = -M/2 .. M/2-1 per axis;
  forward transform  F f = (1/M^d) sum_j e^{-2 pi i j.k/M} f_j  (numpy fftn / M^d);
  inverse transform  F^-1 g = sum_k e^{+2 pi i j.k/M} g_k      (numpy ifftn * M^d).
The phase e^{-i k.x} offset from x_0 = -pi is dropped on both sides, as in
eqs. (ftperdisc) and (utrapkdisc); it cancels in the step.

Propagator (eq. (uhatkinteq) and Lemma 1): over a time interval of length
``tau`` ending at t_b and starting at t_a = t_b - tau,
  P_k = exp(-i |k|^2 tau + i k . (phi(t_b) - phi(t_a))),  phi(t) = int_0^t A.

Order-2 sub-step (eq. (utrapk)): u(t+d) = F^-1[P F((1 - i d/2 V(t)) u(t))] / (1 + i d/2 V(t+d)).
Implicit Adams step (eq. (uadamsk)) with Fourier state uhat and history What:
  B   = P(t_{n-1}->t_n) uhat_{n-1} - i dt sum_{j=1}^{n-1} mu_j P(t_{n-j}->t_n) What_{n-j}
  u_n = F^-1 B / (1 + i mu_0 dt V(t_n)),   What_n = F(V(t_n) u_n),
  uhat_n = B - i mu_0 dt What_n            (the recurrence of Section 2.2).
Start-up: n-2 steps of iterated Richardson extrapolation of the order-2
sub-step (Section 2.2), with V and phi evaluated at the sub-step times.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, List, Optional

import numpy as np

from .adams import adams_coefficients, richardson_extrapolate
from .potential import sampled_V


def make_phi(prob) -> Callable[[float], np.ndarray]:
    """phi(t) = int_0^t A(s) ds (eq. (phi)).

    Smooth A: Gauss-Legendre quadrature step by step.  Stepwise A: exact
    integral of the piecewise-constant samples.
    """
    d = prob.dim
    if prob.A_kind == "none":
        return lambda t: np.zeros(d)
    if prob.A_kind == "stepwise":
        dt = prob.dt
        steps = np.asarray(prob.A_steps, dtype=np.float64)
        cums = np.vstack([np.zeros((1, d)), np.cumsum(steps * dt, axis=0)])

        def phi_step(t: float) -> np.ndarray:
            m = int(np.floor(t / dt + 1e-12))
            m = min(max(m, 0), prob.nsteps - 1)
            return cums[m] + steps[m] * (t - m * dt)

        return phi_step

    # smooth A: phi(t) = sum of quadratures over whole steps [t_i, t_{i+1}] up to the
    # step containing t, plus quad over the remaining part of that step
    dt = prob.dt
    nodes = {0: np.zeros(d)}

    # a 40-point Gauss-Legendre rule on one step (or part of one) is exact to
    # rounding for the smooth pulses used here (omega dt << 1)
    gx, gw = np.polynomial.legendre.leggauss(40)

    def piece(a: float, b: float) -> np.ndarray:
        s = 0.5 * (a + b) + 0.5 * (b - a) * gx
        vals = np.array([prob.A(si) for si in s])
        return 0.5 * (b - a) * (gw @ vals)

    def at_step(m: int) -> np.ndarray:
        top = max(k for k in nodes if k <= m)
        while top < m:
            nodes[top + 1] = nodes[top] + piece(top * dt, (top + 1) * dt)
            top += 1
        return nodes[m]

    def phi_smooth(t: float) -> np.ndarray:
        m = int(np.floor(t / dt + 1e-9))
        if abs(t - m * dt) <= 1e-14 * max(1.0, abs(t)):
            return at_step(m).copy()
        return at_step(m) + piece(m * dt, t)

    return phi_smooth


@dataclass
class PeriodicOracle:
    """The periodic scheme for one problem (workloads.Problem)."""

    prob: object
    phi: Optional[Callable[[float], np.ndarray]] = None

    def __post_init__(self):
        p = self.prob
        assert p.domain == "periodic"
        self.d = p.dim
        self.shape = tuple(p.M)
        # integer modes in numpy's FFT order, k in [-M/2, M/2)
        ks = [np.fft.fftfreq(m) * m for m in self.shape]
        self.K = list(np.meshgrid(*ks, indexing="ij"))
        self.K2 = sum(k * k for k in self.K)
        if self.phi is None:
            self.phi = make_phi(p)
        self._phi_cache = {}
        self.mu = [float(m) for m in adams_coefficients(p.order)]

    # --- transforms (Section 2.1, eq. (ftperdisc)) --------------------------
    def F(self, f: np.ndarray) -> np.ndarray:
        return np.fft.fftn(f) / f.size

    def Finv(self, g: np.ndarray) -> np.ndarray:
        return np.fft.ifftn(g) * g.size

    # --- problem data ---------------------------------------------------------
    def V(self, t: float) -> np.ndarray:
        p = self.prob
        if getattr(p, "V_kind", "fields") == "moving_well":
            return self.moving_well(t)
        if getattr(p, "V_kind", "fields") == "sampled":
            return sampled_V(p.V_samples, t, p.dt)
        out = np.zeros(self.shape)
        for r, Vr in enumerate(p.V_fields):
            out = out + p.f(r, t) * Vr
        return out

    def moving_well(self, t: float) -> np.ndarray:
        """Example 1 of Section 6: the periodic extension of a Gaussian well
        of depth V0 and width beta whose centre moves as c t,
            V(x, t) = sum over k in Z^d of -V0 exp(-|x - 2 pi k - c t|^2 / (2 beta^2)),
        summed over every image within 3 periods of the centre (for beta <= 1
        the rest are below exp(-(5 pi)^2 / 2)).  Cached per time."""
        key = float(t)
        cache = self.__dict__.setdefault("_well_cache", {})
        if key in cache:
            return cache[key].copy()
        p = self.prob
        V0, beta = p.V_well[0], p.V_well[1]
        c = np.asarray(p.V_well[2:2 + p.dim], dtype=np.float64)
        axes = [-np.pi + 2.0 * np.pi * np.arange(m) / m for m in p.M]
        X = np.meshgrid(*axes, indexing="ij")
        out = np.zeros(self.shape)
        # the images that matter have x - 2 pi k - c t in [-pi, pi): k near -c t / (2 pi)
        k0 = [int(np.round(-c[a] * t / (2.0 * np.pi))) for a in range(p.dim)]
        ranges = [range(k0[a] - 3, k0[a] + 4) for a in range(p.dim)]
        for ks in np.array(np.meshgrid(*ranges, indexing="ij")).reshape(p.dim, -1).T:
            r2 = np.zeros(self.shape)
            for a in range(p.dim):
                r2 = r2 + (X[a] - 2.0 * np.pi * ks[a] - c[a] * t) ** 2
            out = out - V0 * np.exp(-r2 / (2.0 * beta * beta))
        cache[key] = out
        return out.copy()

    def phi_at(self, t: float) -> np.ndarray:
        key = float(t)
        if key not in self._phi_cache:
            self._phi_cache[key] = np.asarray(self.phi(t), dtype=np.float64)
        return self._phi_cache[key]

    def prop(self, t_b: float, tau: float) -> np.ndarray:
        """P over [t_b - tau, t_b] (Lemma 1 phase factor)."""
        dphi = self.phi_at(t_b) - self.phi_at(t_b - tau)
        arg = -self.K2 * tau
        for a in range(self.d):
            arg = arg + self.K[a] * dphi[a]
        return np.exp(1j * arg)

    # --- order-2 sub-step and Richardson start-up (Section 2.2) ---------------
    def trap_substep(self, u: np.ndarray, t: float, delta: float) -> np.ndarray:
        g = self.F((1.0 - 0.5j * delta * self.V(t)) * u)
        w = self.Finv(self.prop(t + delta, delta) * g)
        return w / (1.0 + 0.5j * delta * self.V(t + delta))

    def richardson_step(self, u: np.ndarray, t: float, dt: float, levels: int) -> np.ndarray:
        results = []
        for l in range(levels):
            nsub = 2 ** l
            v = u
            for s in range(nsub):
                v = self.trap_substep(v, t + s * dt / nsub, dt / nsub)
            results.append(v)
        return richardson_extrapolate(results)

    # --- full run ------------------------------------------------------------
    def run(self, nsteps: Optional[int] = None, keep: bool = False):
        """March u0 to t = nsteps * dt; returns (u_N, info)."""
        p = self.prob
        dt = p.dt
        N = p.nsteps if nsteps is None else nsteps
        n = p.order
        ns = min(p.start_steps, N)
        levels = n // 2
        mu = self.mu
        u = np.asarray(p.u0, dtype=np.complex128).copy()
        us = [u]
        # start-up: u_1 .. u_ns by iterated Richardson extrapolation
        for m in range(1, ns + 1):
            u = self.richardson_step(u, (m - 1) * dt, dt, levels)
            us.append(u)
        if N <= ns:
            return u, dict(us=us if keep else None)
        # implicit Adams marching
        uhat = self.F(us[ns])
        W = {m: self.F(self.V(m * dt) * us[m]) for m in range(max(0, ns - (n - 2)), ns + 1)}
        traj = us if keep else None
        for step in range(ns + 1, N + 1):
            tn = step * dt
            B = self.prop(tn, dt) * uhat
            for j in range(1, n):
                B = B - 1j * dt * mu[j] * self.prop(tn, j * dt) * W[step - j]
            u = self.Finv(B) / (1.0 + 1j * mu[0] * dt * self.V(tn))
            W[step] = self.F(self.V(tn) * u)
            uhat = B - 1j * mu[0] * dt * W[step]
            W.pop(step - (n - 1), None)
            if keep:
                traj.append(u)
        return u, dict(us=traj, uhat=uhat)


def run_periodic(prob, nsteps: Optional[int] = None, keep: bool = False):
    """Convenience wrapper: oracle solution u(t_N) of a periodic problem."""
    return PeriodicOracle(prob).run(nsteps=nsteps, keep=keep)
