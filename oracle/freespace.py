"""FP64 oracle of the free-space complex-frequency scheme (Sections 3.3-3.4).

Test infrastructure only (see the package docstring).

Transforms are dense (no FFT), axis by axis:
  forward  (eq. (fzdft)):     fhat(zeta_k) = (2/M) sum_j exp(-i zeta_k x_j) f(x_j)
  inverse  (eq. (uciftdisc)): u(x_j) = (1/2pi) sum_k w_k exp(i zeta_k x_j) uhat(zeta_k)
on the grid x_j = -1 + 2 j / M and the Gamma nodes of ``quadrature.gamma_rule``.
The C-type block (nodes on Gamma_2) goes through the Chebyshev interpolant of
``chebyshev`` (Section 4.1) when the problem asks for it or when it has fewer
terms than Gamma_2 has nodes; in 2D the two axes' transforms compose, which
is the (C,E) and (C,C) forms of Section 4.2 with the sums in tensor order.
Propagator over [t_a, t_b] (Lemma 3.1, eq. (uhatzinteq)):
  P = exp(-i (zeta . zeta)(t_b - t_a) + i zeta . (phi(t_b) - phi(t_a))).
Order-2 sub-step (eqs. (uhatzfd), (utrapzfd)) carries (u, uhat):
  B = P (uhat - i d/2 What(t)),  u(t+d) = F^-1 B / (1 + i d/2 V(t+d)),
  uhat(t+d) = B - i d/2 What(t+d),  What = F(V u).
Start-up (Remark on high-order free-space schemes): iterated Richardson
extrapolation of both u and uhat; What_n = F(V(t_n) u_n) from the
extrapolated u_n.  Implicit Adams steps as in the periodic case with the
complex-frequency transforms.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from .adams import adams_coefficients, richardson_extrapolate
from .chebyshev import c_forward, c_inverse, choose_NT
from .potential import sampled_V
from .periodic import make_phi
from .quadrature import choose_H, gamma_rule

KAPPA = {8: 7}   # omitted regular nodes of the order-2p Alpert correction (Section 6, Example 2)


def free_grid(M: int) -> np.ndarray:
    return -1.0 + 2.0 * np.arange(M) / M


@dataclass
class FreeSpaceOracle:
    prob: object
    H: Optional[float] = None

    def __post_init__(self):
        p = self.prob
        assert p.domain == "free"
        self.d = p.dim
        self.shape = tuple(p.M)
        self.phi = make_phi(p)
        self.mu = [float(m) for m in adams_coefficients(p.order)]
        self.xs = [free_grid(m) for m in self.shape]
        # one contour parameter per axis (self.Hs); an H given by the caller
        # applies to every axis; self.H is that of axis 0
        self.Hs = self.default_H() if self.H is None else [float(self.H)] * self.d
        self.H = self.Hs[0]
        kappa = KAPPA[p.p]
        self.nodes = []
        self.G, self.Ginv = [], []
        for a in range(self.d):
            zeta, w, info = gamma_rule(self.shape[a], self.Hs[a], p.nu[a], p.p, kappa, p.q, p.panels)
            x = self.xs[a]
            self.nodes.append((zeta, w, info))
            self.G.append((2.0 / self.shape[a]) * np.exp(-1j * np.outer(zeta, x)))
            self.Ginv.append((w[None, :] / (2 * np.pi)) * np.exp(1j * np.outer(x, zeta)))
        # C-type transforms (Section 4.1): direct sums, or through the
        # Chebyshev interpolant of eqs. (expintrpm)/(expintrpp) with NT terms
        # per axis (prob.cheb: 0 automatic, NT < N_C; -1 direct; n > 0 forced)
        self.NT = [self._cheb_terms(a) for a in range(self.d)]
        Z = np.meshgrid(*[n[0] for n in self.nodes], indexing="ij")
        self.Z = Z
        self.Z2 = sum(z * z for z in Z)

    # --- parameter choice (Remark on H, Section 3.2) -------------------------
    def default_H(self):
        """The Remark's rule in each dimension, with that axis' quiver radius
        max_t |phi_a(t)| (the analysis bounds the growth per dimension)."""
        p = self.prob
        dt = p.dt
        cell = np.prod([2.0 / m for m in self.shape])
        normV, phimax = 0.0, np.zeros(self.d)
        for n in range(p.nsteps + 1):
            t = n * dt
            normV = max(normV, float(np.sqrt(np.sum(self.V(t) ** 2) * cell)))
            phimax = np.maximum(phimax, np.abs(np.asarray(self.phi(t), dtype=np.float64)))
        return [choose_H(p.eps, normV, float(phimax[a]), self.d) for a in range(self.d)]

    def _cheb_terms(self, a: int) -> int:
        mode = int(getattr(self.prob, "cheb", 0))
        NC = self.nodes[a][2]["NC"]
        if mode < 0:
            return 0
        if mode > 0:
            return mode
        NT = choose_NT(self.Hs[a])
        return NT if 0 < NT < NC else 0

    def _c_block(self, a: int) -> slice:
        info = self.nodes[a][2]
        return slice(info["NE"] + info["p"], info["NE"] + info["p"] + info["NC"])

    # --- transforms ----------------------------------------------------------
    def _fwd_axis(self, a: int, f: np.ndarray) -> np.ndarray:
        """Transform along axis 0 of f (grid of axis a) to the nodes of axis a;
        the C-type rows by the interpolant when it is on (Section 4.1)."""
        out = np.tensordot(self.G[a], f, axes=(1, 0))
        if self.NT[a]:
            c = self._c_block(a)
            tau_c = self.nodes[a][0][c].real
            out[c] = (2.0 / self.shape[a]) * c_forward(f, self.xs[a], tau_c, self.Hs[a], self.NT[a])
        return out

    def _inv_axis(self, a: int, g: np.ndarray) -> np.ndarray:
        if not self.NT[a]:
            return np.tensordot(self.Ginv[a], g, axes=(1, 0))
        c = self._c_block(a)
        keep = np.ones(g.shape[0], dtype=bool)
        keep[c] = False
        out = np.tensordot(self.Ginv[a][:, keep], g[keep], axes=(1, 0))
        zeta, w, _ = self.nodes[a]
        wc = (w[c] / (2 * np.pi)).reshape((-1,) + (1,) * (g.ndim - 1))
        return out + c_inverse(wc * g[c], self.xs[a], zeta[c].real, self.Hs[a], self.NT[a])

    def F(self, f: np.ndarray) -> np.ndarray:
        out = f
        for a in range(self.d):
            out = np.moveaxis(self._fwd_axis(a, np.moveaxis(out, a, 0)), 0, a)
        return out

    def Finv(self, g: np.ndarray) -> np.ndarray:
        out = g
        for a in range(self.d):
            out = np.moveaxis(self._inv_axis(a, np.moveaxis(out, a, 0)), 0, a)
        return out

    def evaluate(self, uhat: np.ndarray, points) -> np.ndarray:
        """u on the tensor grid points[0] x ... x points[d-1] from the modes
        uhat on Gamma_K: the discrete representation (eq. (uciftdisc)) taken at
        arbitrary real coordinates, which may lie outside [-1,1] (Remark on
        evaluation outside [-1,1]); the nodes are not refined."""
        out = np.asarray(uhat, dtype=np.complex128)
        for a in range(self.d):
            zeta, w, _ = self.nodes[a]
            x = np.asarray(points[a], dtype=np.float64)
            E = (w[None, :] / (2 * np.pi)) * np.exp(1j * np.outer(x, zeta))
            out = np.moveaxis(np.tensordot(E, np.moveaxis(out, a, 0), axes=(1, 0)), 0, a)
        return out

    # --- problem data ----------------------------------------------------------
    def V(self, t: float) -> np.ndarray:
        p = self.prob
        if getattr(p, "V_kind", "fields") == "sampled":
            return sampled_V(p.V_samples, t, p.dt)
        out = np.zeros(self.shape)
        for r, Vr in enumerate(p.V_fields):
            out = out + p.f(r, t) * Vr
        return out

    def prop(self, t_b: float, tau: float) -> np.ndarray:
        dphi = np.asarray(self.phi(t_b)) - np.asarray(self.phi(t_b - tau))
        arg = -self.Z2 * tau
        for a in range(self.d):
            arg = arg + self.Z[a] * dphi[a]
        return np.exp(1j * arg)

    # --- scheme --------------------------------------------------------------
    def trap_substep(self, u, uh, t, delta):
        W = self.F(self.V(t) * u)
        B = self.prop(t + delta, delta) * (uh - 0.5j * delta * W)
        un = self.Finv(B) / (1.0 + 0.5j * delta * self.V(t + delta))
        Wn = self.F(self.V(t + delta) * un)
        return un, B - 0.5j * delta * Wn

    def richardson_step(self, u, uh, t, dt, levels):
        Us, Uhs = [], []
        for l in range(levels):
            nsub = 2 ** l
            v, vh = u, uh
            for s in range(nsub):
                v, vh = self.trap_substep(v, vh, t + s * dt / nsub, dt / nsub)
            Us.append(v)
            Uhs.append(vh)
        return richardson_extrapolate(Us), richardson_extrapolate(Uhs)

    def run(self, nsteps: Optional[int] = None):
        p = self.prob
        dt = p.dt
        N = p.nsteps if nsteps is None else nsteps
        n = p.order
        ns = min(p.start_steps, N)
        mu = self.mu
        u = np.asarray(p.u0, dtype=np.complex128).copy()
        uh = self.F(u)
        us = [u]
        for m in range(1, ns + 1):
            u, uh = self.richardson_step(u, uh, (m - 1) * dt, dt, n // 2)
            us.append(u)
        if N <= ns:
            return u, dict(uhat=uh)
        W = {m: self.F(self.V(m * dt) * us[m]) for m in range(max(0, ns - (n - 2)), ns + 1)}
        for step in range(ns + 1, N + 1):
            tn = step * dt
            B = self.prop(tn, dt) * uh
            for j in range(1, n):
                B = B - 1j * dt * mu[j] * self.prop(tn, j * dt) * W[step - j]
            u = self.Finv(B) / (1.0 + 1j * mu[0] * dt * self.V(tn))
            W[step] = self.F(self.V(tn) * u)
            uh = B - 1j * mu[0] * dt * W[step]
            W.pop(step - (n - 1), None)
        return u, dict(uhat=uh)
