"""Quadrature on the contour Gamma (Section 3.4) for the free-space oracle.

Test infrastructure only (see the package docstring).

* ``alpert_endpoint_rule(p, kappa)``: Alpert's hybrid Gauss-trapezoidal
  end correction (Section 3.4; the node table itself is only cited there).
  The rule h [sum_k w_k f(x_k h) + sum_{j>=kappa} f(j h)] reproduces the
  integral of f over [0, inf) to high order when it is exact, in the
  zeta-regularised sense, on the monomials x^m, m < 2p:
      sum_k w_k x_k^m = -zeta(-m, kappa) = B_{m+1}(kappa) / (m + 1)
  (B_n the Bernoulli polynomials).  The x_k are the roots of the degree-p
  monic orthogonal polynomial of these moments (exact rational Hankel solve),
  refined in mpmath; the w_k solve the first p moment equations.
* ``gauss_legendre(q)``: numpy's Gauss-Legendre rule (a library primitive).
* ``gamma_rule(...)``: the five node sets E1, A1, C, A3, E3 of Section 3.4 in
  that order, with these readings of the section: E-nodes
  H + kappa h + (k-1) h - iH, k = 1..N_E; panels per side given directly;
  Gamma_2 nodes (1 - i) tau.
* ``choose_H``: the rule of the Remark on the choice of H (Section 3.2),
  H = log(eps / ((1 + ||V||_{2,inf}) eps_m)) / (2 d (1 + phi_max)).
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import comb
from typing import List, Tuple

import mpmath as mp
import numpy as np

from .adams import _solve_exact

EPS_MACHINE = 2.0 ** -52


def _bernoulli_numbers(n: int) -> List[Fraction]:
    """B_0..B_n (B_1 = -1/2) from sum_{k<=m} C(m+1, k) B_k = 0."""
    B = [Fraction(0)] * (n + 1)
    B[0] = Fraction(1)
    for m in range(1, n + 1):
        B[m] = -sum(comb(m + 1, k) * B[k] for k in range(m)) / (m + 1)
    return B


def _bernoulli_poly(n: int, x: int, B: List[Fraction]) -> Fraction:
    return sum(comb(n, k) * B[k] * Fraction(x) ** (n - k) for k in range(n + 1))


def alpert_moments(p: int, kappa: int) -> List[Fraction]:
    """c_m = B_{m+1}(kappa) / (m + 1), m = 0..2p-1 (exact)."""
    B = _bernoulli_numbers(2 * p + 1)
    return [_bernoulli_poly(m + 1, kappa, B) / (m + 1) for m in range(2 * p)]


@lru_cache(maxsize=8)
def alpert_endpoint_rule(p: int = 8, kappa: int = 7, dps: int = 60) -> Tuple[Tuple, Tuple]:
    """Nodes x_k (in units of h from the endpoint) and weights w_k, as mpf."""
    c = alpert_moments(p, kappa)
    # monic orthogonal polynomial x^p + sum_i a_i x^i: sum_i a_i c_{i+j} = -c_{p+j}
    A = [[c[i + j] for i in range(p)] for j in range(p)]
    a = _solve_exact(A, [-c[p + j] for j in range(p)])
    with mp.workdps(dps):
        coeffs = [mp.mpf(1)] + [mp.mpf(a[i].numerator) / a[i].denominator for i in reversed(range(p))]
        roots = sorted(mp.re(r) for r in mp.polyroots(coeffs, maxsteps=400, extraprec=4 * dps))
        V = mp.matrix(p, p)
        for m in range(p):
            for k in range(p):
                V[m, k] = roots[k] ** m
        w = mp.lu_solve(V, mp.matrix([mp.mpf(c[m].numerator) / c[m].denominator for m in range(p)]))
        return tuple(roots), tuple(w[k] for k in range(p))


def alpert_float(p: int = 8, kappa: int = 7) -> Tuple[np.ndarray, np.ndarray]:
    x, w = alpert_endpoint_rule(p, kappa)
    return np.array([float(v) for v in x]), np.array([float(v) for v in w])


def gauss_legendre(q: int) -> Tuple[np.ndarray, np.ndarray]:
    return np.polynomial.legendre.leggauss(q)


def choose_H(eps: float, normV: float, phimax: float, d: int) -> float:
    """Remark on the choice of H (Section 3.2)."""
    return float(np.log(eps / ((1.0 + normV) * EPS_MACHINE)) / (2.0 * d * (1.0 + phimax)))


def gamma_rule(M: int, H: float, nu: int, p: int = 8, kappa: int = 7, q: int = 10, panels: int = 1):
    """Nodes zeta (complex) and weights w (complex) on Gamma_K, ordered
    (E1, A1, C, A3, E3); returns (zeta, w, info).

    FFT-compatible parameters (Section 4.1): K = H + pi M / 2 and
    nu = 2 (N_E + 2 kappa - 1), so h = (K - H)/(N_E + 2 kappa - 1) = pi M / nu.
    """
    NE = nu // 2 - 2 * kappa + 1
    if NE <= M // 2:
        raise ValueError("need N_E > M/2 (Section 4)")
    h = np.pi * M / nu
    K = H + np.pi * M / 2
    xa, wa = alpert_float(p, kappa)
    # Gamma_3: equispaced part and Alpert end correction at tau = H
    tauE3 = H + kappa * h + np.arange(NE) * h
    zE3 = tauE3 - 1j * H
    wE3 = np.full(NE, h, dtype=np.complex128)
    zA3 = H + xa * h - 1j * H
    wA3 = (h * wa).astype(np.complex128)
    # Gamma_2: dyadic composite Gauss-Legendre panels toward 0 on [-H, H]
    gx, gw = gauss_legendre(q)
    edges = [0.0] + [H / 2 ** (panels - k) for k in range(1, panels + 1)]
    taus, wts = [], []
    for k in range(1, panels + 1):
        a, b = edges[k - 1], edges[k]
        taus.append(0.5 * (b - a) * gx + 0.5 * (a + b))
        wts.append(0.5 * (b - a) * gw)
    tpos = np.concatenate(taus)
    wpos = np.concatenate(wts)
    tau_c = np.concatenate([-tpos[::-1], tpos])
    w_c = np.concatenate([wpos[::-1], wpos])
    zC = (1 - 1j) * tau_c
    wC = (1 - 1j) * w_c
    # Gamma_1 by symmetry
    zA1 = -zA3[::-1]
    wA1 = wA3[::-1].copy()
    zE1 = -zE3[::-1]
    wE1 = wE3[::-1].copy()
    zeta = np.concatenate([zE1, zA1, zC, zA3, zE3])
    w = np.concatenate([wE1, wA1, wC, wA3, wE3])
    info = dict(NE=NE, h=h, K=K, H=H, NC=len(zC), N=len(zeta), p=p, kappa=kappa)
    return zeta, w, info
