"""Chebyshev-interpolated C-type transforms on Gamma_2 (Section 4.1).

Test infrastructure only (see the package docstring).

On Gamma_2 the nodes are zeta = gamma(tau) = (1 - i) tau, tau in [-H, H], so
the kernels of the C-type transforms are entire functions of tau for x in
[-1, 1]:
  forward   exp(-i zeta x) = exp(-tau x) exp(-i tau x)
              ~ sum_{l < NT} lambda_{l,j} T_l^H(tau)                 eq. (expintrpm)
  inverse   exp(+i zeta x) = exp(+tau x) exp(+i tau x)
              ~ sum_{l < NT} rho_{j,l} T_l^H(tau)                    eq. (expintrpp)
where T_l^H(tau) = T_l(tau / H).  With these,
  fhat^C_k = sum_l T_l^H(tau_k) sum_j lambda_{l,j} f_j                (1D forward)
  f^C_j    = sum_l rho_{j,l} sum_k T_l^H(tau_k) fhat^C_k              (1D inverse)
at cost O(M NT + NT NC) instead of O(M NC).

Readings (the paper fixes the degree only as O(H) and names no nodes):
  * the interpolant takes its values at the NT Chebyshev points of the first
    kind, s_m = cos(pi (m + 1/2) / NT), and its coefficients are the discrete
    cosine sums a_l = (c_l / NT) sum_m g(H s_m) T_l(s_m), c_0 = 1, c_l = 2;
  * NT is the smallest count for which the interpolation error bound
    4 sum_{l >= NT} I_l(sqrt(2) H) (the Chebyshev coefficients of exp(z s)
    are 2 I_l(z), |I_l(z)| <= I_l(|z|), |z| <= sqrt(2) H for |x| <= 1, and
    interpolation at most doubles the tail) falls below 2^-52, so the
    interpolant is exact to rounding and the scheme's accuracy is that of the
    direct sums;
  * "direct summation for small N_C": the interpolation is used when
    NT < N_C (automatic choice), or when the problem asks for it.
"""
from __future__ import annotations

import numpy as np
from scipy.special import iv

TOL = 2.0 ** -52
NT_MAX = 64


def cheb_points(NT: int) -> np.ndarray:
    """Chebyshev points of the first kind on [-1, 1]."""
    return np.cos(np.pi * (np.arange(NT) + 0.5) / NT)


def cheb_T(NT: int, s: np.ndarray) -> np.ndarray:
    """[len(s), NT] matrix of T_l(s_k) (l < NT), |s| <= 1."""
    return np.polynomial.chebyshev.chebvander(np.asarray(s, dtype=np.float64), NT - 1)


def choose_NT(H: float) -> int:
    """Smallest NT with 4 sum_{l >= NT} I_l(sqrt(2) H) <= 2^-52 (see the reading
    above); 0 if that takes more than NT_MAX terms (direct sums then)."""
    r = np.sqrt(2.0) * H
    for n in range(2, NT_MAX + 1):
        tail = 4.0 * sum(iv(l, r) for l in range(n, n + 60))
        if tail <= TOL:
            return n
    return 0


def interp_coeffs(values: np.ndarray) -> np.ndarray:
    """Coefficients a_l (axis 0) of the interpolant through values[m] = g(H s_m)
    (axis 0 indexed by m)."""
    NT = values.shape[0]
    Ts = cheb_T(NT, cheb_points(NT))          # [m, l]
    c = np.full(NT, 2.0 / NT)
    c[0] = 1.0 / NT
    return c[:, None] * (Ts.T @ values) if values.ndim == 2 else c * (Ts.T @ values)


def lambda_matrix(x: np.ndarray, H: float, NT: int) -> np.ndarray:
    """lambda_{l,j}: coefficients of tau -> exp(-tau x_j) exp(-i tau x_j) on [-H, H]
    (eq. (expintrpm)); shape [NT, M]."""
    tau = H * cheb_points(NT)
    g = np.exp(-(1.0 + 1.0j) * np.outer(tau, x))     # [m, j]
    return interp_coeffs(g)


def rho_matrix(x: np.ndarray, H: float, NT: int) -> np.ndarray:
    """rho_{j,l}: coefficients of tau -> exp(tau x_j) exp(i tau x_j) on [-H, H]
    (eq. (expintrpp)); shape [M, NT]."""
    tau = H * cheb_points(NT)
    g = np.exp((1.0 + 1.0j) * np.outer(tau, x))      # [m, j]
    return interp_coeffs(g).T


def c_forward(f: np.ndarray, x: np.ndarray, tau_c: np.ndarray, H: float, NT: int) -> np.ndarray:
    """fhat^C_k ~ sum_l T_l^H(tau_k) sum_j lambda_{l,j} f_j (axis 0 of f), the
    C-type forward transform of eq. (fhatCsum) through the interpolant."""
    g = np.tensordot(lambda_matrix(x, H, NT), f, axes=(1, 0))     # [l, ...]
    return np.tensordot(cheb_T(NT, tau_c / H), g, axes=(1, 0))      # [k, ...]


def c_inverse(chat: np.ndarray, x: np.ndarray, tau_c: np.ndarray, H: float, NT: int) -> np.ndarray:
    """f^C_j ~ sum_l rho_{j,l} sum_k T_l^H(tau_k) chat_k (axis 0 of chat), the
    C-type part of the inverse transform through the interpolant."""
    s = np.tensordot(cheb_T(NT, tau_c / H).T, chat, axes=(1, 0))    # [l, ...]
    return np.tensordot(rho_matrix(x, H, NT), s, axes=(1, 0))       # [j, ...]
