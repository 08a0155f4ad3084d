"""Exact implicit Adams coefficients and Richardson extrapolation.

Test infrastructure only (see the package docstring).

* ``adams_coefficients(n)`` follows Section 2.2 ("Higher-order time
  discretizations"): the update integral over [t - dt, t] is replaced by the
  integral of the degree n-1 interpolant through t - j dt, j = 0..n-1.  The
  weights mu_j come from the Vandermonde system stated there, solved here in
  exact rational arithmetic.  Table 1 prints the n = 8 result.
* ``richardson_extrapolate`` follows the iterated Richardson tableau of
  Section 2.2: level m combines neighbours with (4^m U_hi - U_lo)/(4^m - 1),
  which removes the dt^(2m) error term of the trapezoid rule.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence


def _solve_exact(A: List[List[Fraction]], b: List[Fraction]) -> List[Fraction]:
    """Gaussian elimination with exact fractions (no pivoting issue: exact)."""
    n = len(b)
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [M[r][k] - f * M[c][k] for k in range(n + 1)]
    return [M[i][n] / M[i][i] for i in range(n)]


def adams_coefficients(n: int) -> List[Fraction]:
    """mu_0..mu_{n-1} of the n-th order implicit Adams rule.

    In units of dt with s = 0 at the new time level, the nodes are s = -j and
    int_{-1}^{0} s^m ds = (-1)^m / (m + 1) must be reproduced for m < n:
        sum_j mu_j (-j)^m = (-1)^m / (m + 1).
    """
    if n < 1:
        raise ValueError("order must be >= 1")
    A = [[Fraction((-j) ** m) if not (j == 0 and m == 0) else Fraction(1) for j in range(n)] for m in range(n)]
    b = [Fraction((-1) ** m, m + 1) for m in range(n)]
    return _solve_exact(A, b)


def richardson_extrapolate(U: Sequence, ratio: int = 2):
    """Iterated Richardson extrapolation of the trapezoid results.

    ``U[l]`` is the order-2 result with 2^l sub-steps (l = 0..L-1).  Level m
    forms U_m^{(l)} = (4^m U_{m-1}^{(l+1)} - U_{m-1}^{(l)}) / (4^m - 1);
    the single entry left at level L-1 is returned.
    """
    col = list(U)
    m = 1
    while len(col) > 1:
        f = (ratio * ratio) ** m
        col = [(f * col[l + 1] - col[l]) / (f - 1) for l in range(len(col) - 1)]
        m += 1
    return col[0]


def richardson_weights_exact(L: int, ratio: int = 2) -> List[Fraction]:
    """Weights r_l with richardson_extrapolate(U) = sum_l r_l U[l] (the tableau
    is linear in its inputs), from unit inputs in exact arithmetic."""
    return [richardson_extrapolate([Fraction(int(i == l)) for i in range(L)], ratio) for l in range(L)]
