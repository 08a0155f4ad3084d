"""Potentials given as samples in time: V(x, t_n) at the step times
t_n = n dt, n = 0..N, evaluated between samples by Lagrange interpolation.

Test infrastructure only (see the package docstring).

The scheme (Sections 2.2 and 3.3) needs V at the step times (implicit Adams
steps) and at the sub-step times t_{m-1} + k dt / 2^l of the Richardson
start-up.  The paper takes V(x, t) as a given function; for a potential known
only through samples the reading here is: at a step time the sample itself;
elsewhere the degree-7 Lagrange interpolant through the eight samples
t_{n0} .. t_{n0+7}, n0 = min(max(floor(t/dt) - 3, 0), N - 7) (all N + 1
samples when N < 7), whose error O(dt^8) matches the eighth-order scheme.
A time within 1e-9 dt of a step time is that step time.
"""
from __future__ import annotations

import numpy as np

DEG = 7


def window(t: float, dt: float, N: int):
    """(n0, weights): the samples n0 .. n0 + len(weights) - 1 and their Lagrange
    weights at time t."""
    s = t / dt
    n = int(np.round(s))
    if abs(s - n) < 1e-9 and 0 <= n <= N:
        return n, np.ones(1)
    count = min(DEG + 1, N + 1)
    n0 = min(max(int(np.floor(s)) - (count // 2 - 1), 0), N + 1 - count)
    nodes = n0 + np.arange(count)
    w = np.ones(count)
    for i in range(count):
        for j in range(count):
            if j != i:
                w[i] *= (s - nodes[j]) / (nodes[i] - nodes[j])
    return n0, w


def sampled_V(samples: np.ndarray, t: float, dt: float) -> np.ndarray:
    """V(., t) from samples [N + 1, *grid] at the step times."""
    N = samples.shape[0] - 1
    n0, w = window(t, dt, N)
    out = np.zeros(samples.shape[1:])
    for i, wi in enumerate(w):
        out = out + wi * samples[n0 + i]
    return out
