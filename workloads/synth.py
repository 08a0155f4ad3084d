"""Seeded synthetic problems shaped like the paper's 1D and 2D examples.

The paper's own examples start from Chebfun ground states that are not
available here, so seeded random Gaussian wells, pulses and wave packets of
the same form stand in for them (Section 6 uses Gaussian wells, the pulse of
eq. (apulse) and Gaussian initial data).  Every draw goes through
``numpy.random.default_rng(seed)`` (PCG64) in the order written below.

Grids (problem statement, Sections 2.1 and 3.3):
  periodic:   x_j = -pi + 2 pi j / M,  j = 0..M-1, on [-pi, pi)
  free space: x_j = -1 + 2 j / M,      j = 0..M-1, on [-1, 1)

A problem is V(x,t) = sum_r f_r(t) V_r(x) with real fields V_r, a vector
potential A(t) and initial data u0, marched to time T with step dt.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

TWO_PI = 2.0 * np.pi


def periodic_grid(M: int) -> np.ndarray:
    return -np.pi + TWO_PI * np.arange(M, dtype=np.float64) / M


def free_grid(M: int) -> np.ndarray:
    return -1.0 + 2.0 * np.arange(M, dtype=np.float64) / M


@dataclass
class Problem:
    """Plain description of one TDSE instance (no solver state)."""

    name: str
    dim: int
    domain: str                      # "periodic" | "free"
    M: Tuple[int, ...]
    T: float
    nsteps: int
    order: int
    u0: np.ndarray                   # complex128, shape M
    V_fields: List[np.ndarray]       # real float64 arrays, shape M
    f_kind: List[str]                # per field: "const" | "sin"
    f_params: List[Tuple[float, float]]  # per field: (amp, omega) for 1 + amp sin(omega t)
    A_kind: str = "none"             # "none" | "pulse_sin2" | "pulse_cos2" | "stepwise"
    A_params: Tuple[float, ...] = ()  # pulse: (E0, omega, Tp, dir_0, dir_1)
    A_steps: Optional[np.ndarray] = None  # stepwise: [nsteps, dim] values on each step
    precision: str = "fp64"          # "fp64" | "fp32split"
    n_start: Optional[int] = None    # default order - 2
    # free-space quadrature parameters
    eps: float = 1e-10
    p: int = 8
    q: int = 10
    panels: int = 1
    nu: Tuple[int, ...] = ()
    cheb: int = 0                    # C-type transforms: 0 automatic, -1 direct sums, n > 0 interpolant of n terms
    # potential kind: "fields" (V_fields with time factors) or "moving_well"
    # with V_well = (V0, beta, c_0[, c_1]) (Example 1 of Section 6)
    V_kind: str = "fields"
    V_well: Tuple[float, ...] = ()
    # V_kind "sampled": V(x, t_n) at the step times t_n = n dt, [nsteps + 1, *M]
    V_samples: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def dt(self) -> float:
        return self.T / self.nsteps

    @property
    def start_steps(self) -> int:
        return self.order - 2 if self.n_start is None else self.n_start

    def f(self, r: int, t: float) -> float:
        """Time factor f_r(t) of field r."""
        if self.f_kind[r] == "const":
            return 1.0
        amp, om = self.f_params[r]
        return 1.0 + amp * np.sin(om * t)

    def A(self, t: float) -> np.ndarray:
        """Vector potential A(t) in R^dim."""
        out = np.zeros(self.dim)
        if self.A_kind == "none":
            return out
        if self.A_kind in ("pulse_sin2", "pulse_cos2"):
            E0, om, Tp = self.A_params[:3]
            d = np.asarray(self.A_params[3:3 + self.dim], dtype=np.float64)
            carrier = np.sin(om * t) if self.A_kind == "pulse_sin2" else np.cos(om * t)
            return E0 * np.sin(np.pi * t / Tp) ** 2 * carrier * d
        if self.A_kind == "stepwise":
            dt = self.dt
            m = int(np.floor(t / dt + 1e-12))
            m = min(max(m, 0), self.nsteps - 1)
            return np.asarray(self.A_steps[m], dtype=np.float64).copy()
        raise ValueError(self.A_kind)

    def grid(self, axis: int) -> np.ndarray:
        g = periodic_grid if self.domain == "periodic" else free_grid
        return g(self.M[axis])

    def mesh(self) -> List[np.ndarray]:
        axes = [self.grid(a) for a in range(self.dim)]
        return list(np.meshgrid(*axes, indexing="ij"))


# --------------------------------------------------------------------------
# periodic workloads


def _periodized_gauss(X: Sequence[np.ndarray], c: Sequence[float], s: float, images: int) -> np.ndarray:
    """sum over image shifts m in {-images..images}^d of exp(-|x - c - 2 pi m|^2 / s^2)."""
    d = len(X)
    out = np.zeros(X[0].shape)
    rng_m = range(-images, images + 1)
    shifts = np.array(np.meshgrid(*([list(rng_m)] * d), indexing="ij")).reshape(d, -1).T
    for m in shifts:
        r2 = np.zeros(X[0].shape)
        for a in range(d):
            r2 += (X[a] - c[a] - TWO_PI * m[a]) ** 2
        out += np.exp(-r2 / (s * s))
    return out


def _normalize(u: np.ndarray, cell: float) -> np.ndarray:
    """Scale so that sum |u|^2 * cell = 1 (left-endpoint rule on the grid)."""
    return u / np.sqrt(np.sum(np.abs(u) ** 2) * cell)


def periodic_1d_256_problem(seed: int = 0, M: int = 256, T: float = 1.0, nsteps: int = 100, order: int = 8) -> Problem:
    """1D periodic well V = -a cos x, A = 0, Gaussian u0 (seed 0)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(1.0, 5.0)
    x0 = rng.uniform(-1.0, 1.0)
    sig = rng.uniform(0.3, 0.6)
    x = periodic_grid(M)
    V0 = -a * np.cos(x)
    u0 = _periodized_gauss([x], [x0], sig, images=2).astype(np.complex128)
    u0 = _normalize(u0, TWO_PI / M)
    return Problem(name="periodic-1d-256", dim=1, domain="periodic", M=(M,), T=T, nsteps=nsteps, order=order,
                   u0=u0, V_fields=[V0], f_kind=["const"], f_params=[(0.0, 0.0)],
                   meta=dict(a=a, x0=x0, sigma=sig))


def periodic_problem_from_seed(seed: int, dim: int, M: Sequence[int], T: float, nsteps: int,
                               order: int = 8, precision: str = "fp64", name: str = "",
                               A_kind: str = "pulse_sin2") -> Problem:
    """The 2D (or 1D and 3D analogue) periodic recipe: four Gaussian wells
    with a sinusoidal modulation, a sin^2-enveloped pulse along e1 and a
    Gaussian u0.

    Draw order: c_j ~ U[2,8] (4), p_j ~ U[-2,2]^d (4), s_j ~ U[0.3,0.8] (4),
    E0 ~ U[0.5,2], omega ~ U[5,15], x0 ~ U[-1,1]^d, sigma ~ U[0.3,0.6].
    """
    rng = np.random.default_rng(seed)
    cj = rng.uniform(2.0, 8.0, size=4)
    pj = rng.uniform(-2.0, 2.0, size=(4, dim))
    sj = rng.uniform(0.3, 0.8, size=4)
    E0 = rng.uniform(0.5, 2.0)
    om = rng.uniform(5.0, 15.0)
    x0 = rng.uniform(-1.0, 1.0, size=dim)
    sig = rng.uniform(0.3, 0.6)
    M = tuple(int(m) for m in M)
    axes = [periodic_grid(m) for m in M]
    X = list(np.meshgrid(*axes, indexing="ij"))
    images = 1 if dim >= 2 else 2
    V0 = np.zeros(M)
    for j in range(4):
        V0 -= cj[j] * _periodized_gauss(X, pj[j], sj[j], images)
    u0 = _periodized_gauss(X, x0, sig, images).astype(np.complex128)
    u0 = _normalize(u0, (TWO_PI) ** dim / np.prod(M))
    direction = (1.0, 0.0) if dim < 3 else (1.0, 0.0, 0.0)
    prob = Problem(name=name or f"periodic{dim}d_seed{seed}", dim=dim, domain="periodic", M=M, T=T,
                   nsteps=nsteps, order=order, u0=u0, V_fields=[V0], f_kind=["sin"],
                   f_params=[(0.1, om)], A_kind="pulse_sin2", A_params=(E0, om, T) + direction,
                   precision=precision,
                   meta=dict(c=cj, p=pj, s=sj, E0=E0, omega=om, x0=x0, sigma=sig))
    if A_kind == "stepwise":
        # piecewise-constant A on each step, sampled at the step midpoint
        dt = T / nsteps
        tm = (np.arange(nsteps) + 0.5) * dt
        steps = np.zeros((nsteps, dim))
        for m, t in enumerate(tm):
            steps[m] = prob.A(t)
        prob.A_kind = "stepwise"
        prob.A_steps = steps
        prob.A_params = ()
    elif A_kind == "none":
        prob.A_kind = "none"
        prob.A_params = ()
    return prob


def periodic_2d_512_problem(seed: int = 1, M: int = 512, T: float = 2.0, nsteps: int = 2000, order: int = 8) -> Problem:
    """2D periodic, 512 x 512, T = 2, 2000 steps, FP64 (seed 1)."""
    return periodic_problem_from_seed(seed, 2, (M, M), T, nsteps, order, name="periodic-2d-512")


def periodic_2d_1024_problem(seed: int = 3, M: int = 1024, T: float = 2.0, nsteps: int = 2000, order: int = 8,
               precision: str = "fp32split") -> Problem:
    """The 2D periodic recipe at 1024 x 1024 (seed 3), FP32-split by default."""
    return periodic_problem_from_seed(seed, 2, (M, M), T, nsteps, order, precision=precision, name="periodic-2d-1024")


def batch_64_problems(T: float = 2.0, nsteps: int = 500, order: int = 8, precision: str = "fp32split",
                count: int = 64, scale: int = 1) -> List[Problem]:
    """64 periodic instances of uneven sizes: i < 32 are 1D with M in
    {256, 512, 1024, 2048}; i >= 32 are 2D with M in {128, 256, 384, 512}^2.
    Instance i uses seed 4000 + i and a stepwise A (one sample per step).
    ``scale`` divides every size (for quick tests)."""
    out = []
    for i in range(count):
        if i < count // 2:
            m = [256, 512, 1024, 2048][i % 4] // scale
            prob = periodic_problem_from_seed(4000 + i, 1, (m,), T, nsteps, order, precision,
                                              name=f"batch-64[{i}]", A_kind="stepwise")
        else:
            m = [128, 256, 384, 512][i % 4] // scale
            prob = periodic_problem_from_seed(4000 + i, 2, (m, m), T, nsteps, order, precision,
                                              name=f"batch-64[{i}]", A_kind="stepwise")
        out.append(prob)
    return out


# --------------------------------------------------------------------------
# free-space workloads


def _bump(s: np.ndarray) -> np.ndarray:
    """C-infinity bump b(s) = exp(1 - 1/(1 - s^2)) for |s| < 1, else 0."""
    out = np.zeros_like(s)
    inside = np.abs(s) < 1.0
    out[inside] = np.exp(1.0 - 1.0 / (1.0 - s[inside] ** 2))
    return out


def moving_well_problem(c: Sequence[float] = (15.0,), M: Sequence[int] = (256,), T: float = 2.0 * np.pi / 15.0,
                        nsteps: int = 400, V0: float = 300.0, beta: float = 0.2, order: int = 8,
                        precision: str = "fp64", name: str = "moving-well") -> Problem:
    """Example 1 of Section 6 (a periodic Gaussian well of depth V0 and width
    beta moving with constant velocity c, A = 0), in 1D or 2D (len(M)).  In
    1D, u0 is the well's normalized ground state (periodic_well_ground_state),
    as in the paper.  The 2D variant is not in the paper; there u0 is a
    periodized Gaussian of the width of the harmonic approximation to the
    ground state, exp(-|x|^2 / (2 s^2)) with s = (2 V0 / beta^2)^(-1/4),
    centred on the well, normalized."""
    dim = len(M)
    if dim == 1:
        u0 = periodic_well_ground_state(V0, beta, int(M[0]))[1].astype(np.complex128)
    else:
        X = list(np.meshgrid(*[periodic_grid(m) for m in M], indexing="ij"))
        s_w = (2.0 * V0 / beta ** 2) ** -0.25
        u0 = _periodized_gauss(X, [0.0] * dim, np.sqrt(2.0) * s_w, images=2).astype(np.complex128)
        u0 = _normalize(u0, float(np.prod([TWO_PI / m for m in M])))
    c = tuple(float(x) for x in c)
    return Problem(name=name, dim=dim, domain="periodic", M=tuple(int(m) for m in M), T=T, nsteps=nsteps,
                   order=order, u0=u0, V_fields=[], f_kind=[], f_params=[], precision=precision,
                   V_kind="moving_well", V_well=(V0, beta) + c)


def free_problem_from_seed(seed: int, dim: int, M: Sequence[int], T: float, nsteps: int,
                           order: int = 8, eps: float = 1e-10, q: int = 10, panels: int = 1,
                           nu: Optional[Sequence[int]] = None, name: str = "",
                           A_kind: str = "pulse_sin2", E0_scale: float = 1.0) -> Problem:
    """Free-space recipe: the periodic draw order with the geometry rescaled
    into [-1,1]^d and every field windowed by a C-infinity bump.

    p_j ~ U[-0.5,0.5]^d, s_j ~ U[0.1,0.3], x0 ~ U[-0.3,0.3]^d, sigma ~ U[0.1,0.2].
    """
    rng = np.random.default_rng(seed)
    cj = rng.uniform(2.0, 8.0, size=4)
    pj = rng.uniform(-0.5, 0.5, size=(4, dim))
    sj = rng.uniform(0.1, 0.3, size=4)
    E0 = rng.uniform(0.5, 2.0) * E0_scale
    om = rng.uniform(5.0, 15.0)
    x0 = rng.uniform(-0.3, 0.3, size=dim)
    sig = rng.uniform(0.1, 0.2)
    M = tuple(int(m) for m in M)
    axes = [free_grid(m) for m in M]
    X = list(np.meshgrid(*axes, indexing="ij"))
    win = np.ones(M)
    for a in range(dim):
        win = win * _bump(X[a])
    V0 = np.zeros(M)
    for j in range(4):
        r2 = sum((X[a] - pj[j, a]) ** 2 for a in range(dim))
        V0 -= cj[j] * np.exp(-r2 / sj[j] ** 2)
    V0 = V0 * win
    r2 = sum((X[a] - x0[a]) ** 2 for a in range(dim))
    u0 = (win * np.exp(-r2 / sig ** 2)).astype(np.complex128)
    u0 = _normalize(u0, 2.0 ** dim / np.prod(M))
    if nu is None:
        nu = tuple(4 * m for m in M)
    prob = Problem(name=name or f"free{dim}d_seed{seed}", dim=dim, domain="free", M=M, T=T, nsteps=nsteps,
                   order=order, u0=u0, V_fields=[V0], f_kind=["sin"], f_params=[(0.1, om)],
                   A_kind="pulse_sin2", A_params=(E0, om, T, 1.0, 0.0) + (0.0,) * (dim - 2), eps=eps, q=q, panels=panels,
                   nu=tuple(int(v) for v in nu),
                   meta=dict(c=cj, p=pj, s=sj, E0=E0, omega=om, x0=x0, sigma=sig))
    if A_kind == "none":
        prob.A_kind = "none"
        prob.A_params = ()
    return prob


def sampled_potential_problem(base: Problem, depth: float = 6.0, width: float = 0.35, radius: float = 1.0,
                              omega: float = 20.0) -> Problem:
    """The problem `base` (periodic or free recipe) with its potential replaced
    by a general, non-separable V(x, t) given as samples at the step times
    t_n = n dt (V_kind "sampled"): the base fields with their time factors
    plus a well of varying depth and width circling the origin,
        W(x, t) = -depth (1 + 0.3 sin(omega t)) exp(-|x - c(t)|^2 / (2 b(t)^2)),
        c(t) = radius (cos(omega t / 2), sin(omega t / 2), 0)[:d],
        b(t) = width (1 + 0.2 cos(omega t)).
    In free space the geometry is scaled by 0.3 into [-1, 1]^d and the well is
    windowed by the recipe's bump; on the periodic box it is periodized."""
    import copy

    prob = copy.copy(base)
    dim, M = base.dim, base.M
    free = base.domain == "free"
    scale = 0.3 if free else 1.0
    g = free_grid if free else periodic_grid
    X = list(np.meshgrid(*[g(m) for m in M], indexing="ij"))
    win = np.ones(M)
    if free:
        for a in range(dim):
            win = win * _bump(X[a])
    samples = np.zeros((base.nsteps + 1,) + tuple(M))
    for n in range(base.nsteps + 1):
        t = n * base.dt
        v = np.zeros(M)
        for r, Vr in enumerate(base.V_fields):
            v = v + base.f(r, t) * Vr
        c = scale * radius * np.array([np.cos(0.5 * omega * t), np.sin(0.5 * omega * t), 0.0])[:dim]
        b = scale * width * (1.0 + 0.2 * np.cos(omega * t))
        d = depth * (1.0 + 0.3 * np.sin(omega * t))
        if free:
            w = np.exp(-sum((X[a] - c[a]) ** 2 for a in range(dim)) / (2.0 * b * b)) * win
        else:
            w = _periodized_gauss(X, c, np.sqrt(2.0) * b, images=1)
        samples[n] = v - d * w
    prob.V_kind = "sampled"
    prob.V_samples = samples
    prob.V_fields = []
    prob.f_kind = []
    prob.f_params = []
    prob.name = base.name + "-sampled"
    return prob


def sampled_2d_512_problem(nsteps: int = 500, T: float = 0.5) -> Problem:
    """The 512^2 periodic workload (seed 1) with a general, non-separable
    potential given as samples at the step times (sampled_potential_problem),
    500 steps to T = 0.5 (dt = 1e-3, as in the 2000-step run), FP64."""
    return sampled_potential_problem(periodic_problem_from_seed(1, 2, (512, 512), T, nsteps, name="sampled-2d-512"))


def periodic_3d_128_problem(seed: int = 50, M: int = 128, T: float = 0.5, nsteps: int = 500,
                            order: int = 8) -> Problem:
    """3D periodic, M^3 = 128^3 points (2,097,152 modes), the periodic recipe
    in three dimensions (seed 50): four modulated Gaussian wells, a sin^2
    pulse along e1, a Gaussian u0; 500 steps to T = 0.5, FP64."""
    return periodic_problem_from_seed(seed, 3, (M, M, M), T, nsteps, order, name="periodic-3d-128")


def free_2d_256_problem(seed: int = 2, M: int = 256, T: float = 1.0, nsteps: int = 1000, order: int = 8,
               nu: int = 2048) -> Problem:
    """2D free space, 256 x 256 physical points, eps = 1e-10, p = 8, q = 10,
    one Gauss panel per side, FFT size nu = 2048 per axis (seed 2)."""
    return free_problem_from_seed(seed, 2, (M, M), T, nsteps, order, nu=(nu, nu), name="free-2d-256")


def free_3d_32_problem(seed: int = 62, M: int = 32, T: float = 0.1, nsteps: int = 100, order: int = 8,
                       nu: int = 256) -> Problem:
    """3D free space, 32^3 physical points, eps = 1e-8, p = 8, q = 8, one
    Gauss panel per side, FFT size nu = 256 per axis (seed 62): the free-space
    recipe in three dimensions, about 1.8e7 complex-frequency modes."""
    return free_problem_from_seed(seed, 3, (M, M, M), T, nsteps, order, eps=1e-8, q=8, nu=(nu, nu, nu),
                                  name="free-3d-32")


def wavepacket(x, t: float, sigma: float):
    """The Gaussian wave packet of Section 6, Example 2 (eq. (wavepacket),
    k0 = 0), divided by sigma so that its L^2(R) norm is 1: the exact solution
    for V = 0, A = 0; with a field A the exact solution is u(x + phi(t), t)."""
    s = sigma ** 2 + 2j * t
    return sigma ** 1.5 / np.pi ** 0.25 / np.sqrt(s) * np.exp(-(np.asarray(x) / np.sqrt(2)) ** 2 / s) / sigma


def example2_long_time_problem(panels: int, cheb: int = 0, M: int = 128, nu: int = 1024, nsteps: int = 1000,
                               T: float = 1000.0) -> Problem:
    """Section 6, Example 2, long-time run: 1D free space, V = 0, u0 the wave
    packet with sigma = 0.1, A of eq. (apulse) with A0 = omega = 1 over
    [0, T], eps = 1e-14, p = 8, q = 16 and `panels` dyadic panels (n_r) per
    side of Gamma_2.  M and nu are this implementation's choice (the paper
    converges each parameter to about fifteen digits)."""
    x = free_grid(M)
    return Problem(name=f"ex2-long-nr{panels}", dim=1, domain="free", M=(M,), T=T, nsteps=nsteps, order=8,
                   u0=wavepacket(x, 0.0, 0.1).astype(complex), V_fields=[np.zeros(M)], f_kind=["const"],
                   f_params=[(0.0, 0.0)], A_kind="pulse_cos2", A_params=(1.0, 1.0, T, 1.0),
                   eps=1e-14, q=16, panels=panels, nu=(nu,), cheb=cheb)


def gaussian_well_ground_state(V0: float, beta: float, L: float = 2.0, n: int = 512):
    """Ground state of -u'' + V u = E u for the well V(x) = -V0 exp(-x^2/(2 beta^2))
    of Section 6, Examples 3 and 4 (1D), which the paper computes with
    Chebfun.  Fourier pseudo-spectral discretization on the periodic box
    [-L, L) with n points (the state is below 1e-15 at |x| = L for the wells
    used here), dense symmetric eigensolve.  Returns (E, evaluate) where
    evaluate(x) is the L^2(R)-normalized, real, positive state at points x
    in [-L, L) by trigonometric interpolation."""
    x = -L + 2.0 * L * np.arange(n) / n
    k = np.fft.fftfreq(n, d=2.0 * L / n) * 2.0 * np.pi
    F = np.fft.fft(np.eye(n), axis=0)
    D2 = np.real(np.fft.ifft(-(k ** 2)[:, None] * F, axis=0))
    Hm = -D2 + np.diag(-V0 * np.exp(-x ** 2 / (2.0 * beta ** 2)))
    Hm = 0.5 * (Hm + Hm.T)
    E, vecs = np.linalg.eigh(Hm)
    g = vecs[:, 0]
    g = g / np.sqrt(np.sum(g ** 2) * (2.0 * L / n))
    if g[n // 2] < 0:
        g = -g
    c = np.fft.fft(g) / n

    def evaluate(pts):
        pts = np.asarray(pts, dtype=np.float64)
        return np.real(np.exp(1j * np.outer(pts + L, k)) @ c)

    return float(E[0]), evaluate


def ionization_1d_problem(omega: float, A0: float = 100.0, V0: float = 1400.0, beta: float = 0.1, M: int = 100,
                          nu: int = 1024, T: float = 0.5, nsteps: int = 4000, eps: float = 1e-10, q: int = 10,
                          panels: int = 1, order: int = 8) -> Problem:
    """Section 6, Example 3: ionization from the ground state of the Gaussian
    well V = -V0 exp(-x^2/(2 beta^2)) (V0 = 1400, beta = 0.1) by the pulse
    A = A0 sin^2(pi t/T) cos(omega t) of eq. (apulse), in free space on
    M = 100 points, eps = 1e-10, q = 10, T = 0.5."""
    x = free_grid(M)
    E, gs = gaussian_well_ground_state(V0, beta)
    V = -V0 * np.exp(-x ** 2 / (2.0 * beta ** 2))
    prob = Problem(name=f"ionization-1d-omega{omega:g}", dim=1, domain="free", M=(M,), T=T, nsteps=nsteps,
                   order=order, u0=gs(x).astype(np.complex128), V_fields=[V], f_kind=["const"], f_params=[(0.0, 0.0)],
                   A_kind="pulse_cos2", A_params=(A0, omega, T, 1.0), eps=eps, q=q, panels=panels, nu=(nu,))
    prob.ground_energy = E
    return prob


def gaussian_well_ground_state_2d(V0: float, beta: float, L: float = 2.0, n: int = 200):
    """Ground state of -Lap u + V u = E u for the radial well
    V(x, y) = -V0 exp(-(x^2 + y^2)/(2 beta^2)) of Section 6, Example 4, which
    the paper computes in polar coordinates with Chebfun.  Fourier
    pseudo-spectral discretization on the periodic box [-L, L)^2 with n
    points per axis; the lowest eigenpair by Lanczos iteration (scipy's
    eigsh) on the FFT-applied operator.  Returns (E, evaluate) where
    evaluate(xs, ys) is the L^2-normalized, real, positive state on the
    tensor grid xs x ys by trigonometric interpolation."""
    from scipy.sparse.linalg import LinearOperator, eigsh

    x = -L + 2.0 * L * np.arange(n) / n
    k = np.fft.fftfreq(n, d=2.0 * L / n) * 2.0 * np.pi
    K2 = k[:, None] ** 2 + k[None, :] ** 2
    X, Y = np.meshgrid(x, x, indexing="ij")
    V = -V0 * np.exp(-(X ** 2 + Y ** 2) / (2.0 * beta ** 2))

    def apply(v):
        u = v.reshape(n, n)
        return (np.real(np.fft.ifft2(K2 * np.fft.fft2(u))) + V * u).ravel()

    op = LinearOperator((n * n, n * n), matvec=apply, dtype=np.float64)
    start = np.exp(-(X ** 2 + Y ** 2) / (2.0 * beta ** 2)).ravel()
    E, vec = eigsh(op, k=1, which="SA", v0=start, tol=1e-13, maxiter=20000)
    g = vec[:, 0].reshape(n, n)
    g = g / np.sqrt(np.sum(g ** 2) * (2.0 * L / n) ** 2)
    if g[n // 2, n // 2] < 0:
        g = -g
    c = np.fft.fft2(g) / (n * n)

    def evaluate(xs, ys):
        Ex = np.exp(1j * np.outer(np.asarray(xs, dtype=np.float64) + L, k))
        Ey = np.exp(1j * np.outer(np.asarray(ys, dtype=np.float64) + L, k))
        return np.real(Ex @ c @ Ey.T)

    return float(E[0]), evaluate


def ionization_2d_problem(omega: float, A0: float = 100.0, V0: float = 1400.0, beta: float = 0.1, M: int = 100,
                          nu: Sequence[int] = (1024, 512), T: float = 0.5, nsteps: int = 8000, eps: float = 1e-10,
                          q: int = 10, panels: int = 1, order: int = 8) -> Problem:
    """Section 6, Example 4: the 2D analogue of Example 3, with the field
    (A_1(t), 0) along x, on M x M = 100 x 100 points, q = 10, T = 0.5.  The
    paper's higher-accuracy runs use eps = 1e-10, h1 ~ 0.3, h2 ~ 0.5 (here
    nu = (1024, 512): h = pi M / nu = 0.31, 0.61); its lower-accuracy runs
    eps = 1e-5, h1 ~ 1.4, h2 ~ 1.6 (here nu = (256, 256): h = 1.23)."""
    x = free_grid(M)
    E, gs = gaussian_well_ground_state_2d(V0, beta)
    X, Y = np.meshgrid(x, x, indexing="ij")
    V = -V0 * np.exp(-(X ** 2 + Y ** 2) / (2.0 * beta ** 2))
    prob = Problem(name=f"ionization-2d-omega{omega:g}", dim=2, domain="free", M=(M, M), T=T, nsteps=nsteps,
                   order=order, u0=gs(x, x).astype(np.complex128), V_fields=[V], f_kind=["const"],
                   f_params=[(0.0, 0.0)], A_kind="pulse_cos2", A_params=(A0, omega, T, 1.0, 0.0), eps=eps, q=q,
                   panels=panels, nu=tuple(nu))
    prob.ground_energy = E
    return prob


def periodic_well_ground_state(V0: float, beta: float, M: int, images: int = 2):
    """Ground state of -u'' + V u = E u on the periodic interval [-pi, pi) for
    the periodic Gaussian well V(x) = -V0 sum_k exp(-(x - 2 pi k)^2/(2 beta^2))
    of Section 6, Example 1 (the well at rest), which the paper computes with
    Chebfun: Fourier pseudo-spectral discretization on the M-point periodic
    grid, dense symmetric eigensolve.  Returns (E, u) with u on the grid,
    real, positive at the well's centre and normalized in L^2([-pi, pi))."""
    x = periodic_grid(M)
    k = np.fft.fftfreq(M, d=TWO_PI / M) * TWO_PI
    F = np.fft.fft(np.eye(M), axis=0)
    D2 = np.real(np.fft.ifft(-(k ** 2)[:, None] * F, axis=0))
    V = -V0 * sum(np.exp(-(x - TWO_PI * j) ** 2 / (2.0 * beta ** 2)) for j in range(-images, images + 1))
    Hm = -D2 + np.diag(V)
    Hm = 0.5 * (Hm + Hm.T)
    E, vecs = np.linalg.eigh(Hm)
    g = vecs[:, 0]
    g = g / np.sqrt(np.sum(g ** 2) * TWO_PI / M)
    if g[np.argmin(np.abs(x))] < 0:
        g = -g
    return float(E[0]), g
