"""Pins of the oracle's Chebyshev-interpolated C-type transforms (Section 4.1,
eqs. (expintrpm) and (expintrpp); Section 4.2's (C,E) and (C,C) forms) against
closed forms, the direct sums that define the transforms (eqs. (fhatCsum),
(dft2d)) and the long-time wave packet of Section 6, Example 2."""
import numpy as np
import pytest
from scipy.special import iv

from oracle.chebyshev import c_forward, c_inverse, cheb_T, choose_NT, interp_coeffs, lambda_matrix, rho_matrix
from oracle.freespace import FreeSpaceOracle, free_grid
from oracle.quadrature import gamma_rule
from workloads.synth import example2_long_time_problem, free_problem_from_seed, wavepacket


def test_coefficients_of_a_chebyshev_polynomial():
    # values of T_5 at the interpolation points give the unit coefficient vector
    NT = 12
    s = np.cos(np.pi * (np.arange(NT) + 0.5) / NT)
    a = interp_coeffs(np.cos(5 * np.arccos(s)))
    assert np.max(np.abs(a - np.eye(NT)[5])) < 1e-15


@pytest.mark.parametrize("H", [0.7, 1.6, 2.9])
def test_lambda_and_rho_are_bessel_coefficients(H):
    # exp(z s) = I_0(z) + 2 sum_l I_l(z) T_l(s) (Jacobi-Anger, modified form):
    # with z = -(1+i) H x the coefficients of eq. (expintrpm) are c_l I_l(z),
    # with z = (1+i) H x those of eq. (expintrpp)
    x = free_grid(64)
    NT = choose_NT(H)
    c = np.full(NT, 2.0)
    c[0] = 1.0
    l = np.arange(NT)[:, None]
    lam_ex = c[:, None] * iv(l, -(1 + 1j) * H * x[None, :])
    rho_ex = (c[:, None] * iv(l, (1 + 1j) * H * x[None, :])).T
    scale = np.exp(H)
    assert np.max(np.abs(lambda_matrix(x, H, NT) - lam_ex)) < 1e-14 * scale
    assert np.max(np.abs(rho_matrix(x, H, NT) - rho_ex)) < 1e-14 * scale


@pytest.mark.parametrize("H", [0.5, 0.95, 2.4, 3.0, 5.0])
def test_terms_rule_makes_the_interpolant_exact_to_rounding(H):
    x = np.linspace(-1, 1, 129)
    tau = np.linspace(-H, H, 1001)
    NT = choose_NT(H)
    ex = np.exp(-(1 + 1j) * np.outer(tau, x))
    err = np.max(np.abs(cheb_T(NT, tau / H) @ lambda_matrix(x, H, NT) - ex))
    assert err < 5e-14 * np.exp(H), (NT, err)
    if H < 1.0:
        # and it is not oversized: four fewer terms leave a visible error
        err4 = np.max(np.abs(cheb_T(NT - 4, tau / H) @ lambda_matrix(x, H, NT - 4) - ex))
        assert err4 > 30 * err


def _c_nodes(M, H, q, panels):
    zeta, w, info = gamma_rule(M, H, 4 * M, 8, 7, q, panels)
    c = slice(info["NE"] + info["p"], info["NE"] + info["p"] + info["NC"])
    return zeta[c], w[c]


@pytest.mark.parametrize("q,panels,H", [(16, 1, 0.95), (16, 3, 2.4), (16, 5, 3.0), (10, 4, 1.7)])
def test_c_type_transforms_match_the_direct_sums(q, panels, H):
    rng = np.random.default_rng(q * 10 + panels)
    M = 96
    x = free_grid(M)
    zc, wc = _c_nodes(M, H, q, panels)
    NT = choose_NT(H)
    f = rng.standard_normal((M, 3)) + 1j * rng.standard_normal((M, 3))
    direct = np.exp(-1j * np.outer(zc, x)) @ f                                   # eq. (fhatCsum)
    cheb = c_forward(f, x, zc.real, H, NT)
    assert np.linalg.norm(cheb - direct) < 1e-13 * np.linalg.norm(direct) * np.exp(H)
    g = rng.standard_normal((len(zc), 2)) + 1j * rng.standard_normal((len(zc), 2))
    direct_i = np.exp(1j * np.outer(x, zc)) @ g                                   # C part of the inverse
    cheb_i = c_inverse(g, x, zc.real, H, NT)
    assert np.linalg.norm(cheb_i - direct_i) < 1e-13 * np.linalg.norm(direct_i) * np.exp(H)


def test_2d_ce_and_cc_blocks_match_the_2d_dft():
    # Section 4.2: the (C,E) and (C,C) subsets of the forward DFT of eq.
    # (dft2d), through the interpolant, against the direct double sum, and
    # the (C,E1) subset in the rearranged order the paper writes it in
    M1, M2 = 32, 48
    prob = free_problem_from_seed(41, 2, (M1, M2), 0.05, 4, nu=(256, 256), eps=1e-10, q=16, panels=3)
    prob.cheb = 0
    orc = FreeSpaceOracle(prob)
    assert all(orc.NT), orc.NT
    rng = np.random.default_rng(3)
    f = rng.standard_normal((M1, M2)) + 1j * rng.standard_normal((M1, M2))
    fh = orc.F(f)
    (z1, _, i1), (z2, _, i2) = orc.nodes
    x, y = orc.xs
    direct = (2.0 / M1) * (2.0 / M2) * np.exp(-1j * np.outer(z1, x)) @ f @ np.exp(-1j * np.outer(y, z2))
    c1, c2 = orc._c_block(0), orc._c_block(1)
    e1 = slice(0, i2["NE"])
    e3 = slice(i2["N"] - i2["NE"], i2["N"])
    for blk in [(c1, e1), (c1, e3), (c1, c2), (slice(0, i1["NE"]), c2)]:
        d = direct[blk]
        assert np.linalg.norm(fh[blk] - d) < 1e-12 * np.linalg.norm(d), blk
    # (C,E1) as sum_l T_l(tau_k1) sum_j2 e^{-i xi y}(e^{H2 y} sum_j1 lambda_{l,j1} f)
    H1, H2 = orc.Hs
    NT = orc.NT[0]
    lam = lambda_matrix(x, H1, NT)
    xi = z2[e1].real
    inner = lam @ f                                                      # [l, j2]
    mid = (inner * np.exp(H2 * y)[None, :]) @ np.exp(-1j * np.outer(y, xi))   # [l, k2]
    ce1 = (2.0 / M1) * (2.0 / M2) * cheb_T(NT, z1[c1].real / H1) @ mid
    assert np.linalg.norm(ce1 - direct[c1, e1]) < 1e-12 * np.linalg.norm(direct[c1, e1])


def _wavepacket(x, t, sig):
    return wavepacket(x, t, sig)


@pytest.mark.parametrize("cheb", [-1, 0])
def test_example2_long_time_refinement(cheb):
    # T = 1000: each level of dyadic refinement of Gamma_2 gains orders of
    # magnitude, and n_r = 5 is exact to rounding (Section 6, Example 2:
    # n_r = O(log T) keeps the accuracy uniform)
    errs = []
    for nr in range(1, 6):
        orc = FreeSpaceOracle(example2_long_time_problem(nr, cheb, nsteps=100))
        if cheb == 0:
            assert orc.NT[0] > 0 and orc.NT[0] < 32 * nr
        u, _ = orc.run()
        ex = _wavepacket(orc.xs[0] + orc.phi(orc.prob.T)[0], orc.prob.T, 0.1)
        errs.append(np.linalg.norm(u - ex) / np.linalg.norm(ex))
    assert all(errs[i + 1] < errs[i] / 10 for i in range(3)), errs
    assert errs[0] > 1e-3 and errs[4] < 1e-14, errs


@pytest.mark.parametrize("dim", [1, 2])
def test_free_run_through_the_interpolant_equals_the_direct_run(dim):
    M = (48,) if dim == 1 else (32, 32)
    nu = (512,) if dim == 1 else (256, 256)
    prob = free_problem_from_seed(43 + dim, dim, M, 0.05, 12, nu=nu, eps=1e-10, q=16, panels=3)
    prob.cheb = -1
    ud, _ = FreeSpaceOracle(prob).run()
    prob.cheb = 0
    orc = FreeSpaceOracle(prob)
    assert all(orc.NT)
    uc, _ = orc.run()
    assert np.linalg.norm(uc - ud) < 1e-12 * np.linalg.norm(ud)
