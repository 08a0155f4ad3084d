"""Pins of the free-space oracle in three dimensions (Section 4.3: the line
transforms of Section 4.1 along each axis, so the 125 node-type subsets in
tensor order; Lemma 3.1's propagator with zeta . zeta and zeta . dphi over
three axes) against what the mathematics fixes: the transform pair inverts
on compactly supported data, and with V = 0 the scheme applies the exact
propagator, so an anisotropic Gaussian packet (a product of Section 6,
Example 2's packets), shifted by a field along axis 0, is reproduced."""
import numpy as np

from oracle.freespace import FreeSpaceOracle, free_grid
from workloads import Problem, free_problem_from_seed, wavepacket


def test_round_trip_3d():
    # data resolved by the grid and negligible at the box edge: F^-1 F f = f
    # to the contour rule's accuracy (the 1D pin's bound, per axis)
    M = (40, 44, 48)
    prob = free_problem_from_seed(63, 3, M, 0.05, 2, order=2, nu=(256, 256, 256), eps=1e-10, q=10)
    orc = FreeSpaceOracle(prob)
    xs = [free_grid(m) for m in M]
    f = np.einsum("i,j,k->ijk", *[wavepacket(x - c0, 0, 0.12) * np.exp(2j * x) for x, c0 in zip(xs, (0.1, 0.0, -0.1))])
    g = orc.Finv(orc.F(f))
    assert np.max(np.abs(g - f)) < 1e-9 * np.max(np.abs(f))


def test_free_wavepacket_3d_exact_with_field():
    M, nu, T = (40, 36, 44), 256, 0.02
    sig = (0.12, 0.11, 0.125)
    c = (0.1, -0.05, 0.0)
    xs = [free_grid(m) for m in M]
    u0 = np.einsum("i,j,k->ijk", *[wavepacket(x - c0, 0, s) for x, c0, s in zip(xs, c, sig)])
    prob = Problem(name="wp3", dim=3, domain="free", M=M, T=T, nsteps=2, order=2, u0=u0.astype(complex),
                   V_fields=[np.zeros(M)], f_kind=["const"], f_params=[(0, 0)], A_kind="pulse_sin2",
                   A_params=(15.0, 40.0, T, 1.0, 0.0, 0.0), eps=1e-10, q=10, panels=1, nu=(nu, nu, nu))
    orc = FreeSpaceOracle(prob)
    u, _ = orc.run()
    ph = orc.phi(T)
    assert abs(ph[0]) > 1e-3 and ph[1] == 0.0 and ph[2] == 0.0
    ex = np.einsum("i,j,k->ijk", *[wavepacket(x - c0 + p, T, s) for x, c0, p, s in zip(xs, c, ph, sig)])
    err = np.max(np.abs(u - ex)) / np.max(np.abs(ex))
    assert err < 1e-8, err
    # and without the shift the comparison fails: the field is really applied
    ex0 = np.einsum("i,j,k->ijk", *[wavepacket(x - c0, T, s) for x, c0, s in zip(xs, c, sig)])
    assert np.max(np.abs(u - ex0)) / np.max(np.abs(ex)) > 100 * err
