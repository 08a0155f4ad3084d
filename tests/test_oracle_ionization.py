"""Pins of the ground-state input and of the free-space oracle against the
values Section 6, Example 3 prints (tests/golden/example3_ionization.txt):
the ground-state eigenvalue of the Gaussian well, the quiver radii of the
cosine pulse of eq. (apulse), and the ionization fractions after T = 0.5."""
import os

import numpy as np
import pytest

from oracle.freespace import FreeSpaceOracle
from workloads import free_grid, gaussian_well_ground_state, ionization_1d_problem

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "example3_ionization.txt")


def golden():
    E, rows = None, []
    for line in open(GOLDEN):
        if line.startswith("# ground_eigenvalue"):
            E = float(line.split()[2])
        elif not line.startswith("#"):
            om, ph, ion = (float(v) for v in line.split())
            rows.append((om, ph, ion))
    return E, rows


def ionization_percent(u, M):
    # 1 - int_{-1}^{1} |u(x,T)|^2 dx by the left endpoint rule on the grid
    return 100.0 * (1.0 - np.sum(np.abs(u) ** 2) * 2.0 / M)


def test_ground_state_matches_the_printed_eigenvalue():
    E_paper, _ = golden()
    E, gs = gaussian_well_ground_state(1400.0, 0.1)
    assert abs(E - E_paper) < 0.5                      # "approximately -1154": -1154.29
    # a finer discretization changes nothing: the state is resolved
    E2, gs2 = gaussian_well_ground_state(1400.0, 0.1, n=768)
    assert abs(E - E2) < 1e-8
    x = np.linspace(-1.9, 1.9, 77)
    assert np.max(np.abs(gs(x) - gs2(x))) < 1e-10
    # normalized, and below 1e-12 outside [-1,1] as the example states
    xf = np.linspace(-2, 2, 4001)[:-1]
    assert abs(np.sum(gs(xf) ** 2) * 0.001 - 1.0) < 1e-10
    assert np.max(np.abs(gs(np.array([-1.5, -1.0, 1.0, 1.5])))) < 1e-12
    # it solves -u'' + V u = E u: a centred difference of the interpolant
    h = 1e-3
    xs = np.linspace(-0.3, 0.3, 13)
    d2 = (gs(xs + h) - 2 * gs(xs) + gs(xs - h)) / h ** 2
    V = -1400.0 * np.exp(-xs ** 2 / 0.02)
    assert np.max(np.abs(-d2 + V * gs(xs) - E * gs(xs))) < 1e-3 * np.max(np.abs(E * gs(xs)))


def test_quiver_radii_of_the_cosine_pulse():
    _, rows = golden()
    for om, ph_paper, _ in rows:
        prob = ionization_1d_problem(om, nsteps=200)
        orc_phi = FreeSpaceOracle(prob).phi
        phimax = max(abs(orc_phi(t)[0]) for t in np.linspace(0.0, 0.5, 401))
        assert abs(phimax - ph_paper) < 0.02 * ph_paper, (om, phimax)


@pytest.mark.parametrize("omega", [100.0, 200.0])
def test_oracle_ionization_matches_the_printed_fractions(omega):
    # 4000 steps; the printed fractions have four digits
    _, rows = golden()
    ion_paper = {om: ion for om, _, ion in rows}[omega]
    prob = ionization_1d_problem(omega, nsteps=4000)
    u, _ = FreeSpaceOracle(prob).run()
    assert abs(ionization_percent(u, prob.M[0]) - ion_paper) < 0.005


def test_2d_ground_state_matches_the_printed_eigenvalue():
    # Section 6, Example 4: eigenvalue about -922, state below 1e-11 outside [-1,1]^2
    from workloads import gaussian_well_ground_state_2d

    E, gs = gaussian_well_ground_state_2d(1400.0, 0.1)
    assert abs(E - (-922.0)) < 0.5                    # -922.068
    E2, gs2 = gaussian_well_ground_state_2d(1400.0, 0.1, n=160)
    assert abs(E - E2) < 1e-7
    x = np.linspace(-1.9, 1.9, 39)
    assert np.max(np.abs(gs(x, x) - gs2(x, x))) < 1e-8
    edge = np.linspace(-2, 2, 81)
    g = np.abs(gs(edge, edge))
    out = (np.abs(edge)[:, None] > 1) | (np.abs(edge)[None, :] > 1)
    assert g[out].max() < 1e-11
    xf = np.linspace(-2, 2, 401)[:-1]
    assert abs(np.sum(gs(xf, xf) ** 2) * 0.01 ** 2 - 1.0) < 1e-10
    # radially symmetric, as the well is
    r = np.linspace(0.0, 0.5, 11)
    assert np.max(np.abs(gs(r, [0.0])[:, 0] - np.diag(gs(r / np.sqrt(2), r / np.sqrt(2))))) < 1e-9
