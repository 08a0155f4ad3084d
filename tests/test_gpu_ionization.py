"""GPU run of Section 6, Example 3 (ionization from a Gaussian well in 1D,
free space, the cosine pulse of eq. (apulse)) through the C ABI: u(T) against
the free-space oracle (relative L2 <= 1e-11) and the ionization fractions
against the values the paper prints (tests/golden/example3_ionization.txt)."""
import os

import numpy as np
import pytest

from oracle.freespace import FreeSpaceOracle
from test_oracle_ionization import golden, ionization_percent
from workloads import ionization_1d_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2001_06113_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2001_06113_amd import build

        build.build()
    yield


@pytest.mark.parametrize("omega", [50.0, 100.0, 200.0])
def test_ionization_matches_oracle_and_printed_fraction(omega):
    from paper_2001_06113_amd.tdse import Plan

    _, rows = golden()
    ion_paper = {om: ion for om, _, ion in rows}[omega]
    prob = ionization_1d_problem(omega, nsteps=4000)
    print(f"case ionization omega={omega} steps={prob.nsteps}", flush=True)
    plan = Plan.from_problem(prob, device="cuda:0")
    u = plan.run(prob.u0).cpu().numpy()
    plan.close()
    ref, _ = FreeSpaceOracle(prob).run()
    r = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    ion = ionization_percent(u, prob.M[0])
    print(f"  rel-L2 vs oracle = {r:.3e}; ionization {ion:.4f}% (printed {ion_paper}%)", flush=True)
    assert r <= 1e-11, r
    assert abs(ion - ion_paper) < 0.005, ion
