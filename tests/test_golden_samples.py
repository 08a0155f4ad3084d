"""The stored oracle samples of the benchmarked workloads
(tests/golden/*_oracle_sample.txt): every file parses, its sub-grid matches
its stated stride and shape, and the cheap cases are reproduced exactly by
re-running the generator's own recipe on the oracle (so the files are what
tests/golden/make_bench_oracle_samples.py writes)."""
import os

import numpy as np
import pytest

from workloads.golden import GOLDEN, load_samples, sampled_error

CASES = ["periodic_1d_256", "periodic_2d_512", "periodic_2d_1024", "free_2d_256_default_h", "moving_well_2d_512", "batch_64",
         "example2_long_time_nr5", "periodic_3d_128", "free_3d_32"]


@pytest.mark.parametrize("case", CASES)
def test_sample_file_is_well_formed(case):
    inst = load_samples(case)
    assert len(inst) == (64 if case == "batch_64" else 1)
    for i, d in inst.items():
        s, shape = d["stride"], d["shape"]
        want = int(np.prod([len(range(0, m, s)) for m in shape]))
        assert len(d["val"]) == want, (i, len(d["val"]), want)
        assert np.all(d["idx"] % s == 0)
        assert np.isfinite(d["norm"]) and d["norm"] > 0
        assert np.all(np.isfinite(d["val"]))
        # the samples' norm is consistent with the full-grid norm
        frac = np.linalg.norm(d["val"]) * np.sqrt(np.prod([s] * len(shape))) / d["norm"]
        assert 0.2 < frac < 5.0, (i, frac)
        if case == "free_2d_256_default_h":
            assert len(d["H"]) == 2 and all(1.0 < h < 4.0 for h in d["H"])


def _rerun(case, inst):
    import importlib.util

    spec = importlib.util.spec_from_file_location("mk", os.path.join(GOLDEN, "make_bench_oracle_samples.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    from oracle.periodic import PeriodicOracle

    kind, prob, s2, s1 = mk.cases()[case]()[inst]
    if kind == "free":
        from oracle.freespace import FreeSpaceOracle

        return FreeSpaceOracle(prob).run()[0]
    u, _ = PeriodicOracle(prob).run()
    return u


@pytest.mark.parametrize("case,inst", [("periodic_1d_256", 0), ("batch_64", 0), ("batch_64", 1),
                                       ("example2_long_time_nr5", 0)])
def test_cheap_cases_reproduce_exactly(case, inst):
    u = _rerun(case, inst)
    e = sampled_error(u, load_samples(case)[inst])
    assert e["rel_l2"] == 0.0 and e["norm_rel"] == 0.0, e
