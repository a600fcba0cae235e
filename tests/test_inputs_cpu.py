"""Seeded input generators (CPU): the same seed gives the same cohort whether
subjects are generated in one process or in a pool."""

import numpy as np
import pytest

from synthetic.cohorts import WORKLOADS, make_cohort


@pytest.mark.parametrize("name", sorted(WORKLOADS))
def test_cohort_pool_matches_serial(name):
    w = WORKLOADS[name]
    a = make_cohort(w, n=3, dims=(10, 12, 14))
    b = make_cohort(w, n=3, dims=(10, 12, 14), workers=2)
    assert a.dtype == np.float32 and a.shape == (3, 10, 12, 14)
    assert np.array_equal(a, b)


def test_cohort_subjects_differ_and_seed_matters():
    w = WORKLOADS["brain-16x160x192x160-lncc9"]
    a = make_cohort(w, n=2, dims=(10, 12, 14))
    assert not np.array_equal(a[0], a[1])
    assert not np.array_equal(a, make_cohort(w, n=2, dims=(10, 12, 14), seed=w.seed + 1))
