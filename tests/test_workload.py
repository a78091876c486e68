"""Checks of the seeded input generators (collocation, differences, draws)."""
import numpy as np
import pytest
from scipy.interpolate import BSpline

import workload
from workload.bspline import clamped_knots


@pytest.mark.parametrize("m,n", [(48, 32), (96, 64), (36, 24), (192, 128), (24, 16), (9, 5)])
def test_collocation_matches_scipy(m, n):
    A = workload.collocation_matrix(m, n)
    t = np.arange(m) / (m - 1)
    ref = BSpline.design_matrix(t, clamped_knots(n), 3).toarray()
    np.testing.assert_allclose(A, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("m,n", [(48, 32), (144, 96), (36, 24)])
def test_collocation_properties(m, n):
    A = workload.collocation_matrix(m, n)
    np.testing.assert_allclose(A.sum(axis=1), 1.0, atol=1e-14)   # partition of unity
    assert (np.count_nonzero(A, axis=1) <= 4).all()             # cubic: <= 4 per row
    np.testing.assert_allclose(A[::-1, ::-1], A, atol=1e-14)     # centro-symmetric
    assert np.linalg.matrix_rank(A) == n                          # full column rank


def test_second_difference():
    D = workload.second_difference(6)
    assert D.shape == (4, 6)
    assert np.array_equal(D[1], [0, 1, -2, 1, 0, 0])


def test_seeded_draws_reproducible():
    a = workload.config_problem(0)
    b = workload.config_problem(0)
    assert np.array_equal(a.X_true, b.X_true) and np.array_equal(a.noise, b.noise)
    assert a.X_true.shape == (32, 32, 32) and a.noise.shape == (48, 48, 48)


def test_batched_sizes():
    s = workload.batched_sizes()
    assert s.shape == (256, 3)
    assert set(np.unique(s)) <= {24, 32, 48, 64, 96}
    p = workload.batched_problem(5, s)
    assert p.m == tuple(3 * v // 2 for v in p.n)


def test_blob_field():
    p = workload.warmstart_problem(3, n=(16, 12, 10, 8), m=(24, 18, 15, 12))
    assert p.X_true.shape == (16, 12, 10, 8)
    assert np.isfinite(p.X_true).all()
