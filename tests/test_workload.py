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


def test_blob_field_torch_deterministic_and_shaped():
    torch = pytest.importorskip("torch")
    X1, _ = workload.blob_field_torch((6, 7, 5, 4), 12, device="cpu")
    X2, _ = workload.blob_field_torch((6, 7, 5, 4), 12, device="cpu")
    X3, _ = workload.blob_field_torch((6, 7, 5, 4), 13, device="cpu")
    assert X1.dtype == torch.float32 and tuple(X1.shape) == (6, 7, 5, 4)
    assert torch.equal(X1, X2) and not torch.equal(X1, X3)
    # without the white noise the field is a sum of at most 8 separable blobs
    Xn, _ = workload.blob_field_torch((6, 7, 5, 4), 12, noise_sigma=0.0, device="cpu")
    M = Xn.double().reshape(6, -1).numpy()
    assert np.linalg.matrix_rank(M, tol=1e-6 * np.abs(M).max()) <= 8
    assert float(Xn.abs().max()) <= 8 * 2.0 + 1e-6


def test_scattered_sites_seeded_and_in_range():
    import workload
    a = workload.scattered_sites(4, 5000, seed=9, clustered=0.4)
    b = workload.scattered_sites(4, 5000, seed=9, clustered=0.4)
    assert a.dtype == np.float32 and a.shape == (4, 5000)
    assert np.array_equal(a, b)
    assert a.min() >= 0.0 and a.max() <= 1.0
    e = workload.with_endpoints(a)
    for s in range(16):
        for k in range(4):
            assert e[k, s] == (1.0 if (s >> k) & 1 else 0.0)
    assert np.array_equal(e[:, 16:], a[:, 16:])


def test_scattered_config_shapes():
    import workload
    p = workload.scattered_config(scale=8)
    assert p.n == (16, 16, 16, 4) and p.coords.shape[0] == 4
    assert p.X_true.shape == p.n and p.noise.shape == (p.count,)
    assert p.count == int(9_000_000 * np.prod(p.n) / (128 * 128 * 128 * 16))
    full = workload.SCATTERED
    assert full["n"] == (128, 128, 128, 16) and full["count"] == 9_000_000
