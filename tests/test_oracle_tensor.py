"""Pins of the oracle's mode products (Sec. 2.1, eq. separable_transf).

The oracle's chain of mode products is checked against the matrix form of a
separable transformation built independently with np.kron (Sec. 3: a tensor
equation is a matrix equation after reshaping), in both vectorisation
conventions, and against the commutativity that ordered spaces give (Sec. 2.1).
"""
import itertools

import numpy as np
import pytest

import oracle
import workload


def _kron_all(mats):
    out = np.ones((1, 1))
    for M in mats:
        out = np.kron(out, M)
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_chain_equals_kronecker_row_major(seed):
    rng = np.random.default_rng(seed)
    shape = (6, 5, 4, 3)
    rows = (4, 3, 5, 2)  # rectangular, so a transposed factor cannot pass
    X = rng.standard_normal(shape)
    mats = [rng.standard_normal((r, s)) for r, s in zip(rows, shape)]
    Y = oracle.multi_mode_product(X, mats)
    # row-major vec: vec_C(Y) = (M1 (x) M2 (x) M3 (x) M4) vec_C(X)
    ref = _kron_all(mats) @ X.reshape(-1)
    assert Y.shape == rows
    np.testing.assert_allclose(Y.reshape(-1), ref, rtol=1e-12, atol=1e-12)


def test_chain_equals_kronecker_column_major():
    rng = np.random.default_rng(5)
    shape = (3, 4, 2)
    mats = [rng.standard_normal((r, s)) for r, s in zip((2, 5, 3), shape)]
    X = rng.standard_normal(shape)
    Y = oracle.multi_mode_product(X, mats)
    # column-major vec: vec_F(Y) = (M3 (x) M2 (x) M1) vec_F(X)
    ref = _kron_all(mats[::-1]) @ X.reshape(-1, order="F")
    np.testing.assert_allclose(Y.reshape(-1, order="F"), ref, rtol=1e-12, atol=1e-12)


def test_chain_integer_exact():
    X = workload.integer_tensor((6, 5, 4, 3), -3, 3, seed=11)
    mats = [workload.integer_tensor((r, s), -3, 3, seed=20 + k)
            for k, (r, s) in enumerate(zip((4, 6, 2, 3), X.shape))]
    Y = oracle.multi_mode_product(X, mats)
    ref = _kron_all(mats) @ X.reshape(-1)
    assert np.array_equal(Y.reshape(-1), ref)


def test_single_mode_explicit_sum():
    # brute force on one mode with explicit loops over every index
    rng = np.random.default_rng(3)
    X = rng.standard_normal((3, 4, 5))
    M = rng.standard_normal((6, 4))
    Y = oracle.mode_product(X, M, 1)
    ref = np.zeros((3, 6, 5))
    for a in range(3):
        for j in range(6):
            for c in range(5):
                ref[a, j, c] = sum(M[j, i] * X[a, i, c] for i in range(4))
    np.testing.assert_allclose(Y, ref, rtol=1e-13, atol=1e-13)


def test_commutativity_all_orders_integer_exact():
    # Sec. 2.1: products on distinct ordered spaces commute; on integers the
    # 24 evaluation orders agree bit for bit.
    X = workload.integer_tensor((5, 4, 6, 3), -3, 3, seed=7)
    mats = [workload.integer_tensor((r, s), -3, 3, seed=30 + k)
            for k, (r, s) in enumerate(zip((3, 5, 2, 4), X.shape))]
    ref = oracle.multi_mode_product(X, mats, order=[0, 1, 2, 3])
    for order in itertools.permutations(range(4)):
        assert np.array_equal(oracle.multi_mode_product(X, mats, order=list(order)), ref)


def test_commutativity_random_within_rounding():
    rng = np.random.default_rng(8)
    X = rng.standard_normal((7, 6, 5, 4))
    mats = [rng.standard_normal((s, s)) for s in X.shape]
    ref = oracle.multi_mode_product(X, mats)
    for order in itertools.permutations(range(4)):
        out = oracle.multi_mode_product(X, mats, order=list(order))
        np.testing.assert_allclose(out, ref, rtol=1e-11, atol=1e-11)


def test_mode_product_shape_check():
    with pytest.raises(ValueError):
        oracle.mode_product(np.zeros((3, 4)), np.zeros((2, 3)), 1)


def test_inner_product_is_vdot():
    # App. A.6: full contraction = sum of the elementwise product
    rng = np.random.default_rng(4)
    A = rng.standard_normal((3, 4, 5))
    B = rng.standard_normal((3, 4, 5))
    assert oracle.inner(A, B) == pytest.approx(np.vdot(A.ravel(), B.ravel()), rel=1e-14)
