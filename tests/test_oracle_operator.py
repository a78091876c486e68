"""Pins of the oracle's normal operator, right-hand side and regulariser."""
import os

import numpy as np
import pytest

import oracle
import workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.txt")


def _golden():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[k] = int(v)
    return out


def _tiny_problem(n=(4, 5, 6), lam=0.3, seed=1):
    m = tuple(max(6, (3 * v) // 2) for v in n)
    return workload.make_problem(n, m, lam, 0.01, seed, 1e-10)


def _kron_all(mats):
    out = np.ones((1, 1))
    for M in mats:
        out = np.kron(out, M)
    return out


def test_assembled_operator_equals_kronecker_formula():
    # Matrix form (Sec. 3) of N: kron of Grams plus the Kronecker sum of R_k,
    # built with np.kron independently of the oracle's mode products.
    p = _tiny_problem()
    op = oracle.NormalOperator(p.A, p.D, p.lam)
    M = oracle.assemble(op, p.n)
    G = [a.T @ a for a in p.A]
    R = [d.T @ d for d in p.D]
    I = [np.eye(k) for k in p.n]
    ref = _kron_all(G)
    for k in range(len(p.n)):
        facs = [R[j] if j == k else I[j] for j in range(len(p.n))]
        ref = ref + p.lam * _kron_all(facs)
    np.testing.assert_allclose(M, ref, rtol=1e-12, atol=1e-13)


def test_gram_form_equals_literal_form():
    p = _tiny_problem(n=(6, 5, 4, 4), lam=0.05)
    rng = np.random.default_rng(9)
    X = rng.standard_normal(p.n)
    a = oracle.normal_apply(X, [oracle.gram(x) for x in p.A],
                            [oracle.reg_factor(d) for d in p.D], p.lam)
    b = oracle.normal_apply_literal(X, p.A, p.D, p.lam)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)


def test_operator_symmetric_positive_definite():
    p = _tiny_problem(n=(5, 4, 6), lam=1e-3)
    op = oracle.NormalOperator(p.A, p.D, p.lam)
    rng = np.random.default_rng(2)
    u = rng.standard_normal(p.n)
    v = rng.standard_normal(p.n)
    assert oracle.inner(u, op(v)) == pytest.approx(oracle.inner(op(u), v), rel=1e-12)
    M = oracle.assemble(op, p.n)
    np.linalg.cholesky(M)
    assert np.linalg.eigvalsh(M)[0] > 0


def test_rhs_is_transpose_of_forward():
    # <forward(X), Y> = <X, rhs(Y)>: rhs applies the transposed factors (App. A.7)
    p = _tiny_problem(n=(4, 6, 5))
    rng = np.random.default_rng(6)
    X = rng.standard_normal(p.n)
    Y = rng.standard_normal(p.m)
    lhs = oracle.inner(oracle.forward(X, p.A), Y)
    rhs_ = oracle.inner(X, oracle.rhs(Y, p.A))
    assert lhs == pytest.approx(rhs_, rel=1e-12)
    # and the forward model equals the Kronecker product of the A_k
    ref = _kron_all(p.A) @ X.reshape(-1)
    np.testing.assert_allclose(oracle.forward(X, p.A).reshape(-1), ref, rtol=1e-12, atol=1e-12)


def test_regulariser_factor_properties():
    n = 9
    R = oracle.reg_factor(workload.second_difference(n))
    # annihilates constants and linear ramps
    np.testing.assert_allclose(R @ np.ones(n), 0, atol=1e-14)
    np.testing.assert_allclose(R @ np.arange(n, dtype=float), 0, atol=1e-12)
    # interior row is the pentadiagonal [1, -4, 6, -4, 1]
    assert np.array_equal(R[4, 2:7], [1, -4, 6, -4, 1])
    assert np.count_nonzero(R[4]) == 5
    assert np.array_equal(R, R.T)


def test_regulariser_is_kronecker_sum_stencil():
    # lam * sum_k X x_k R_k equals the 5-point-per-mode stencil written out
    n = (6, 7, 5)
    rng = np.random.default_rng(12)
    X = rng.standard_normal(n)
    R = [oracle.reg_factor(workload.second_difference(k)) for k in n]
    out = oracle.regulariser_apply(X, R, 0.5)
    ref = np.zeros(n)
    for idx in np.ndindex(*n):
        s = 0.0
        for k in range(3):
            for j in range(max(0, idx[k] - 2), min(n[k], idx[k] + 3)):
                src = list(idx)
                src[k] = j
                s += R[k][idx[k], j] * X[tuple(src)]
        ref[idx] = 0.5 * s
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)


def test_gram_band_and_paper_nonzero_count():
    # Cubic B-spline Grams have half-bandwidth exactly 3.  The matrix form of
    # the 128x128x128x16 reconstruction stored as block-band upper triangles
    # then holds prod_k (4 n_k - 6) entries, which is the count Sec. 6 prints.
    counts = []
    for n in (128, 128, 128, 16):
        A = workload.collocation_matrix((3 * n) // 2, n)
        G = oracle.gram(A)
        nz = np.argwhere(np.abs(G) > 0)
        band = int(np.max(np.abs(nz[:, 0] - nz[:, 1])))
        assert band == 3
        upper = int(np.count_nonzero(np.triu(G)))
        assert upper == 4 * n - 6
        counts.append(upper)
    g = _golden()
    assert int(np.prod(counts, dtype=np.int64)) == g["band_storage_nonzeros_128x128x128x16"]
    assert 128 * 128 * 128 * 16 == g["unknowns_128x128x128x16"]
