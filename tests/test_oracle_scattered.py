"""Pins of the scattered-measurement oracle (Sec. 6, Sec. 2.2) to facts outside it.

* basis windows against the full Cox-de Boor rows of the grid problems
  (a separate implementation over all knots), and the closed form of the
  uniform cubic B-spline at interior knots (1/6, 2/3, 1/6);
* partition of unity and linear precision (Greville abscissae reproduce t):
  the forward model of all-ones is 1 and of the abscissae of mode k is t_k,
  which fixes the mode order and the index offsets;
* brute force: the dense system matrix built row by row from Kronecker
  products of full basis rows (np.kron) on tiny shapes;
* the Khatri-Rao reduction: sites on a full tensor grid give
  sum_i a_i a_i^T = (x)_k A_k^T A_k, so the CP-sum operator must equal the
  separable Gram-chain operator of the grid problems (independent code);
* the adjoint identity, symmetry and positivity, and a CG solve judged by the
  dense solution.
"""
import itertools

import numpy as np
import pytest

import oracle
import workload
from oracle import scattered as sc
from workload.bspline import _basis_row, clamped_knots, collocation_matrix, second_difference


def _full_rows(coords, n):
    """Dense Kronecker rows (S, prod n) from full per-mode basis rows."""
    N, S = coords.shape
    out = np.zeros((S, int(np.prod(n))))
    for i in range(S):
        row = np.ones(1)
        for k in range(N):
            row = np.kron(row, _basis_row(float(coords[k, i]), clamped_knots(n[k]), n[k], 3))
        out[i] = row
    return out


@pytest.mark.parametrize("n", [4, 5, 7, 16, 33])
def test_basis_window_matches_full_recursion(n):
    rng = np.random.default_rng(n)
    t = np.concatenate([rng.random(200), [0.0, 1.0], np.linspace(0, 1, n - 2)])
    first, w = sc.basis_window(t, n)
    assert first.min() >= 0 and first.max() <= n - 4
    for i, ti in enumerate(t):
        full = _basis_row(float(ti), clamped_knots(n), n, 3)
        win = np.zeros(n)
        win[first[i]:first[i] + 4] = w[i]
        assert np.max(np.abs(win - full)) <= 1e-14


def test_uniform_interior_values():
    # at an interior knot far from the clamped ends the cubic B-spline takes 1/6, 2/3, 1/6
    n = 20
    t = 8.0 / (n - 3)
    first, w = sc.basis_window(np.array([t]), n)
    vals = np.zeros(n)
    vals[first[0]:first[0] + 4] = w[0]
    nz = vals[vals > 1e-15]
    assert np.allclose(nz, [1 / 6, 2 / 3, 1 / 6], atol=1e-15)


@pytest.mark.parametrize("n", [(6, 5, 7), (4, 9, 5, 6), (12, 11)])
def test_partition_of_unity_and_linear_precision(n):
    coords = workload.with_endpoints(workload.scattered_sites(len(n), 500, seed=3))
    f = sc.forward(np.ones(n), coords)
    assert np.max(np.abs(f - 1.0)) <= 1e-14
    for k, nk in enumerate(n):
        u = clamped_knots(nk)
        greville = np.array([(u[j + 1] + u[j + 2] + u[j + 3]) / 3.0 for j in range(nk)])
        shape = [1] * len(n)
        shape[k] = nk
        X = np.broadcast_to(greville.reshape(shape), n)
        f = sc.forward(X, coords)
        assert np.max(np.abs(f - coords[k].astype(np.float64))) <= 1e-14


@pytest.mark.parametrize("n", [(5, 6, 7), (4, 5, 4, 6), (7, 5)])
def test_brute_force_dense_rows(n):
    rng = np.random.default_rng(sum(n))
    coords = workload.with_endpoints(workload.scattered_sites(len(n), 60, seed=7))
    A = _full_rows(coords, n)
    X = rng.standard_normal(n)
    y = rng.standard_normal(coords.shape[1])
    D = [second_difference(k) for k in n]
    lam = 0.3
    op = sc.ScatteredOperator(coords, n, D, lam)
    assert np.max(np.abs(op.forward(X) - A @ X.ravel())) <= 1e-13
    assert np.max(np.abs(op.rhs(y).ravel() - A.T @ y)) <= 1e-13
    # regulariser assembled densely as the Kronecker sum of D_k^T D_k
    Rd = np.zeros((A.shape[1], A.shape[1]))
    for k in range(len(n)):
        mats = [np.eye(m) for m in n]
        mats[k] = D[k].T @ D[k]
        K = np.ones((1, 1))
        for M in mats:
            K = np.kron(K, M)
        Rd += K
    want = (A.T @ A + lam * Rd) @ X.ravel()
    assert np.max(np.abs(op(X).ravel() - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("n,m", [((6, 5, 7), (9, 8, 10)), ((5, 4, 6, 4), (7, 6, 8, 6))])
def test_grid_sites_reduce_to_separable_operator(n, m):
    grids = [np.arange(mk) / (mk - 1) for mk in m]
    pts = np.array(list(itertools.product(*grids))).T.astype(np.float32)
    # the grid points i/(m-1) are not all float32-exact; use the float32 values on both sides
    A = []
    for k, (mk, nk) in enumerate(zip(m, n)):
        Ak = np.stack([_basis_row(float(t), clamped_knots(nk), nk, 3)
                       for t in np.unique(pts[k].astype(np.float64))])
        A.append(Ak)
    D = [second_difference(k) for k in n]
    lam = 1e-2
    X = np.random.default_rng(1).standard_normal(n)
    op = sc.ScatteredOperator(pts, n, D, lam)
    sep = oracle.NormalOperator(A, D, lam)
    got, want = op(X), sep(X)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    # and the right-hand side: adjoint of grid data = separable transposed chain
    Y = np.random.default_rng(2).standard_normal(m)
    assert np.allclose(op.rhs(Y.ravel()), sep.rhs(Y), rtol=0, atol=1e-12 * np.max(np.abs(sep.rhs(Y))))


def test_grid_collocation_matches_workload_collocation():
    # the float64 grid of the grid problems gives the same rows as the oracle windows
    m, n = 11, 8
    C = collocation_matrix(m, n)
    first, w = sc.basis_window(np.arange(m) / (m - 1), n)
    for i in range(m):
        row = np.zeros(n)
        row[first[i]:first[i] + 4] = w[i]
        assert np.max(np.abs(row - C[i])) <= 1e-15


def test_adjoint_identity_symmetry_positivity():
    n = (9, 8, 7, 6)
    p = workload.scattered_problem(n, 3000, 1e-2, 0.01, seed=11, rtol=1e-8, clustered=0.5)
    op = sc.ScatteredOperator(p.coords, n, p.D, p.lam)
    rng = np.random.default_rng(5)
    X, Z = rng.standard_normal(n), rng.standard_normal(n)
    y = rng.standard_normal(p.count)
    assert abs(oracle.inner(op.forward(X), y) - oracle.inner(X, op.rhs(y))) <= 1e-11 * np.sqrt(p.count)
    a, b = oracle.inner(op(X), Z), oracle.inner(X, op(Z))
    assert abs(a - b) <= 1e-12 * abs(a)
    assert oracle.inner(op(X), X) > 0
    # <X, N X> = ||A X||^2 + lam <X, R X>
    f = op.forward(X)
    reg = oracle.inner(X, oracle.regulariser_apply(X, op.R, p.lam))
    assert abs(oracle.inner(op(X), X) - (f @ f + reg)) <= 1e-12 * (f @ f + reg)


def test_cg_on_scattered_operator_matches_dense_solve():
    n = (6, 5, 7)
    p = workload.scattered_problem(n, 150, 1e-2, 0.01, seed=12, rtol=1e-10)
    op = sc.ScatteredOperator(p.coords, n, p.D, p.lam)
    y = op.forward(p.X_true) + p.noise
    B = op.rhs(y)
    res = oracle.cg(op, B, rtol=1e-12, max_iter=2000)
    A = _full_rows(p.coords, n)
    Rd = np.zeros((A.shape[1], A.shape[1]))
    for k in range(len(n)):
        mats = [np.eye(m) for m in n]
        mats[k] = p.D[k].T @ p.D[k]
        K = np.ones((1, 1))
        for M in mats:
            K = np.kron(K, M)
        Rd += K
    xd = np.linalg.solve(A.T @ A + p.lam * Rd, B.ravel())
    assert res.status == 0
    assert np.max(np.abs(res.x.ravel() - xd)) <= 1e-8 * np.max(np.abs(xd))


def test_empty_site_set():
    n = (5, 5, 5)
    coords = np.zeros((3, 0), dtype=np.float32)
    op = sc.ScatteredOperator(coords, n, [second_difference(k) for k in n], 0.5)
    X = np.random.default_rng(0).standard_normal(n)
    assert op.forward(X).shape == (0,)
    assert np.allclose(op(X), oracle.regulariser_apply(X, op.R, 0.5))
