"""Pins of the oracle's tensor CG (Fig. Tensor_CG) and tensor inverse (Sec. 3)."""
import numpy as np
import pytest

import oracle
import workload
from oracle.cg import BREAKDOWN, CONVERGED, NOT_CONVERGED


def _problem(n, lam, seed=0):
    m = tuple((3 * v) // 2 for v in n)
    p = workload.make_problem(n, m, lam, 0.01, seed, 1e-12)
    op = oracle.NormalOperator(p.A, p.D, p.lam)
    Y = op.forward(p.X_true) + p.noise
    return p, op, op.rhs(Y)


@pytest.mark.parametrize("n,lam", [((6, 5, 4), 1e-3), ((5, 4, 4, 4), 1e-2), ((8, 8, 8), 1e-4)])
def test_cg_matches_dense_cholesky(n, lam):
    p, op, B = _problem(n, lam)
    res = oracle.cg(op, B, rtol=1e-13)
    assert res.status == CONVERGED
    ref = oracle.dense_solve(op, B)
    M = oracle.assemble(op, p.n)
    kappa = np.linalg.cond(M)
    err = np.linalg.norm(res.x - ref) / np.linalg.norm(ref)
    assert err <= kappa * 1e-12
    assert oracle.relative_residual(res.x, B, op) <= 1e-12


def test_identity_operator_one_iteration():
    # orthogonal square A_k and lam = 0 give N = I: one iteration, X = B
    rng = np.random.default_rng(0)
    n = (4, 5, 3)
    A = [np.linalg.qr(rng.standard_normal((k, k)))[0] for k in n]
    D = [np.zeros((1, k)) for k in n]
    op = oracle.NormalOperator(A, D, 0.0)
    B = rng.standard_normal(n)
    res = oracle.cg(op, B, rtol=1e-14)
    assert res.iters == 1
    np.testing.assert_allclose(res.x, B, rtol=1e-14, atol=1e-14)


def test_tensor_inverse_square_case():
    # Sec. 3 (eq. TensorEq): with lam = 0 and square invertible A_k the solution
    # of the normal equations is Y x_k A_k^{-1} on every mode.
    rng = np.random.default_rng(1)
    n = (5, 4, 6)
    A = [np.eye(k) * 2.0 + 0.3 * rng.standard_normal((k, k)) for k in n]
    D = [np.zeros((1, k)) for k in n]
    op = oracle.NormalOperator(A, D, 0.0)
    Y = rng.standard_normal(n)
    B = op.rhs(Y)
    res = oracle.cg(op, B, rtol=1e-14)
    # per-mode inverses via np.linalg.solve on each mode's unfolding
    ref = Y.copy()
    for k, Ak in enumerate(A):
        moved = np.moveaxis(ref, k, 0)
        sol = np.linalg.solve(Ak, moved.reshape(moved.shape[0], -1))
        ref = np.moveaxis(sol.reshape(moved.shape), 0, k)
    np.testing.assert_allclose(res.x, ref, rtol=1e-9, atol=1e-10)


def test_finite_termination_distinct_eigenvalues():
    # diagonal G_k whose Kronecker products take d distinct values: CG ends in
    # at most d iterations (exact-arithmetic property; rounding leaves ~1e-8
    # after d steps, so the test asks for 1e-6)
    n = (3, 2, 2)
    A = [np.diag(np.sqrt([1.0, 2.0, 4.0])), np.diag(np.sqrt([1.0, 3.0])),
         np.diag(np.sqrt([1.0, 5.0]))]
    D = [np.zeros((1, k)) for k in n]
    op = oracle.NormalOperator(A, D, 0.0)
    vals = {a * b * c for a in (1, 2, 4) for b in (1, 3) for c in (1, 5)}
    B = np.random.default_rng(2).standard_normal(n)
    res = oracle.cg(op, B, rtol=1e-6, restart=False)
    assert res.status == CONVERGED
    assert res.iters <= len(vals)


def test_energy_norm_error_decreases():
    p, op, B = _problem((6, 6, 5), 1e-3, seed=4)
    xs = oracle.dense_solve(op, B)
    errs = []
    for k in range(1, 25):
        r = oracle.cg(op, B, rtol=0.0, max_iter=k, restart=False)
        e = r.x - xs
        errs.append(oracle.inner(e, op(e)))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs, errs[1:]))


def test_lanczos_extremes_match_eigenvalues():
    p, op, B = _problem((6, 5, 5), 1e-3, seed=3)
    res = oracle.cg(op, B, rtol=1e-14, restart=False)
    lo, hi = oracle.lanczos_extremes(res.alphas, res.betas)
    ev = np.linalg.eigvalsh(oracle.assemble(op, p.n))
    # Ritz values lie inside the spectrum and approach its ends
    assert ev[0] * (1 - 1e-9) <= lo <= hi <= ev[-1] * (1 + 1e-9)
    assert hi == pytest.approx(ev[-1], rel=1e-6)
    assert lo == pytest.approx(ev[0], rel=1e-2)


def test_breakdown_on_indefinite_operator():
    p, op, B = _problem((5, 5, 5), 1e-3)
    bad = oracle.NormalOperator(p.A, p.D, -50.0)
    res = oracle.cg(bad, B, rtol=1e-12)
    assert res.status == BREAKDOWN


def test_not_converged_at_max_iter():
    p, op, B = _problem((6, 6, 6), 1e-4)
    res = oracle.cg(op, B, rtol=1e-12, max_iter=2)
    assert res.status == NOT_CONVERGED and res.iters == 2


def test_zero_rhs_returns_start():
    p, op, B = _problem((5, 5, 5), 1e-3)
    res = oracle.cg(op, np.zeros(p.n), rtol=1e-8)
    assert res.iters == 0 and not res.x.any()


def test_warm_start_from_solution():
    p, op, B = _problem((5, 6, 5), 1e-3)
    xs = oracle.dense_solve(op, B)
    res = oracle.cg(op, B, x0=xs, rtol=1e-8)
    assert res.iters == 0 and res.status == CONVERGED


@pytest.mark.parametrize("n,lam", [((4, 5, 3), 1e-2), ((4, 4, 5, 4), 1e-3)])
def test_relative_residual_against_kronecker_matrix(n, lam):
    """The judge equals ||b - M x|| / ||b|| with M assembled from np.kron of the
    factors (the matrix form of the tensor equation, Sec. 3), not from the
    oracle's own mode products."""
    n = tuple(max(v, 4) for v in n)
    p, op, B = _problem(n, lam)
    G = [a.T @ a for a in p.A]
    R = [d.T @ d for d in p.D]
    M = np.ones((1, 1))
    for g in G:
        M = np.kron(M, g)
    for k in range(len(n)):
        term = np.ones((1, 1))
        for l in range(len(n)):
            term = np.kron(term, R[k] if l == k else np.eye(n[l]))
        M = M + lam * term
    X = np.random.default_rng(6).standard_normal(n)
    ref = np.linalg.norm(B.reshape(-1) - M @ X.reshape(-1)) / np.linalg.norm(B.reshape(-1))
    assert np.isclose(oracle.relative_residual(X, B, op), ref, rtol=1e-12)
    # exact solution: residual at rounding level; zero right-hand side: scale 1
    Xs = np.linalg.solve(M, B.reshape(-1)).reshape(n)
    assert oracle.relative_residual(Xs, B, op) <= 1e-12
    assert oracle.relative_residual(X, np.zeros(n), op) == pytest.approx(
        np.linalg.norm(M @ X.reshape(-1)), rel=1e-12)


def test_fp32_storage_model():
    """store=float32 keeps every vector on the float32 grid and reaches the
    tolerance that FP32 vectors allow; without it the oracle is unchanged."""
    p, op, B = _problem((6, 5, 4), 1e-3)
    a = oracle.cg(op, B, rtol=1e-10)
    b = oracle.cg(op, B, rtol=1e-10, store=None)
    assert np.array_equal(a.x, b.x) and a.iters == b.iters
    c = oracle.cg(op, B, rtol=1e-5, store=np.float32)
    assert np.array_equal(c.x, c.x.astype(np.float32).astype(np.float64))
    assert c.status == CONVERGED and oracle.relative_residual(c.x, B, op) <= 1e-5
