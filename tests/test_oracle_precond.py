"""Pins of the oracle's tensor-inverse preconditioner and preconditioned CG.

The separable part of N has the per-mode tensor inverse of Sec. 3; with
lambda = 0 and c = 0 the preconditioner is the exact inverse of N."""
import numpy as np
import pytest

import oracle
import workload
from oracle import precond
from oracle.tensor import inner


def _op(n, lam, seed=0):
    m = tuple((3 * v) // 2 for v in n)
    p = workload.make_problem(n, m, lam, 0.01, seed, 1e-12)
    op = oracle.NormalOperator(p.A, p.D, p.lam)
    return p, op, op.rhs(op.forward(p.X_true) + p.noise)


@pytest.mark.parametrize("n", [(6, 5, 4), (5, 4, 4, 4)])
def test_exact_inverse_when_unregularised(n):
    """lambda = 0, c = 0: M^-1 (N X) = X (the tensor inverse of Sec. 3)."""
    p, op, _ = _op(n, 0.0)
    X = np.random.default_rng(1).standard_normal(n)
    inv = precond.inverse_factors(op.G, [None] * len(n), 0.0)
    back = precond.apply(op(X), inv)
    assert np.max(np.abs(back - X)) <= 1e-9 * np.max(np.abs(X))


def test_inverse_of_one_mode_by_brute_force():
    """M^-1 as a dense matrix equals the Kronecker product of the inverse
    factors (row-major vec: kron in mode order) and inverts the dense
    Kronecker product of (G_k + c R_k)."""
    n = (4, 4, 5)
    p, op, _ = _op(n, 1e-2)
    c = 0.3
    inv = precond.inverse_factors(op.G, op.R, c)
    Mk = [op.G[k] + c * op.R[k] for k in range(3)]
    dense_m = np.kron(np.kron(Mk[0], Mk[1]), Mk[2])
    cols = []
    for i in range(int(np.prod(n))):
        e = np.zeros(int(np.prod(n)))
        e[i] = 1.0
        cols.append(precond.apply(e.reshape(n), inv).ravel())
    dense_inv = np.array(cols).T
    assert np.allclose(dense_inv @ dense_m, np.eye(dense_m.shape[0]), atol=1e-9)


def test_preconditioner_is_symmetric_positive():
    n = (5, 4, 6)
    p, op, _ = _op(n, 1e-3)
    inv = precond.inverse_factors(op.G, op.R, 4e-3)
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    mu, mv = precond.apply(u, inv), precond.apply(v, inv)
    assert abs(inner(u, mv) - inner(mu, v)) <= 1e-10 * abs(inner(u, mv))
    assert inner(u, mu) > 0 and inner(v, mv) > 0


def test_pcg_one_iteration_with_exact_inverse():
    n = (6, 5, 4)
    p, op, B = _op(n, 0.0)
    inv = precond.inverse_factors(op.G, [None] * 3, 0.0)
    X, it, ok = precond.pcg(op, B, lambda r: precond.apply(r, inv), rtol=1e-10, max_iter=10)
    assert ok and it == 1


@pytest.mark.parametrize("lam,c", [(1e-3, 1.6e-2), (1e-2, 4e-2)])
def test_pcg_matches_dense_solution(lam, c):
    n = (6, 5, 4)
    p, op, B = _op(n, lam)
    inv = precond.inverse_factors(op.G, op.R, c)
    X, it, ok = precond.pcg(op, B, lambda r: precond.apply(r, inv), rtol=1e-12, max_iter=500)
    assert ok
    xs = oracle.dense_solve(op, B)
    assert np.linalg.norm(X - xs) <= 1e-8 * np.linalg.norm(xs)


def test_preconditioning_cuts_iterations():
    n = (16, 12, 10, 8)
    p, op, B = _op(n, 1e-3)
    plain = oracle.cg(op, B, rtol=1e-8, max_iter=3000, restart=False)
    inv = precond.inverse_factors(op.G, op.R, 1.6e-2)
    X, it, ok = precond.pcg(op, B, lambda r: precond.apply(r, inv), rtol=1e-8, max_iter=3000)
    assert ok and it < plain.iters / 2, (it, plain.iters)
    assert oracle.relative_residual(X, B, op) <= 1.01e-8
