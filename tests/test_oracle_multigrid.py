"""Pins of the oracle's tensor Jacobi (Fig. Tensor_Jacobi) and tensor
multigrid V-cycle (Fig. TMG).

Each pin checks the oracle against something outside itself: the diagonal and
the two-grid cycle against matrices assembled with np.kron (the matrix form of
Sec. 3, built without the oracle's mode products), the smoother's eigenvalue
bound against the generalised eigenvalues of the assembled matrix,
interpolation against exact linear reproduction, and the solvers against a
dense Cholesky solve."""
import numpy as np
import pytest
import scipy.linalg

import oracle
import workload
from oracle import jacobi, multigrid, precond
from oracle.tensor import inner


def _problem(n, lam, seed=0):
    m = tuple((3 * v) // 2 for v in n)
    p = workload.make_problem(n, m, lam, 0.01, seed, 1e-10)
    op = oracle.NormalOperator(p.A, p.D, p.lam)
    return p, op, op.rhs(op.forward(p.X_true) + p.noise)


def _kron_all(mats):
    out = np.ones((1, 1))
    for m in mats:
        out = np.kron(out, m)
    return out


def _dense_normal(G, R, lam):
    """Row-major matrix of N: kron of the G_k plus lam * sum_k I (x) R_k (x) I."""
    n = [g.shape[0] for g in G]
    M = _kron_all(G)
    for k in range(len(n)):
        M = M + lam * _kron_all([R[k] if l == k else np.eye(n[l]) for l in range(len(n))])
    return M


@pytest.mark.parametrize("n,lam", [((5, 4, 6), 1e-2), ((4, 5, 4, 4), 1e-3), ((7, 6), 0.5)])
def test_diagonal_is_main_diagonal_of_assembled_operator(n, lam):
    p, op, _ = _problem(n, lam)
    M = _dense_normal(op.G, op.R, lam)
    assert np.allclose(jacobi.diagonal(op.G, op.R, lam).reshape(-1), np.diag(M), rtol=1e-14, atol=0)
    # and the oracle's own column-by-column assembly agrees
    assert np.allclose(np.diag(oracle.assemble(op, n)), np.diag(M), rtol=1e-13, atol=0)


@pytest.mark.parametrize("n,lam", [((5, 4, 6), 1e-2), ((4, 5, 4, 4), 1e-3), ((6, 6, 6), 1.0),
                                   ((12, 10, 9), 1e-4)])
def test_smoother_bound_covers_the_spectrum(n, lam):
    p, op, _ = _problem(n, lam)
    M = _dense_normal(op.G, op.R, lam)
    d = np.diag(M)
    ev = scipy.linalg.eigh(M, np.diag(d), eigvals_only=True)   # spectrum of D^-1 M
    bound = jacobi.smoother_bound(op.G, op.R, lam)
    assert ev.max() <= bound * (1 + 1e-12)
    # tight when the data term dominates: it is the data term's exact maximum
    data = np.prod([np.linalg.eigvalsh(g / np.sqrt(np.outer(np.diag(g), np.diag(g))))[-1]
                    for g in op.G])
    assert bound >= data * (1 - 1e-12)
    if lam <= 1e-3 and min(n) >= 9:       # data-dominated, away from the tiny-grid edge effects
        assert bound <= 1.05 * ev.max()


def test_jacobi_converges_to_dense_solution_with_damping():
    p, op, B = _problem((5, 4, 6), 1e-2)
    d = jacobi.diagonal(op.G, op.R, p.lam)
    omega = 1.0 / jacobi.smoother_bound(op.G, op.R, p.lam)
    U, it, ok = jacobi.jacobi(op, B, d, omega=omega, rtol=1e-9, max_iter=200000)
    assert ok
    ref = oracle.dense_solve(op, B)
    assert np.linalg.norm(U - ref) <= 1e-6 * np.linalg.norm(ref)
    assert oracle.relative_residual(U, B, op) <= 1e-9


def test_jacobi_exact_in_one_step_for_a_diagonal_operator():
    """Diagonal A_k and no regulariser: N is diagonal, E = N^-1, so the printed
    (undamped) iteration lands on the solution in one step."""
    rng = np.random.default_rng(3)
    n = (4, 3, 5)
    A = [np.diag(rng.uniform(0.5, 2.0, k)) for k in n]
    op = oracle.NormalOperator(A, [np.zeros((1, k)) for k in n], 0.0)
    B = rng.standard_normal(n)
    d = jacobi.diagonal(op.G, op.R, 0.0)
    U, it, ok = jacobi.jacobi(op, B, d, omega=1.0, rtol=1e-14)
    assert ok and it == 1
    assert np.allclose(U, B / d, rtol=1e-15)


def test_undamped_jacobi_diverges_on_the_spline_operator():
    """The printed iteration needs 2 diag(N) - N > 0; the Gram products of
    B-spline collocation violate it (lambda_max(D^-1 N) > 2), so the residual
    grows: the reason for the damping reading."""
    p, op, B = _problem((6, 5, 6), 1e-3)
    M = _dense_normal(op.G, op.R, p.lam)
    assert np.linalg.eigvalsh(2 * np.diag(np.diag(M)) - M).min() < 0
    d = jacobi.diagonal(op.G, op.R, p.lam)
    U, it, ok = jacobi.jacobi(op, B, d, omega=1.0, rtol=1e-8, max_iter=60)
    assert not ok
    r = op(U) - B
    assert np.sqrt(inner(r, r)) > np.sqrt(inner(B, B))


def test_jacobi_preconditioned_cg_matches_dense_solution():
    p, op, B = _problem((6, 5, 4, 4), 1e-3)
    d = jacobi.diagonal(op.G, op.R, p.lam)
    X, it, ok = precond.pcg(op, B, jacobi.precondition(d), rtol=1e-11)
    assert ok
    ref = oracle.dense_solve(op, B)
    kappa = np.linalg.cond(oracle.assemble(op, p.n))
    assert np.linalg.norm(X - ref) <= kappa * 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,nc", [(9, 5), (8, 4), (128, 64), (24, 12), (7, 4)])
def test_interpolation_reproduces_linear_functions(n, nc):
    P = multigrid.interpolation(n, nc)
    xc = np.arange(nc) * (n - 1) / (nc - 1)          # coarse points on the fine index axis
    assert np.allclose(P @ np.ones(nc), np.ones(n), rtol=0, atol=1e-14)
    assert np.allclose(P @ xc, np.arange(n), rtol=0, atol=1e-12)
    assert np.allclose(P @ (3 - 0.5 * xc), 3 - 0.5 * np.arange(n), atol=1e-12)
    assert (P >= 0).all() and (np.count_nonzero(P, axis=1) <= 2).all()
    if (n - 1) % (nc - 1) == 0:                       # nested grids: injection at coarse points
        step = (n - 1) // (nc - 1)
        assert np.array_equal(P[::step], np.eye(nc))


def test_restriction_is_transpose_of_prolongation():
    P = [multigrid.interpolation(n, nc) for n, nc in [(8, 4), (9, 5), (6, 3)]]
    rng = np.random.default_rng(4)
    f = rng.standard_normal((8, 9, 6))
    c = rng.standard_normal((4, 5, 3))
    # <R f, c> = <f, P c> for every pair: the maps are adjoint
    assert np.isclose(inner(multigrid.restrict(f, P), c), inner(f, multigrid.prolong(c, P)),
                      rtol=1e-13)
    # and both equal the Kronecker matrices (row-major vec)
    K = _kron_all(P)
    assert np.allclose(multigrid.prolong(c, P).reshape(-1), K @ c.reshape(-1), atol=1e-13)
    assert np.allclose(multigrid.restrict(f, P).reshape(-1), K.T @ f.reshape(-1), atol=1e-13)


def test_coarse_data_term_is_galerkin():
    p, op, _ = _problem((10, 9, 8), 1e-3)
    scales, _ = multigrid.build_scales(p.A, p.D, p.lam, coarse_max=100)
    assert len(scales) >= 2
    P = scales[0].P
    for k in range(3):
        assert np.allclose(scales[1].op.G[k], P[k].T @ op.G[k] @ P[k], rtol=1e-13, atol=1e-13)
    # the lumped regulariser: s_k^2 R-image with s_k^2 = prod_{l != k} n_l / n_c,l
    n, nc = op.shape, scales[1].op.shape
    for k in range(3):
        s2 = np.prod([n[l] / nc[l] for l in range(3) if l != k])
        assert np.allclose(scales[1].op.R[k], s2 * P[k].T @ op.R[k] @ P[k], rtol=1e-12, atol=1e-14)


def test_two_grid_cycle_equals_dense_two_grid_operator():
    """Two scales: the tensor V-cycle equals the matrix two-grid cycle built
    from np.kron matrices -- smoothing with omega D^-1, restriction K^T,
    coarse solve with the assembled coarse matrix, prolongation K."""
    p, op, _ = _problem((8, 9, 6), 1e-2)
    scales, chol = multigrid.build_scales(p.A, p.D, p.lam, max_levels=2, coarse_max=50)
    assert len(scales) == 2
    f, c = scales
    Mf = _dense_normal(f.op.G, f.op.R, p.lam)
    Mc = _dense_normal(c.op.G, c.op.R, p.lam)
    K = _kron_all(f.P)
    S = f.omega / np.diag(Mf)
    r = np.random.default_rng(5).standard_normal(op.shape)
    for nu in (1, 2):
        x = np.zeros(r.size)
        b = r.reshape(-1)
        for _ in range(nu):
            x = x + S * (b - Mf @ x)
        x = x + K @ np.linalg.solve(Mc, K.T @ (b - Mf @ x))
        for _ in range(nu):
            x = x + S * (b - Mf @ x)
        z = multigrid.vcycle(scales, chol, 0, np.zeros(op.shape), r, nu)
        assert np.allclose(z.reshape(-1), x, rtol=1e-11, atol=1e-11 * np.abs(x).max())


def test_vcycle_preconditioner_is_symmetric_positive_definite():
    p, op, _ = _problem((16, 8, 8), 1e-3)
    scales, chol = multigrid.build_scales(p.A, p.D, p.lam, coarse_max=40)
    assert len(scales) >= 3
    V = oracle.assemble(multigrid.preconditioner(scales, chol), op.shape)
    assert np.allclose(V, V.T, rtol=0, atol=1e-12 * np.abs(V).max())
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0


def test_vcycle_solver_and_preconditioned_cg_converge():
    p, op, B = _problem((16, 12, 10, 8), 1e-3)
    scales, chol = multigrid.build_scales(p.A, p.D, p.lam, coarse_max=200)
    assert len(scales) >= 3
    # Fig. TMG as a stationary solver: repeated cycles contract the error
    C = np.zeros_like(B)
    norms = []
    for _ in range(6):
        C = multigrid.vcycle(scales, chol, 0, C, B, nu=2)
        norms.append(oracle.relative_residual(C, B, op))
    assert all(b < a for a, b in zip(norms, norms[1:]))
    # as a CG preconditioner it reaches the dense solution and cuts iterations
    X, it, ok = precond.pcg(op, B, multigrid.preconditioner(scales, chol, nu=2), rtol=1e-10)
    assert ok and oracle.relative_residual(X, B, op) <= 1e-10
    plain = oracle.cg(op, B, rtol=1e-10)
    assert it < plain.iters
    ref = oracle.dense_solve(op, B) if np.prod(p.n) <= 4096 else None
    if ref is not None:
        assert np.linalg.norm(X - ref) <= 1e-6 * np.linalg.norm(ref)
