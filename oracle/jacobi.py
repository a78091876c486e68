"""Tensor Jacobi: the main diagonal of the normal operator, the stationary
Jacobi iteration and the diagonal preconditioner (oracle; test infrastructure
only).

Fig. Tensor_Jacobi (Sec. 4.1) iterates U <- U - E (N U - B), where E is the
inverse of the diagonal tensor formed from the main diagonal of the system
tensor.  For N(X) = X x_1 G_1 ... x_N G_N + lam sum_k X x_k R_k the entry of
that diagonal at multi-index (i_1, ..., i_N) is

    d[i] = prod_k G_k[i_k, i_k] + lam * sum_k R_k[i_k, i_k],

because the Kronecker product's diagonal is the product of the factors'
diagonals and a Kronecker-sum term I (x) .. R_k .. (x) I contributes R_k's
diagonal along mode k.  It is built from the N per-mode diagonals, so it costs
O(sum n_k) numbers to describe.

Readings:
* The printed iteration has no damping.  Plain Jacobi converges only when
  2 diag(N) - N is positive definite, which the B-spline Gram products do not
  satisfy, so a damping weight omega multiplies the update
  (U <- U - omega E (N U - B)); omega = 1 is the printed form.
* The loop test compares <R, R> with a threshold; as for CG the threshold is
  relative, ||R|| <= rtol ||B||.
* The diagonal preconditioner of CG applies z = E r (elementwise).
"""
import numpy as np

from .tensor import inner


def diagonal(G, R, lam):
    """Main diagonal of N as a tensor (float64)."""
    order = len(G)
    shape = tuple(np.asarray(g).shape[0] for g in G)
    prod = np.ones(shape)
    for k, g in enumerate(G):
        view = [1] * order
        view[k] = shape[k]
        prod = prod * np.diag(np.asarray(g, dtype=np.float64)).reshape(view)
    total = prod
    for k, r in enumerate(R):
        if r is None:
            continue
        view = [1] * order
        view[k] = shape[k]
        total = total + lam * np.diag(np.asarray(r, dtype=np.float64)).reshape(view)
    return total


def _scaled_lambda_max(M):
    """Largest eigenvalue of diag(M)^-1/2 M diag(M)^-1/2 over the rows with a
    nonzero diagonal (M symmetric positive semidefinite)."""
    M = np.asarray(M, dtype=np.float64)
    d = np.diag(M)
    keep = d > 0
    if not np.any(keep):
        return 0.0
    s = 1.0 / np.sqrt(d[keep])
    S = M[np.ix_(keep, keep)] * s[:, None] * s[None, :]
    return float(np.linalg.eigvalsh(S)[-1])


def smoother_bound(G, R, lam):
    """Upper bound of the largest eigenvalue of diag(N)^-1 N.

    With g_k = diag(G_k) and r_k = diag(R_k), the data term satisfies
    x^T (x G_k) x <= mu_d x^T (x g_k) x with mu_d = prod_k lambda_max(g_k^-1/2
    G_k g_k^-1/2) (the eigenvalues of a Kronecker product of PSD matrices are
    the products of the factors'), and each regulariser term
    x^T (I .. R_k .. I) x <= mu_k x^T (I .. r_k .. I) x with
    mu_k = lambda_max(r_k^-1/2 R_k r_k^-1/2).  Adding up,
    x^T N x <= max(mu_d, max_k mu_k) x^T diag(N) x."""
    data = 1.0
    for g in G:
        data *= _scaled_lambda_max(g)
    reg = 0.0
    if lam > 0:
        for r in R:
            if r is not None:
                reg = max(reg, _scaled_lambda_max(r))
    return max(data, reg)


def jacobi(apply, B, diag, omega=1.0, rtol=1e-8, max_iter=10000, x0=None):
    """Stationary tensor Jacobi of Fig. Tensor_Jacobi with damping omega.

    Returns (U, iterations, converged)."""
    B = np.asarray(B, dtype=np.float64)
    U = np.zeros_like(B) if x0 is None else np.array(x0, dtype=np.float64)
    threshold = rtol * rtol * inner(B, B)
    Rt = apply(U) - B
    it = 0
    while inner(Rt, Rt) > threshold:
        if it == max_iter:
            return U, it, False
        U = U - omega * Rt / diag
        Rt = apply(U) - B
        it += 1
    return U, it, True


def precondition(diag):
    """z = E r: the diagonal preconditioner as a callable."""
    inv = 1.0 / np.asarray(diag, dtype=np.float64)
    return lambda r: np.asarray(r, dtype=np.float64) * inv
