"""Regularised normal operator and right-hand side (oracle; test infrastructure only).

The tensor equation (Sec. 3) for a separable forward model with per-mode
factors A_k (eq. separable_transf) and the normal-equation pattern A^T A of
App. A.7 give the operator

    N(X) = X x_1 G_1 ... x_N G_N  +  lam * sum_k X x_k R_k,
    G_k = A_k^T A_k,   R_k = D_k^T D_k,

and the right-hand side B = Y x_1 A_1^T ... x_N A_N^T.  The regulariser is a
sum of one 1-D transformation per mode, the Kronecker-sum form Sec. 4.1 gives
for the discrete Poisson equation.  D_k is a 1-D finite difference (Table 1).
The operator is symmetric positive definite when every A_k has full column rank
and lam >= 0 (Gram and regulariser factors are positive (semi)definite).
"""
import numpy as np

from .tensor import mode_product


def gram(A):
    """G = A^T A (n x n) in float64."""
    A = np.asarray(A, dtype=np.float64)
    return A.T @ A


def reg_factor(D):
    """R = D^T D (n x n) in float64."""
    D = np.asarray(D, dtype=np.float64)
    return D.T @ D


def forward(X, A):
    """Y = X x_1 A_1 ... x_N A_N (the separable forward model)."""
    Y = np.asarray(X, dtype=np.float64)
    for k, Ak in enumerate(A):
        Y = mode_product(Y, Ak, k)
    return Y


def rhs(Y, A):
    """B = Y x_1 A_1^T ... x_N A_N^T (App. A.7 applied to the data term)."""
    B = np.asarray(Y, dtype=np.float64)
    for k, Ak in enumerate(A):
        B = mode_product(B, np.asarray(Ak, dtype=np.float64).T, k)
    return B


def regulariser_apply(X, R, lam):
    """lam * sum_k X x_k R_k (Kronecker sum, Sec. 4.1)."""
    X = np.asarray(X, dtype=np.float64)
    out = np.zeros_like(X)
    for k, Rk in enumerate(R):
        out += mode_product(X, Rk, k)
    return lam * out


def normal_apply(X, G, R, lam):
    """N(X) in the Gram form: chain of G_k plus the regulariser."""
    X = np.asarray(X, dtype=np.float64)
    T = X
    for k, Gk in enumerate(G):
        T = mode_product(T, Gk, k)
    return T + regulariser_apply(X, R, lam)


def normal_apply_literal(X, A, D, lam):
    """N(X) formed literally: forward model, then its transpose; same for D_k.

    (X x_k A_k)_k followed by x_k A_k^T, plus lam * sum_k (X x_k D_k) x_k D_k^T.
    Equal to ``normal_apply`` by the mixed-product property of mode products.
    """
    X = np.asarray(X, dtype=np.float64)
    T = rhs(forward(X, A), A)
    reg = np.zeros_like(X)
    for k, Dk in enumerate(D):
        Dk = np.asarray(Dk, dtype=np.float64)
        reg += mode_product(mode_product(X, Dk, k), Dk.T, k)
    return T + lam * reg


class NormalOperator:
    """Callable N(.) for per-mode factors A_k, D_k and weight lam."""

    def __init__(self, A, D, lam):
        self.A = [np.asarray(a, dtype=np.float64) for a in A]
        self.D = [np.asarray(d, dtype=np.float64) for d in D]
        self.lam = float(lam)
        self.G = [gram(a) for a in self.A]
        self.R = [reg_factor(d) for d in self.D]
        self.shape = tuple(a.shape[1] for a in self.A)

    def __call__(self, X):
        return normal_apply(X, self.G, self.R, self.lam)

    def rhs(self, Y):
        return rhs(Y, self.A)

    def forward(self, X):
        return forward(X, self.A)
