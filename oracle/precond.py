"""Tensor-inverse preconditioner and preconditioned CG (oracle; test
infrastructure only).

The separable part of the normal operator, X ×_1 G_1 ⋯ ×_N G_N, has the
tensor inverse X ×_1 G_1⁻¹ ⋯ ×_N G_N⁻¹ (Sec. 3: the inverse of a separable
system is applied mode by mode).  The preconditioner replaces each G_k by
G_k + c R_k, which keeps it separable and SPD for c >= 0:

    M⁻¹(R) = R ×_1 (G_1 + c R_1)⁻¹ ⋯ ×_N (G_N + c R_N)⁻¹.

With λ = 0 and c = 0 it is the exact inverse of N.  The preconditioned CG is
the textbook one (Hestenes and Stiefel with a preconditioner): the paper's CG
of Fig. Tensor_CG with the search direction built from z = M⁻¹ r and the
step lengths from <r, z>.  Everything is float64 NumPy.
"""
import numpy as np

from .tensor import inner, multi_mode_product


def inverse_factors(G, R, c):
    """(G_k + c R_k)⁻¹ for every mode (R_k may be None: no regulariser)."""
    out = []
    for k, g in enumerate(G):
        m = np.array(g, dtype=np.float64)
        if R[k] is not None:
            m = m + c * np.asarray(R[k], dtype=np.float64)
        out.append(np.linalg.inv(m))
    return out


def apply(Rt, inv):
    """M⁻¹(Rt): the mode products of Rt with the inverse factors."""
    return multi_mode_product(np.asarray(Rt, dtype=np.float64), inv)


def pcg(apply_n, B, apply_m, rtol=1e-8, max_iter=10000, x0=None):
    """Preconditioned CG for apply_n(X) = B; returns (X, iterations, converged).

    Stops when ||r||_2 <= rtol ||B||_2 (the same relative test as the
    unpreconditioned iteration)."""
    B = np.asarray(B, dtype=np.float64)
    X = np.zeros_like(B) if x0 is None else np.array(x0, dtype=np.float64)
    r = B - apply_n(X)
    thr = rtol * rtol * inner(B, B)
    if inner(r, r) <= thr:
        return X, 0, True
    z = apply_m(r)
    p = z.copy()
    rz = inner(r, z)
    for it in range(1, max_iter + 1):
        q = apply_n(p)
        alpha = rz / inner(p, q)
        X = X + alpha * p
        r = r - alpha * q
        if inner(r, r) <= thr:
            return X, it, True
        z = apply_m(r)
        rz1 = inner(r, z)
        p = z + (rz1 / rz) * p
        rz = rz1
    return X, max_iter, False
