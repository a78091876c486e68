"""Tensor conjugate gradients (oracle; test infrastructure only).

The iteration is the one of Fig. Tensor_CG, in its order and notation
(C is the solution tensor, R the residual, P the search direction, Q = A*P):

    R = B - A*C ;  P = R ;  rho = <R, R>
    repeat
        Q     = A*P
        alpha = rho / <P, Q>
        C     = C + alpha * P
        R     = R - alpha * Q
        rho1  = <R, R>
        P     = R + (rho1 / rho) * P
        rho   = rho1
    until convergence

The Kronecker-delta relabelling of the figure (P*D) changes no component value
(App. A.5), so it is the identity here.  Readings where the figure is silent or
garbled:

* the printed loop test reads "until rho > threshold", which would stop after
  one pass; it is read as "until rho <= threshold", the test the Jacobi solver
  of Fig. Tensor_Jacobi uses;
* the threshold is relative: rho <= (rtol * ||B||)^2, so that solutions from
  any starting tensor are judged against the same right-hand side;
* the loop is entered only when the initial residual is above the threshold
  (a zero right-hand side returns C unchanged);
* <P, Q> <= 0 or a non-finite scalar is a breakdown (the operator is not SPD);
* after the loop the true residual ||B - A*C|| is recomputed; if it is above
  the tolerance the iteration restarts once from it.
"""
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from .tensor import inner

CONVERGED = 0
NOT_CONVERGED = 1
BREAKDOWN = -6


@dataclass
class CGResult:
    x: np.ndarray
    iters: int
    status: int
    rel_res_recursive: float
    rel_res_true: float
    alphas: List[float] = field(default_factory=list)
    betas: List[float] = field(default_factory=list)
    rho_history: List[float] = field(default_factory=list)
    restarts: int = 0


def _cg_pass(apply, B, C, threshold, max_iter, hist):
    R = B - apply(C)
    P = R.copy()
    rho = inner(R, R)
    hist["rho"].append(rho)
    it = 0
    status = NOT_CONVERGED
    if rho <= threshold:
        return C, it, CONVERGED, rho
    while it < max_iter:
        Q = apply(P)
        pq = inner(P, Q)
        if not np.isfinite(pq) or pq <= 0.0:
            status = BREAKDOWN
            break
        alpha = rho / pq
        C = C + alpha * P
        R = R - alpha * Q
        rho1 = inner(R, R)
        beta = rho1 / rho
        P = R + beta * P
        rho = rho1
        it += 1
        hist["alpha"].append(alpha)
        hist["beta"].append(beta)
        hist["rho"].append(rho)
        if not np.isfinite(rho):
            status = BREAKDOWN
            break
        if rho <= threshold:
            status = CONVERGED
            break
    return C, it, status, rho


def cg(apply: Callable, B, x0: Optional[np.ndarray] = None, rtol=1e-8,
       max_iter=10000, restart=True) -> CGResult:
    """Solve apply(X) = B by the tensor CG of Fig. Tensor_CG in float64."""
    B = np.asarray(B, dtype=np.float64)
    C = np.zeros_like(B) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.sqrt(inner(B, B))
    threshold = (rtol * bnorm) ** 2
    hist = {"alpha": [], "beta": [], "rho": []}
    C, it, status, rho = _cg_pass(apply, B, C, threshold, max_iter, hist)
    total = it
    restarts = 0
    denom = bnorm if bnorm > 0 else 1.0
    true_res = np.sqrt(inner(B - apply(C), B - apply(C))) / denom
    if restart and status == CONVERGED and true_res > rtol and total < max_iter:
        restarts = 1
        C, it, status, rho = _cg_pass(apply, B, C, threshold, max_iter - total, hist)
        total += it
        R = B - apply(C)
        true_res = np.sqrt(inner(R, R)) / denom
    if status == CONVERGED and true_res > rtol:
        status = NOT_CONVERGED
    return CGResult(x=C, iters=total, status=status,
                    rel_res_recursive=float(np.sqrt(max(rho, 0.0)) / denom),
                    rel_res_true=float(true_res), alphas=hist["alpha"],
                    betas=hist["beta"], rho_history=hist["rho"], restarts=restarts)


def lanczos_extremes(alphas, betas):
    """Extreme Ritz values of the operator from the CG coefficients.

    CG's coefficients define the Lanczos tridiagonal matrix T with
    T[i,i] = 1/alpha_i + beta_{i-1}/alpha_{i-1} and T[i,i+1] = sqrt(beta_i)/alpha_i
    (textbook CG-Lanczos relation); its extreme eigenvalues approximate those of
    the operator, so max/min estimates the condition number.
    """
    a = np.asarray(alphas, dtype=np.float64)
    b = np.asarray(betas, dtype=np.float64)
    k = len(a)
    if k == 0:
        raise ValueError("no CG iterations")
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = 1.0 / a[i] + (b[i - 1] / a[i - 1] if i > 0 else 0.0)
        if i + 1 < k:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(b[i]) / a[i]
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])
