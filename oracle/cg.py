"""Tensor conjugate gradients in FP64 (oracle; test infrastructure only).

The solver of Fig. Tensor_CG (Sec. 4.1) is conjugate gradients written with
tensor operations only: the operator is applied as a tensor multiplication,
every scalar comes from a full contraction <U, V> (App. A.6), and the Kronecker
delta that relabels the direction's indices before the multiplication (App.
A.5) leaves every component unchanged, so it is the identity here.  This module
follows the textbook method: from the residual of the current iterate, each
step moves the iterate along a search direction by the step length that
minimises the energy norm of the error, updates the residual with the
operator's image of the direction, and makes the next direction conjugate to
the previous one with the ratio of successive squared residual norms.

Readings where the figure is silent or garbled:

* Its loop test reads as if the loop ended while the squared residual is still
  large, which would stop after one pass; the loop instead runs until the
  squared residual is at or below the threshold, the test of the Jacobi solver
  in Fig. Tensor_Jacobi.
* The threshold is relative to the right-hand side: ||r|| <= rtol ||B||, so
  that solutions from any starting tensor are judged against the same B.
* No step is taken when the starting residual already meets the threshold
  (a zero right-hand side returns the start unchanged).
* A curvature <d, N d> <= 0 or a non-finite scalar is a breakdown (the
  operator is not SPD).
* When the loop ends on the threshold, the residual is recomputed from the
  iterate; if that true residual misses the tolerance, the iteration starts
  over once from the current iterate.

Storage model (the paper does not fix the precision): with ``store`` given
(e.g. numpy.float32) the iterate, residual, direction and the operator's image
are rounded to that type each time they are formed, while every inner product
and scalar stays FP64.  This is the arithmetic of a solver that keeps its
vectors in FP32 and reduces in FP64; it lets iteration counts of such a solver
be compared with the same recurrence under the same rounding.  The default
(no ``store``) is plain FP64.
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


@dataclass
class _Log:
    steps: List[float] = field(default_factory=list)      # step lengths
    ratios: List[float] = field(default_factory=list)     # conjugation ratios
    res2: List[float] = field(default_factory=list)       # squared residual norms


def _sweep(apply, rhs, x, tol2, budget, log, keep):
    """CG from iterate x for at most `budget` steps; `keep` rounds a vector to
    the storage type.

    Returns (x, steps taken, status, last squared residual norm)."""
    res = keep(rhs - apply(x))
    res2 = inner(res, res)
    log.res2.append(res2)
    if res2 <= tol2:
        return x, 0, CONVERGED, res2
    direction = res.copy()
    taken = 0
    while taken < budget:
        image = keep(apply(direction))
        curvature = inner(direction, image)
        if not np.isfinite(curvature) or curvature <= 0.0:
            return x, taken, BREAKDOWN, res2
        step = res2 / curvature
        x = keep(x + step * direction)
        res = keep(res - step * image)
        res2_next = inner(res, res)
        ratio = res2_next / res2
        direction = keep(res + ratio * direction)
        res2 = res2_next
        taken += 1
        log.steps.append(step)
        log.ratios.append(ratio)
        log.res2.append(res2)
        if not np.isfinite(res2):
            return x, taken, BREAKDOWN, res2
        if res2 <= tol2:
            return x, taken, CONVERGED, res2
    return x, taken, NOT_CONVERGED, res2


def _true_relative_residual(apply, rhs, x, scale):
    res = rhs - apply(x)
    return float(np.sqrt(inner(res, res)) / scale)


def cg(apply: Callable, B, x0: Optional[np.ndarray] = None, rtol=1e-8,
       max_iter=10000, restart=True, store=None) -> CGResult:
    """Solve apply(X) = B by tensor CG (Fig. Tensor_CG) in float64 (vectors
    rounded to `store` when given, see the storage model above)."""
    if store is None:
        keep = lambda v: v  # noqa: E731
    else:
        keep = lambda v: np.asarray(v).astype(store).astype(np.float64)  # noqa: E731
    rhs = keep(np.asarray(B, dtype=np.float64))
    x = np.zeros_like(rhs) if x0 is None else keep(np.array(x0, dtype=np.float64))
    bnorm = np.sqrt(inner(rhs, rhs))
    scale = bnorm if bnorm > 0 else 1.0
    tol2 = (rtol * bnorm) ** 2
    log = _Log()
    x, taken, status, res2 = _sweep(apply, rhs, x, tol2, max_iter, log, keep)
    restarts = 0
    true_rel = _true_relative_residual(apply, rhs, x, scale)
    if restart and status == CONVERGED and true_rel > rtol and taken < max_iter:
        restarts = 1
        x, more, status, res2 = _sweep(apply, rhs, x, tol2, max_iter - taken, log, keep)
        taken += more
        true_rel = _true_relative_residual(apply, rhs, x, scale)
    if status == CONVERGED and true_rel > rtol:
        status = NOT_CONVERGED
    return CGResult(x=x, iters=taken, status=status,
                    rel_res_recursive=float(np.sqrt(max(res2, 0.0)) / scale),
                    rel_res_true=true_rel, alphas=log.steps, betas=log.ratios,
                    rho_history=log.res2, restarts=restarts)


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
