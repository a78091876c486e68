"""Tensor multigrid V-cycle (oracle; test infrastructure only).

Fig. TMG (Sec. 4.2): on every scale but the last, the V-cycle smooths the
current solution, restricts the residual B - N C to the next scale with one
matrix per mode (a separable restriction), solves there by the V-cycle from a
zero start, adds the separable prolongation of that correction, and smooths
again; on the last scale it solves directly.  GetScale supplies each scale's
system and its per-mode restriction and prolongation matrices.

Readings where the figure leaves the method open:

* Prolongation along mode k (n_k -> n_c coefficients) is linear interpolation
  from a uniform coarse grid over the same index interval: fine index i sits at
  coarse coordinate x = i (n_c - 1) / (n_k - 1) and takes weights 1 - (x - J)
  and x - J from coarse points J = floor(x) and J + 1.  Its columns sum to
  partition-of-unity rows (P 1 = 1).  A mode is coarsened to
  n_c = ceil(n_k / 2) while n_k >= 2 * min_extent, else kept (P = I).
* Restriction is the transpose of prolongation, so the cycle is symmetric.
* GetScale forms the next scale's system from the same parts as the fine one:
  collocation factors A_k P_k and regulariser factors s_k D_k P_k with the same
  lambda.  The data term is then exactly the Galerkin product
  P^T (x G_k) P = (x) P_k^T G_k P_k.  In the regulariser's Kronecker sum the
  identity factors I_l of the other modes would become P_l^T P_l; they are
  lumped to (n_l / n_c,l) I (the row sums of P_l^T P_l average n_l / n_c,l
  since P_l 1 = 1), which is folded into s_k^2 = prod_{l != k} n_l / n_c,l.
  Every scale is thus an operator of the fine one's form.
* Scales are added while the coarse size exceeds `coarse_max` unknowns and
  some mode can still be coarsened, up to `max_levels` scales in all.
* Presmooth and Postsmooth are `nu` sweeps of damped Jacobi (Fig.
  Tensor_Jacobi) C <- C + omega diag(N)^-1 (B - N C), with
  omega = omega_scale / g, g an upper bound of the largest eigenvalue of
  diag(N)^-1 N formed from per-mode eigenvalues (jacobi.smoother_bound), so
  omega * lambda_max <= omega_scale < 2 and the smoother converges.
* DirectSolve is a Cholesky solve of the last scale's assembled matrix.
* As a preconditioner of CG one V-cycle is applied to the residual from a
  zero start: z = V(r).
"""
from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.linalg

from .dense import assemble
from .jacobi import diagonal, smoother_bound
from .normal import NormalOperator
from .tensor import multi_mode_product


def interpolation(n, nc):
    """Linear interpolation matrix (n x nc) from nc uniform coarse points."""
    if nc == n:
        return np.eye(n)
    if nc < 2 or n < 2:
        raise ValueError("interpolation needs at least two points on each grid")
    P = np.zeros((n, nc))
    for i in range(n):
        x = i * (nc - 1) / (n - 1)
        J = min(int(np.floor(x)), nc - 2)
        w = x - J
        P[i, J] += 1.0 - w
        P[i, J + 1] += w
    return P


@dataclass
class Scale:
    op: NormalOperator
    diag: np.ndarray
    omega: float
    P: List[np.ndarray]          # prolongation to this scale from the next one (per mode)


def coarse_extents(n, min_extent=4):
    return tuple((v + 1) // 2 if v >= 2 * min_extent else v for v in n)


def build_scales(A, D, lam, max_levels=8, coarse_max=2048, min_extent=4, omega_scale=1.5):
    """GetScale for every scale: list of Scale (fine first) and the last
    scale's Cholesky factor."""
    A = [np.asarray(a, dtype=np.float64) for a in A]
    D = [np.asarray(d, dtype=np.float64) for d in D]
    scales = []
    while True:
        op = NormalOperator(A, D, lam)
        n = op.shape
        nc = coarse_extents(n, min_extent)
        last = (len(scales) + 1 == max_levels or int(np.prod(n)) <= coarse_max or nc == n)
        d = diagonal(op.G, op.R, lam)
        omega = omega_scale / smoother_bound(op.G, op.R, lam)
        if last:
            scales.append(Scale(op, d, omega, []))
            break
        P = [interpolation(a, b) for a, b in zip(n, nc)]
        ratio = [a / b for a, b in zip(n, nc)]
        scales.append(Scale(op, d, omega, P))
        A = [a @ p for a, p in zip(A, P)]
        D = [np.sqrt(np.prod([ratio[l] for l in range(len(n)) if l != k])) * (d_k @ P[k])
             for k, d_k in enumerate(D)]
    last = scales[-1]
    M = assemble(last.op, last.op.shape)
    chol = scipy.linalg.cho_factor(M)
    return scales, chol


def restrict(Rt, P):
    """Separable restriction: Rt x_k P_k^T on every mode."""
    return multi_mode_product(Rt, [p.T for p in P])


def prolong(Cc, P):
    """Separable prolongation: Cc x_k P_k on every mode."""
    return multi_mode_product(Cc, P)


def smooth(scale, C, B, nu):
    for _ in range(nu):
        C = C + scale.omega * (B - scale.op(C)) / scale.diag
    return C


def vcycle(scales, chol, level, C, B, nu=1):
    """One V-cycle of Fig. TMG on scale `level` for N_level(C) = B."""
    s = scales[level]
    if level == len(scales) - 1:
        return scipy.linalg.cho_solve(chol, np.asarray(B, dtype=np.float64).reshape(-1)
                                      ).reshape(B.shape)
    C = smooth(s, C, B, nu)
    Bc = restrict(B - s.op(C), s.P)
    Cc = vcycle(scales, chol, level + 1, np.zeros_like(Bc), Bc, nu)
    C = C + prolong(Cc, s.P)
    return smooth(s, C, B, nu)


def preconditioner(scales, chol, nu=1):
    """z = V(r): one V-cycle from zero on the residual."""
    return lambda r: vcycle(scales, chol, 0, np.zeros_like(r), np.asarray(r, dtype=np.float64), nu)
