"""FP64 residual judge (oracle; test infrastructure only).

Any solution X, whatever produced it, is judged by the relative residual of the
normal equations, ||B - N(X)||_2 / ||B||_2, computed in float64.
"""
import numpy as np

from .tensor import inner


def relative_residual(X, B, apply):
    B = np.asarray(B, dtype=np.float64)
    R = B - apply(np.asarray(X, dtype=np.float64))
    bn = np.sqrt(inner(B, B))
    return float(np.sqrt(inner(R, R)) / (bn if bn > 0 else 1.0))
