"""Scattered-measurement forward operator (oracle; test infrastructure only).

Sec. 6: the application samples a spline field at scattered points.  The
measurement at site t^i = (t^i_1, .., t^i_N) is the field's value there, so
row i of the system matrix is the product of one basis row per mode,

    a_i = b^i_1 (x) b^i_2 (x) ... (x) b^i_N,    b^i_k[j] = B_j(t^i_k),

the repeated-index (Khatri-Rao) product of Sec. 2.2 taken over the sample
index i.  The normal operator is the rank-S CANDECOMP sum of Sec. 6,

    N(X) = sum_i a_i <a_i, X>  +  lam * sum_k X x_k R_k,   R_k = D_k^T D_k,

which is applied matrix-free: neither N nor its CP factors are stored, only
the sites.  The basis is the one of the grid problems (cubic, clamped uniform
knots on [0, 1], n_k functions per mode); a cubic basis row has at most four
non-zero entries, at consecutive indices, so each sample touches a 4^N block
of coefficients.

Every routine is plain float64 NumPy without blocking or fusion beyond the
definitions above.  Samples are processed in chunks only to bound memory.
"""
import numpy as np

from .normal import regulariser_apply, reg_factor

DEGREE = 3
WIDTH = DEGREE + 1
_CHUNK = 32768


def knots(n):
    """Clamped uniform knot vector of ``n`` cubic basis functions on [0, 1]."""
    inner = np.linspace(0.0, 1.0, n - DEGREE + 1)
    return np.concatenate([np.zeros(DEGREE), inner, np.ones(DEGREE)])


def basis_window(t, n):
    """Non-zero basis values of one mode at the points ``t``.

    Returns (first, w): ``first`` (S,) int64 is the index of the first of the
    four functions that can be non-zero at t, ``w`` (S, 4) float64 their
    values.  The knot span holding t is the last span [u_s, u_{s+1}) with
    u_s <= t (the right end point t = 1 belongs to the last non-empty span);
    the values come from the Cox-de Boor recursion (de Boor, 1972) raised one
    degree at a time on that span: B_{j,p} = (t - u_j)/(u_{j+p} - u_j) B_{j,p-1}
    + (u_{j+p+1} - t)/(u_{j+p+1} - u_{j+1}) B_{j+1,p-1}.
    """
    t = np.asarray(t, dtype=np.float64).reshape(-1)
    u = knots(n)
    # span index s in [DEGREE, n-1]: u[s] <= t < u[s+1]
    s = np.searchsorted(u, t, side="right") - 1
    s = np.clip(s, DEGREE, n - 1)
    # degree 0: only B_{s,0} = 1 on the span; keep the functions s-p .. s
    B = np.ones((t.size, 1))
    for p in range(1, DEGREE + 1):
        nb = np.zeros((t.size, p + 1))
        for r in range(p + 1):
            j = s - p + r  # function B_{j,p}
            if r > 0:
                # left term uses B_{j,p-1} = B[:, r-1]
                den = u[j + p] - u[j]
                nb[:, r] += np.where(den > 0, (t - u[j]) / np.where(den > 0, den, 1.0), 0.0) * B[:, r - 1]
            if r < p:
                # right term uses B_{j+1,p-1} = B[:, r]
                den = u[j + p + 1] - u[j + 1]
                nb[:, r] += np.where(den > 0, (u[j + p + 1] - t) / np.where(den > 0, den, 1.0), 0.0) * B[:, r]
        B = nb
    return s - DEGREE, B


def sample_rows(coords, n):
    """Per-mode (first, w) windows of every site; ``coords`` is (N, S)."""
    coords = np.asarray(coords, dtype=np.float64)
    if coords.shape[0] != len(n):
        raise ValueError("coords must have one row per mode")
    return [basis_window(coords[k], int(n[k])) for k in range(len(n))]


def _block_index(rows, lo, hi):
    """Broadcast index arrays of the 4^N coefficient blocks of samples lo..hi."""
    N = len(rows)
    idx = []
    for k, (first, _) in enumerate(rows):
        shape = [hi - lo] + [1] * N
        shape[1 + k] = WIDTH
        idx.append((first[lo:hi, None] + np.arange(WIDTH)[None, :]).reshape(shape))
    return tuple(idx)


def _weights(rows, lo, hi):
    """(chunk, 4, .., 4) outer product of the per-mode weights: the non-zero block of a_i."""
    N = len(rows)
    W = np.ones([hi - lo] + [1] * N)
    for k, (_, w) in enumerate(rows):
        shape = [hi - lo] + [1] * N
        shape[1 + k] = WIDTH
        W = W * w[lo:hi].reshape(shape)
    return W


def forward(X, coords, rows=None):
    """f_i = <a_i, X> for every site (the measurement model)."""
    X = np.asarray(X, dtype=np.float64)
    rows = rows or sample_rows(coords, X.shape)
    S = rows[0][0].size
    f = np.empty(S)
    axes = tuple(range(1, X.ndim + 1))
    for lo in range(0, S, _CHUNK):
        hi = min(S, lo + _CHUNK)
        blk = X[_block_index(rows, lo, hi)]
        f[lo:hi] = np.sum(blk * _weights(rows, lo, hi), axis=axes)
    return f


def adjoint(y, coords, n, rows=None):
    """sum_i y_i a_i (the transposed measurement model, App. A.7)."""
    n = tuple(int(v) for v in n)
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    rows = rows or sample_rows(coords, n)
    B = np.zeros(n)
    S = rows[0][0].size
    for lo in range(0, S, _CHUNK):
        hi = min(S, lo + _CHUNK)
        W = _weights(rows, lo, hi) * y[lo:hi].reshape([hi - lo] + [1] * len(n))
        idx = tuple(np.broadcast_to(i, W.shape) for i in _block_index(rows, lo, hi))
        np.add.at(B, idx, W)
    return B


class ScatteredOperator:
    """N(X) = sum_i a_i <a_i, X> + lam * sum_k X x_k R_k for sites ``coords``."""

    def __init__(self, coords, n, D, lam):
        self.n = tuple(int(v) for v in n)
        self.coords = np.asarray(coords)
        self.rows = sample_rows(self.coords, self.n)
        self.lam = float(lam)
        self.R = [reg_factor(d) for d in D] if D is not None else [np.zeros((k, k)) for k in self.n]
        self.shape = self.n

    def forward(self, X):
        return forward(X, self.coords, self.rows)

    def rhs(self, y):
        return adjoint(y, self.coords, self.n, self.rows)

    def __call__(self, X):
        X = np.asarray(X, dtype=np.float64)
        return adjoint(forward(X, self.coords, self.rows), self.coords, self.n, self.rows) + \
            regulariser_apply(X, self.R, self.lam)
