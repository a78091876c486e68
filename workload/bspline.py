"""Problem-input matrices: cubic B-spline collocation and second differences.

The paper's application (Sec. 6) is a spline-based variational reconstruction;
the per-mode factors of such a problem are a spline collocation matrix A_k and a
finite-difference regulariser D_k (Table 1 lists finite differences as a
separable building block).  The paper does not fix the spline basis, so the
choice made here is a reading: degree 3, clamped (open) uniform knots on [0, 1],
``n`` basis functions, sampled at ``m`` equispaced points including both ends.
"""
import numpy as np


def clamped_knots(n, degree=3):
    """Clamped uniform knot vector with ``n + degree + 1`` entries on [0, 1]."""
    if n < degree + 1:
        raise ValueError("need at least degree+1 basis functions")
    inner = np.linspace(0.0, 1.0, n - degree + 1)
    return np.concatenate([np.zeros(degree), inner, np.ones(degree)])


def _basis_row(t, knots, n, degree):
    """Values of all ``n`` B-spline basis functions at one point ``t``.

    Cox-de Boor recursion, written from the textbook definition: start with the
    indicator of the knot span that holds ``t`` (the last non-empty span holds
    the right end point) and raise the degree one step at a time.
    """
    nk = len(knots)
    # degree-0 functions: indicator of [knots[i], knots[i+1])
    b = np.zeros(nk - 1)
    if t >= knots[-1]:
        # right end point belongs to the last non-empty span
        i = nk - 2
        while knots[i] == knots[i + 1]:
            i -= 1
        b[i] = 1.0
    else:
        for i in range(nk - 1):
            if knots[i] <= t < knots[i + 1]:
                b[i] = 1.0
                break
    for p in range(1, degree + 1):
        nb = np.zeros(nk - 1 - p)
        for i in range(nk - 1 - p):
            left = 0.0
            den = knots[i + p] - knots[i]
            if den > 0.0:
                left = (t - knots[i]) / den * b[i]
            right = 0.0
            den = knots[i + p + 1] - knots[i + 1]
            if den > 0.0:
                right = (knots[i + p + 1] - t) / den * b[i + 1]
            nb[i] = left + right
        b = nb
    assert len(b) == n
    return b


_CACHE = {}


def collocation_matrix(m, n, degree=3):
    """m x n matrix: entry (i, j) is basis function j at sample t_i = i/(m-1)."""
    key = (int(m), int(n), int(degree))
    if key not in _CACHE:
        _CACHE[key] = _collocation(*key)
    return _CACHE[key].copy()


def _collocation(m, n, degree):
    if m < 2:
        raise ValueError("need at least two sample points")
    knots = clamped_knots(n, degree)
    A = np.zeros((m, n))
    for i in range(m):
        A[i] = _basis_row(i / (m - 1), knots, n, degree)
    return A


def second_difference(n):
    """(n-2) x n unscaled second difference: row j holds [1, -2, 1] at j..j+2."""
    if n < 3:
        raise ValueError("second difference needs n >= 3")
    D = np.zeros((n - 2, n))
    for j in range(n - 2):
        D[j, j] = 1.0
        D[j, j + 1] = -2.0
        D[j, j + 2] = 1.0
    return D
