"""Mode products and the inner product (oracle; test infrastructure only).

Sec. 2.1, eq. separable_transf: a separable transformation of a tensor is the
sequential application of one 1-D transformation per index.  For an index k
of T and a matrix M (rows = new index, columns = old index) the 1-D
transformation along k is the mode-k product

    (T x_k M)[i_1, .., j, .., i_N] = sum_{i_k} M[j, i_k] * T[i_1, .., i_k, .., i_N].

Ordered spaces fix the position of every index in the result (Sec. 2.1), so the
new index j stays at position k and products on distinct modes commute.
"""
import itertools

import numpy as np


def mode_product(T, M, k):
    """T x_k M in float64; ``k`` is the 0-based mode, M has shape (J, T.shape[k])."""
    T = np.asarray(T, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    if M.ndim != 2 or M.shape[1] != T.shape[k]:
        raise ValueError(f"mode {k}: matrix {M.shape} does not match extent {T.shape[k]}")
    # contract the column index of M with index k of T; the new index comes first
    out = np.tensordot(M, T, axes=([1], [k]))
    # put the new index back at position k (ordered spaces)
    return np.moveaxis(out, 0, k)


def multi_mode_product(T, mats, modes=None, order=None):
    """Apply M_k along mode k for each k in ``modes`` (default: all), in ``order``.

    ``mats[k]`` is the matrix of mode k (or ``None`` to skip that mode).  The
    result does not depend on ``order`` (commutativity on distinct spaces,
    Sec. 2.1) up to rounding; ``order`` only chooses the evaluation sequence.
    """
    if modes is None:
        modes = [k for k in range(len(mats)) if mats[k] is not None]
    if order is None:
        order = list(modes)
    if sorted(order) != sorted(modes):
        raise ValueError("order must be a permutation of modes")
    out = np.asarray(T, dtype=np.float64)
    for k in order:
        out = mode_product(out, mats[k], k)
    return out


def all_orders(modes):
    """Every evaluation order of a set of modes."""
    return list(itertools.permutations(modes))


def inner(A, B):
    """<A, B>: contraction over all index pairs = sum of the elementwise product (App. A.6)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if A.shape != B.shape:
        raise ValueError("inner product of tensors of different shape")
    return float(np.sum(A * B))
