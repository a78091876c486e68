"""Matrix-equivalent form of the tensor equation (oracle; test infrastructure only).

Sec. 3: a tensor equation A*U = B is a matrix equation after reshaping the
tensors into vectors.  For tiny sizes the operator is assembled column by
column (apply it to every unit tensor) and the SPD system is solved by a
Cholesky factorisation.  Row-major (C-order) vectorisation is used.
"""
import numpy as np
import scipy.linalg


def assemble(apply, shape):
    """Dense matrix of ``apply`` on tensors of ``shape`` (C-order vec)."""
    shape = tuple(shape)
    n = int(np.prod(shape))
    if n > 8192:
        raise ValueError("dense assembly is for tiny problems only")
    M = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        M[:, j] = np.asarray(apply(e.reshape(shape)), dtype=np.float64).reshape(n)
    return M


def dense_solve(apply, B):
    """Solve apply(X) = B through Cholesky of the assembled SPD matrix."""
    B = np.asarray(B, dtype=np.float64)
    M = assemble(apply, B.shape)
    c, low = scipy.linalg.cho_factor(M)
    return scipy.linalg.cho_solve((c, low), B.reshape(-1)).reshape(B.shape)
