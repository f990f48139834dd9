"""Triangle encoding of symmetric matrices (test infrastructure; see package doc).

The paper projects "the slack matrix" of each PSD block but does not say how
a symmetric block is laid out in the vector s.  Reading used here: column-major
upper triangle, off-diagonal entries multiplied by sqrt(2), which makes
svec an isometry, so one penalty per block keeps the scaled projection of
eq:cosmo_projection a Euclidean projection.
"""
import math

import numpy as np

_R2 = math.sqrt(2.0)


def svec_len(p: int) -> int:
    return p * (p + 1) // 2


def order_from_len(ell: int) -> int:
    p = int(round((math.sqrt(8 * ell + 1) - 1) / 2))
    if svec_len(p) != ell:
        raise ValueError(f"{ell} is not a triangular number")
    return p


def svec(X: np.ndarray) -> np.ndarray:
    """Symmetric p x p -> vector of length p(p+1)/2 (column j holds i <= j)."""
    p = X.shape[0]
    out = []
    for j in range(p):
        for i in range(j + 1):
            out.append(X[i, j] if i == j else _R2 * X[i, j])
    return np.array(out, dtype=np.float64)


def smat(v: np.ndarray) -> np.ndarray:
    """Inverse of svec (and its adjoint, since svec is an isometry)."""
    p = order_from_len(len(v))
    X = np.zeros((p, p))
    k = 0
    for j in range(p):
        for i in range(j + 1):
            if i == j:
                X[i, i] = v[k]
            else:
                X[i, j] = X[j, i] = v[k] / _R2
            k += 1
    return X
