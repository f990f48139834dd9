"""Container for one conic instance and the row layout of its cone product.

Standard form (eq:conic-standard):  minimize 1/2 x'Px + q'x  s.t.  Ax + s = b,
s in K, with K a Cartesian product of zero, nonnegative, second-order and PSD
cones (Sec. "Deep Unfolding Conic Optimization").  Rows of A, b, s, y are
grouped by cone block, in the order the blocks are listed.

PSD blocks are stored in the "svec" triangle encoding: a symmetric p x p
matrix X occupies p(p+1)/2 rows, ordered column-major over the upper triangle
(column j holds rows i = 0..j), with every off-diagonal entry scaled by
sqrt(2) so that the encoding is an isometry (<svec X, svec Y> = tr(XY)).
The paper does not fix an encoding; this is the convention used throughout.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np
import scipy.sparse as sp

ZERO, NONNEG, SOC, PSD = "zero", "nonneg", "soc", "psd"
KINDS = (ZERO, NONNEG, SOC, PSD)


@dataclass(frozen=True)
class Cone:
    kind: str   # one of KINDS
    size: int   # rows for zero/nonneg/soc; matrix order p for psd

    @property
    def rows(self) -> int:
        return psd_rows(self.size) if self.kind == PSD else self.size


def psd_rows(p: int) -> int:
    return p * (p + 1) // 2


def svec_index(i: int, j: int) -> int:
    """Row of entry (i, j) of a symmetric matrix in the svec encoding."""
    if i > j:
        i, j = j, i
    return j * (j + 1) // 2 + i


def svec_of_dense(X: np.ndarray) -> np.ndarray:
    """Encode a symmetric matrix in the svec layout of svec_index (upper
    triangle column by column, off-diagonal entries times sqrt(2))."""
    p = X.shape[0]
    r, c = np.tril_indices(p)            # row-major lower = column-major upper of X'
    return X[c, r] * np.where(r == c, 1.0, np.sqrt(2.0))


@dataclass
class ConicInstance:
    P: sp.csr_matrix          # n x n, symmetric, full storage (may be empty)
    q: np.ndarray             # [n]
    A: sp.csr_matrix          # m x n
    b: np.ndarray             # [m]
    cones: List[Cone]
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.shape[1]

    @property
    def m(self) -> int:
        return self.A.shape[0]

    def check(self) -> None:
        m, n = self.A.shape
        assert self.P.shape == (n, n)
        assert self.q.shape == (n,) and self.b.shape == (m,)
        assert sum(c.rows for c in self.cones) == m, "cone rows must cover A"
        for c in self.cones:
            assert c.kind in KINDS and c.size >= 1

    def astype(self, dtype) -> "ConicInstance":
        """Round the data to `dtype` (the instance actually solved).

        Data are generated in float64; a float32 run rounds them once and the
        float64 oracle is fed the rounded values so both solve one instance.
        """
        dt = np.dtype(dtype)
        P = self.P.astype(dt).astype(np.float64)
        A = self.A.astype(dt).astype(np.float64)
        return ConicInstance(sp.csr_matrix(P), self.q.astype(dt).astype(np.float64),
                             sp.csr_matrix(A), self.b.astype(dt).astype(np.float64),
                             list(self.cones), dict(self.meta))


def cone_row_slices(cones: List[Cone]) -> List[Tuple[Cone, slice]]:
    out, r = [], 0
    for c in cones:
        out.append((c, slice(r, r + c.rows)))
        r += c.rows
    return out
