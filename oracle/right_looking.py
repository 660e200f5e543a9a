"""Pure-Python right-looking formulations -- TEST INFRASTRUCTURE ONLY, small inputs.

* ``right_looking``: the hybrid column-based right-looking algorithm (Alg. 2):
  for each column j left to right, divide L(:,j) by the pivot, then update every
  subcolumn k with A_s(j,k) != 0 by the submatrix update of Alg. 5:
  A_s(i,k) -= A_s(i,j) * A_s(j,k) for every i with A_s(i,j) != 0 below j.
  ``order`` lets the columns be visited in any sequence (e.g. level order).

* ``levelized_right_looking``: the same algorithm executed the way a parallel
  device runs one level: every column of a level reads the matrix as it was
  when the level started, writes its own normalised L column at once, and all
  submatrix-update writes are deferred to the end of the level and applied per
  target entry in ascending source column.  With a sufficient dependency DAG
  (Alg. 4) the result is bitwise identical to ``right_looking`` visiting the
  columns in level order; with an insufficient one (e.g. the U-only detection
  of GLU1.0, which misses the double-U hazard of Section II-C) it is not.

Both work in float64 on the filled pattern (lu_colptr, lu_rowind) of A_s and
use Python floats, so no fused multiply-add occurs.
"""

from __future__ import annotations

import numpy as np


class _Pattern:
    def __init__(self, n, lu_colptr, lu_rowind):
        self.n = n
        self.cp = [int(x) for x in lu_colptr]
        self.ri = [int(x) for x in lu_rowind]
        self.pos = {}
        self.diag = [-1] * n
        self.lcol = [[] for _ in range(n)]  # rows of L(:,j)
        self.urow = [[] for _ in range(n)]  # columns k > j with A_s(j,k) != 0
        for j in range(n):
            for p in range(self.cp[j], self.cp[j + 1]):
                i = self.ri[p]
                self.pos[(i, j)] = p
                if i == j:
                    self.diag[j] = p
                elif i > j:
                    self.lcol[j].append(i)
                else:
                    self.urow[i].append(j)
        for j in range(n):
            self.urow[j].sort()


def scatter_values(n, lu_colptr, lu_rowind, B) -> np.ndarray:
    """Place B's values on the filled pattern (fill entries start at zero)."""
    pat = _Pattern(n, lu_colptr, lu_rowind)
    val = np.zeros(int(lu_colptr[-1]))
    for j in range(n):
        for p in range(int(B.colptr[j]), int(B.colptr[j + 1])):
            val[pat.pos[(int(B.rowind[p]), j)]] = float(B.values[p])
    return val


def right_looking(n, lu_colptr, lu_rowind, B, order=None) -> np.ndarray:
    pat = _Pattern(n, lu_colptr, lu_rowind)
    v = [float(x) for x in scatter_values(n, lu_colptr, lu_rowind, B)]
    cols = range(n) if order is None else [int(c) for c in order]
    for j in cols:
        d = v[pat.diag[j]]
        if d == 0.0:
            raise ZeroDivisionError(f"zero pivot in column {j}")
        for i in pat.lcol[j]:
            v[pat.pos[(i, j)]] = v[pat.pos[(i, j)]] / d
        for k in pat.urow[j]:
            u = v[pat.pos[(j, k)]]
            for i in pat.lcol[j]:
                q = pat.pos.get((i, k))
                if q is None:
                    raise KeyError(f"fill closure violated at ({i},{k})")
                v[q] = v[q] - v[pat.pos[(i, j)]] * u
    return np.array(v)


def levelized_right_looking(n, lu_colptr, lu_rowind, B, level_ptr, level_cols) -> np.ndarray:
    pat = _Pattern(n, lu_colptr, lu_rowind)
    v = [float(x) for x in scatter_values(n, lu_colptr, lu_rowind, B)]
    for lvl in range(len(level_ptr) - 1):
        cols = sorted(int(c) for c in level_cols[level_ptr[lvl]:level_ptr[lvl + 1]])
        snap = list(v)
        deferred = []  # (target position, source column, l, u) in ascending source column
        for j in cols:
            d = snap[pat.diag[j]]
            if d == 0.0:
                raise ZeroDivisionError(f"zero pivot in column {j}")
            lvals = {}
            for i in pat.lcol[j]:
                lvals[i] = snap[pat.pos[(i, j)]] / d
                v[pat.pos[(i, j)]] = lvals[i]
            for k in pat.urow[j]:
                u = snap[pat.pos[(j, k)]]
                for i in pat.lcol[j]:
                    deferred.append((pat.pos[(i, k)], j, lvals[i], u))
        deferred.sort(key=lambda t: (t[0], t[1]))
        for q, _, l, u in deferred:
            v[q] = v[q] - l * u
    return np.array(v)


def u_only_dag(n, lu_colptr, lu_rowind):
    """GLU1.0's dependency detection ("look up" only), kept as a negative fixture:
    k depends on i < k when A_s(i,k) != 0 and L(:,i) is not empty."""
    pat = _Pattern(n, lu_colptr, lu_rowind)
    ptr = [0]
    idx = []
    for k in range(n):
        deps = sorted(i for i in range(k) if (i, k) in pat.pos and pat.lcol[i])
        idx.extend(deps)
        ptr.append(len(idx))
    return np.array(ptr, np.int64), np.array(idx, np.int32)
