"""Independent brute-force references used to pin the oracle (dense numpy, tiny n).

Nothing here calls the oracle or the product; each function restates a
textbook definition directly.
"""

from __future__ import annotations

import itertools

import numpy as np


def parse_golden(path):
    """Sections of a golden text fixture: name -> list of int lists."""
    out, cur = {}, None
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if cur is None:
                cur = line
                out[cur] = []
            elif line == "end":
                cur = None
            else:
                out[cur].append([int(t) for t in line.replace(":", " ").split()])
    return out


def boolean_elimination(F: np.ndarray) -> np.ndarray:
    """Structural Gaussian elimination without pivoting: eliminating k makes
    (i, j) nonzero for every i > k with F(i,k) and every j > k with F(k,j)."""
    F = F.astype(bool).copy()
    n = F.shape[0]
    for k in range(n):
        rows = np.nonzero(F[k + 1:, k])[0] + k + 1
        cols = np.nonzero(F[k, k + 1:])[0] + k + 1
        if rows.size and cols.size:
            F[np.ix_(rows, cols)] = True
    return F


def fill_path(F: np.ndarray) -> np.ndarray:
    """Rose-Tarjan fill-path characterization: (i,j) is in the filled pattern iff
    G(F) has a directed path i -> ... -> j whose intermediate vertices are all
    smaller than min(i, j).  Brute force by BFS restricted to small vertices."""
    F = F.astype(bool)
    n = F.shape[0]
    R = np.zeros_like(F)
    for i in range(n):
        for j in range(n):
            if F[i, j] or i == j and F[i, i]:
                R[i, j] = True
                continue
            lim = min(i, j)
            seen = {i}
            frontier = [i]
            found = False
            while frontier and not found:
                nxt = []
                for u in frontier:
                    for v in np.nonzero(F[u])[0]:
                        v = int(v)
                        if v == j:
                            found = True
                            break
                        if v < lim and v not in seen:
                            seen.add(v)
                            nxt.append(v)
                    if found:
                        break
                frontier = nxt
            R[i, j] = found
    return R


def dense_doolittle(D: np.ndarray):
    """No-pivot Doolittle LU of a dense matrix: L unit lower, U upper."""
    n = D.shape[0]
    L = np.eye(n)
    U = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            U[i, j] = D[i, j] - L[i, :i] @ U[:i, j]
        for r in range(i + 1, n):
            L[r, i] = (D[r, i] - L[r, :i] @ U[:i, i]) / U[i, i]
    return L, U


def exact_hazards(F: np.ndarray):
    """Read-after-write hazards between columns of the right-looking algorithm
    on the filled pattern F (dense bool, A_s = L + U - I).

    Column j reads A_s(j,j), A_s(i,j) for i > j, and A_s(j,k) for k > j with
    U(j,k) != 0; it writes its own L column and A_s(i,k) for i in L(:,j),
    k in U(j,:).  A write by j1 read by j2 > j1 is a hazard:
      U(j1,j2) != 0 and L(i,j1) != 0 for some i >= j2, or
      L(j2,j1) != 0, L(:,j2) not empty and U(j1,k) != 0 for some k > j2.
    Write-after-read cannot occur (j2 only writes rows > j2 > j1).
    """
    n = F.shape[0]
    E = set()
    for j1, j2 in itertools.combinations(range(n), 2):
        Lj1 = [i for i in range(j1 + 1, n) if F[i, j1]]
        if F[j1, j2] and any(i >= j2 for i in Lj1):
            E.add((j1, j2))
        Lj2 = any(F[i, j2] for i in range(j2 + 1, n))
        if F[j2, j1] and Lj2 and any(F[j1, k] for k in range(j2 + 1, n)):
            E.add((j1, j2))
    return E


def csc_pattern_to_dense(n, colptr, rowind) -> np.ndarray:
    F = np.zeros((n, n), bool)
    for j in range(n):
        F[rowind[colptr[j]:colptr[j + 1]], j] = True
    return F


def dense_pattern_to_csc(F: np.ndarray):
    n = F.shape[0]
    colptr = np.zeros(n + 1, np.int64)
    rows = []
    for j in range(n):
        r = np.nonzero(F[:, j])[0].astype(np.int32)
        rows.append(r)
        colptr[j + 1] = colptr[j] + r.size
    return colptr, (np.concatenate(rows) if rows else np.zeros(0, np.int32))


def edges_of(n, ptr, idx):
    return {(int(i), k) for k in range(n) for i in idx[ptr[k]:ptr[k + 1]]}
