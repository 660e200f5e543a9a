"""Seeded synthetic circuit-like sparse matrices, right-hand sides and value streams.

This module only *creates inputs*.  It contains none of the factorization's
arithmetic (no ordering, no fill, no dependency detection, no LU), so both the
CPU oracle and the HIP path may consume its output without sharing any of the
method's code.

The paper measures on circuit matrices from the University of Florida sparse
matrix collection (Section IV, Table 1).  Those matrices are not available
here; the generator below stands in for them with node-conductance matrices of
the same character: a few nonzeros per row, a nearly symmetric pattern, strong
diagonals, plus optional high-degree "rail" nodes that create the wide early
levels and the dense late levels the paper describes around its level-size
figure in Section III-B.

Recipe (every unstated detail fixed here):

* nodes ``0 .. n-R-1`` are regular, ``n-R .. n-1`` are rails (rails count in n);
* every regular node ``i`` draws 2 partners ``i +/- d`` with ``d ~ U{1..window}``
  and an equiprobable sign, clipped to the regular range; self loops dropped;
* ``round(long_frac * #local edges)`` long-range edges with endpoints uniform
  over regular nodes (self loops dropped);
* every rail connects to ``round(rail_frac * n)`` distinct uniform regular nodes;
* every edge gets a conductance ``g = exp(U(ln gmin, ln gmax))`` stamped as a
  Laplacian (``A_uu += g, A_vv += g, A_uv -= g, A_vu -= g``), duplicates summed;
* every stored off-diagonal entry independently, with probability
  ``asym_frac``, gets ``a += N(0, asym_scale * |a|)`` (unsymmetric values on a
  symmetric pattern);
* finally ``A_ii += diag_shift``.

Output is CSC: ``colptr`` int64[n+1], ``rowind`` int32[nnz] sorted ascending
within each column, no duplicates, ``values`` float64[nnz].
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "CscMatrix",
    "circuit_matrix",
    "config_matrix",
    "rhs",
    "perturbed_values",
    "CONFIGS",
    "from_dense",
    "to_dense",
    "random_pattern_matrix",
]


@dataclass
class CscMatrix:
    n: int
    colptr: np.ndarray  # int64[n+1]
    rowind: np.ndarray  # int32[nnz]
    values: np.ndarray  # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])


# Named workloads (sizes of the paper-like circuit matrices used by tests and the benchmark).
CONFIGS = {
    # n=2,000, no rails: the small case.
    "c0": dict(n=2_000, rails=0, rail_frac=0.0),
    # n=100,000 with 150 rails at 2% connectivity: wide early levels, dense late levels.
    "c1": dict(n=100_000, rails=150, rail_frac=0.02),
    # n=1,000,000 with 400 rails at 0.5% connectivity.
    "c2": dict(n=1_000_000, rails=400, rail_frac=0.005),
}

_CONFIG_INDEX = {"c0": 0, "c1": 1, "c2": 2, "c3": 3, "c4": 4}


def _assemble_csc(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CscMatrix:
    """Sum duplicate (row, col) entries and return sorted CSC."""
    key = cols.astype(np.int64) * n + rows.astype(np.int64)
    uniq, inv = np.unique(key, return_inverse=True)
    summed = np.bincount(inv, weights=vals, minlength=uniq.size)
    c = (uniq // n).astype(np.int64)
    r = (uniq % n).astype(np.int32)
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(colptr, c + 1, 1)
    colptr = np.cumsum(colptr)
    return CscMatrix(n, colptr, r, summed.astype(np.float64))


def circuit_matrix(
    n: int,
    rails: int = 0,
    rail_frac: float = 0.0,
    seed: int = 0,
    window: int = 40,
    long_frac: float = 0.01,
    asym_frac: float = 0.05,
    asym_scale: float = 0.1,
    diag_shift: float = 1e-3,
    gmin: float = 1e-3,
    gmax: float = 1e3,
) -> CscMatrix:
    """Circuit-like node-conductance matrix following the module recipe."""
    if n < 1:
        raise ValueError("n must be >= 1")
    if rails < 0 or rails >= n and n > 1:
        raise ValueError("rails must satisfy 0 <= rails < n")
    rng = np.random.default_rng(seed)
    nr = n - rails
    # local edges
    src = np.repeat(np.arange(nr, dtype=np.int64), 2)
    d = rng.integers(1, window + 1, size=src.size)
    sign = rng.integers(0, 2, size=src.size) * 2 - 1
    dst = np.clip(src + sign * d, 0, max(nr - 1, 0))
    keep = dst != src
    eu, ev = src[keep], dst[keep]
    n_local = eu.size
    # long-range edges
    n_long = int(round(long_frac * n_local))
    if n_long > 0 and nr > 1:
        lu = rng.integers(0, nr, size=n_long)
        lv = rng.integers(0, nr, size=n_long)
        k = lu != lv
        eu = np.concatenate([eu, lu[k]])
        ev = np.concatenate([ev, lv[k]])
    # rails
    per_rail = int(round(rail_frac * n))
    per_rail = min(per_rail, nr)
    rail_u, rail_v = [], []
    for r in range(rails):
        if per_rail == 0:
            break
        tgt = rng.choice(nr, size=per_rail, replace=False)
        rail_u.append(np.full(per_rail, nr + r, dtype=np.int64))
        rail_v.append(tgt.astype(np.int64))
    if rail_u:
        eu = np.concatenate([eu] + rail_u)
        ev = np.concatenate([ev] + rail_v)
    # conductances, Laplacian stamps
    g = np.exp(rng.uniform(math.log(gmin), math.log(gmax), size=eu.size))
    rows = np.concatenate([eu, ev, eu, ev, np.arange(n, dtype=np.int64)])
    cols = np.concatenate([eu, ev, ev, eu, np.arange(n, dtype=np.int64)])
    vals = np.concatenate([g, g, -g, -g, np.zeros(n)])
    A = _assemble_csc(n, rows, cols, vals)
    # unsymmetric perturbation of off-diagonal entries
    colidx = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.colptr))
    offd = A.rowind.astype(np.int64) != colidx
    hit = (rng.random(A.nnz) < asym_frac) & offd
    noise = rng.standard_normal(A.nnz)
    A.values[hit] += noise[hit] * asym_scale * np.abs(A.values[hit])
    # diagonal shift
    A.values[~offd] += diag_shift
    return A


def config_matrix(name: str, index: int = 0) -> CscMatrix:
    """Matrix of a named workload; seed = 1000 * config number + index."""
    cfg = CONFIGS[name]
    seed = 1000 * _CONFIG_INDEX[name] + index
    return circuit_matrix(seed=seed, **cfg)


def rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """Right-hand sides uniform in [-1, 1], column-major ``(n, nrhs)`` Fortran-ordered."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.uniform(-1.0, 1.0, size=(n, nrhs)))


def perturbed_values(base: np.ndarray, seed: int, sigma: float = 0.1) -> np.ndarray:
    """Newton-iteration-like value change: every nonzero times an independent
    log-normal(0, sigma) factor, relative to ``base`` (not compounding)."""
    rng = np.random.default_rng(seed)
    return base * np.exp(rng.normal(0.0, sigma, size=base.size))


def from_dense(D: np.ndarray, pattern: np.ndarray | None = None) -> CscMatrix:
    """CSC of a dense array; ``pattern`` (bool) keeps explicit zeros structurally."""
    D = np.asarray(D, dtype=np.float64)
    n = D.shape[0]
    mask = (D != 0) if pattern is None else np.asarray(pattern, dtype=bool)
    colptr = np.zeros(n + 1, dtype=np.int64)
    rows, vals = [], []
    for j in range(n):
        r = np.nonzero(mask[:, j])[0]
        rows.append(r.astype(np.int32))
        vals.append(D[r, j])
        colptr[j + 1] = colptr[j] + r.size
    return CscMatrix(
        n,
        colptr,
        np.concatenate(rows) if rows else np.zeros(0, np.int32),
        np.concatenate(vals) if vals else np.zeros(0),
    )


def to_dense(A: CscMatrix) -> np.ndarray:
    D = np.zeros((A.n, A.n))
    for j in range(A.n):
        s, e = A.colptr[j], A.colptr[j + 1]
        D[A.rowind[s:e], j] = A.values[s:e]
    return D


def random_pattern_matrix(n: int, density: float, seed: int, symmetric_pattern: bool = False) -> CscMatrix:
    """Small random matrix with a full, dominant diagonal (so no pivot vanishes).

    Used for property tests of the symbolic and numeric steps on tiny inputs.
    """
    rng = np.random.default_rng(seed)
    M = rng.random((n, n)) < density
    if symmetric_pattern:
        M = M | M.T
    np.fill_diagonal(M, True)
    V = rng.uniform(-1.0, 1.0, size=(n, n)) * M
    rowsum = np.abs(V).sum(axis=1)
    V[np.arange(n), np.arange(n)] = rowsum + 1.0
    return from_dense(V, pattern=M)
