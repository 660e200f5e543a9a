"""CPU oracle for the levelized sparse LU path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the product library: the product
never imports it, and it never imports the product.  Inputs come from the
seeded generators in ``circuitgen`` (which hold none of the method's
arithmetic), or from the caller.

What it computes, and the passage each piece follows:

* ``permute``   B = P A P^T (static symmetric reordering before factorization,
                Section II-C's preprocessing)
* ``symbolic``  fill pattern of A_s = L + U - I (Section II-A, symbolic
                analysis before Alg. 1)
* ``dag``       relaxed dependency detection (Alg. 4, Section III-A)
* ``levels``    levelization (Section II-C)
* ``factor``    Gilbert-Peierls left-looking numeric LU (Alg. 1)
* ``solve``     the two triangular solves (Section I)
* ``factor_extended``  Alg. 1 accumulated in extended precision, an accuracy
                reference closer to the exact factors than any FP64 order
* ``right_looking`` / ``levelized_right_looking`` (``oracle.right_looking``):
                Alg. 2 with the submatrix update of Alg. 5, run sequentially
                or level by level, in pure Python for small inputs.
* ``mmd_order`` a fill-reducing symmetric ordering taken from SciPy's SuperLU
                (multiple minimum degree on A + A^T), used only to give test
                inputs a realistic ordering independent of the product.

Parity pins for every function live in ``tests/test_oracle_pins.py``.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from circuitgen import CscMatrix

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

ORC_OK = 0
ORC_ERR_ARG = -1
ORC_ERR_ZERO_PIVOT = -3
ORC_ERR_STRUCT_SINGULAR = -4
ORC_ERR_NOMEM = -5
ORC_ERR_NONFINITE = -7


class OracleError(RuntimeError):
    def __init__(self, code: int, column: int = -1):
        super().__init__(f"oracle error {code} (column {column})")
        self.code = code
        self.column = column


def _lib():
    global _LIB
    if _LIB is None:
        from . import _build

        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.c_void_p
        i32, i64 = C.c_int32, C.c_int64
        L.orc_free.argtypes = [P]
        L.orc_check_csc.argtypes = [i32, P, P]
        L.orc_check_csc.restype = C.c_int
        L.orc_permute.argtypes = [i32, P, P, P, P, P, P, P]
        L.orc_permute.restype = C.c_int
        L.orc_symbolic.argtypes = [i32, P, P, P, C.POINTER(P), C.POINTER(i32)]
        L.orc_symbolic.restype = i64
        L.orc_dag.argtypes = [i32, P, P, P, C.POINTER(P)]
        L.orc_dag.restype = i64
        L.orc_levels.argtypes = [i32, P, P, P, P, P]
        L.orc_levels.restype = i32
        L.orc_factor.argtypes = [i32, P, P, P, P, P, P, C.POINTER(i32)]
        L.orc_factor.restype = C.c_int
        L.orc_solve.argtypes = [i32, P, P, P, P, i32, P, i64, P, i64]
        L.orc_solve.restype = C.c_int
        L.orc_factor_extended.argtypes = [i32, P, P, P, P, P, P, C.POINTER(i32)]
        L.orc_factor_extended.restype = C.c_int
        L.orc_fill_lower.argtypes = [i32, P, P, i32, P]
        L.orc_fill_lower.restype = i32
        L.orc_fill_upper.argtypes = [i32, P, P, i32, P]
        L.orc_fill_upper.restype = i32
        _LIB = L
    return _LIB


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _take(ptr: C.c_void_p, count: int, dtype) -> np.ndarray:
    """Copy a malloc'ed C array into numpy and free it."""
    L = _lib()
    if count > 0:
        buf = (C.c_byte * (count * np.dtype(dtype).itemsize)).from_address(ptr.value)
        out = np.frombuffer(buf, dtype=dtype).copy()
    else:
        out = np.zeros(0, dtype=dtype)
    L.orc_free(ptr)
    return out


def _csc_arrays(A: CscMatrix):
    return (
        np.ascontiguousarray(A.colptr, dtype=np.int64),
        np.ascontiguousarray(A.rowind, dtype=np.int32),
        np.ascontiguousarray(A.values, dtype=np.float64),
    )


def permute(A: CscMatrix, perm: np.ndarray) -> CscMatrix:
    """B = P A P^T with B(i, j) = A(perm[i], perm[j]) (perm[new] = old)."""
    cp, ri, v = _csc_arrays(A)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    bcp = np.zeros(A.n + 1, np.int64)
    bri = np.zeros(max(A.nnz, 1), np.int32)
    bv = np.zeros(max(A.nnz, 1), np.float64)
    rc = _lib().orc_permute(A.n, _p(cp), _p(ri), _p(v), _p(perm), _p(bcp), _p(bri), _p(bv))
    if rc != ORC_OK:
        raise OracleError(rc)
    return CscMatrix(A.n, bcp, bri[: A.nnz], bv[: A.nnz])


def symbolic(B: CscMatrix):
    """Pattern of A_s (lu_colptr int64[n+1], lu_rowind int32[nnz]) for B without pivoting."""
    cp, ri, _ = _csc_arrays(B)
    lcp = np.zeros(B.n + 1, np.int64)
    out = C.c_void_p()
    bad = C.c_int32(-1)
    nnz = _lib().orc_symbolic(B.n, _p(cp), _p(ri), _p(lcp), C.byref(out), C.byref(bad))
    if nnz < 0:
        if out.value:
            _lib().orc_free(out)
        raise OracleError(int(nnz), bad.value)
    return lcp, _take(out, int(nnz), np.int32)


def dag(n: int, lu_colptr: np.ndarray, lu_rowind: np.ndarray):
    """Relaxed column dependency DAG (Alg. 4) as CSR (dag_ptr int64[n+1], dag_idx int32)."""
    dp = np.zeros(n + 1, np.int64)
    out = C.c_void_p()
    lcp = np.ascontiguousarray(lu_colptr, np.int64)
    lri = np.ascontiguousarray(lu_rowind, np.int32)
    m = _lib().orc_dag(n, _p(lcp), _p(lri), _p(dp), C.byref(out))
    if m < 0:
        raise OracleError(int(m))
    return dp, _take(out, int(m), np.int32)


def levels(n: int, dag_ptr: np.ndarray, dag_idx: np.ndarray):
    """(lev int32[n], level_ptr int32[L+1], level_cols int32[n])."""
    lev = np.zeros(max(n, 1), np.int32)
    lp = np.zeros(n + 1, np.int32)
    lc = np.zeros(max(n, 1), np.int32)
    dp = np.ascontiguousarray(dag_ptr, np.int64)
    di = np.ascontiguousarray(dag_idx, np.int32)
    nl = _lib().orc_levels(n, _p(dp), _p(di if di.size else np.zeros(1, np.int32)), _p(lev), _p(lp), _p(lc))
    if nl < 0:
        raise OracleError(int(nl))
    return lev[:n], lp[: nl + 1].copy(), lc[:n]


def factor(B: CscMatrix, lu_colptr: np.ndarray, lu_rowind: np.ndarray) -> np.ndarray:
    """Values of A_s (L strictly below the diagonal, U on and above) by Alg. 1."""
    cp, ri, v = _csc_arrays(B)
    nnz = int(lu_colptr[-1])
    val = np.zeros(max(nnz, 1), np.float64)
    bad = C.c_int32(-1)
    lcp = np.ascontiguousarray(lu_colptr, np.int64)
    lri = np.ascontiguousarray(lu_rowind, np.int32)
    rc = _lib().orc_factor(B.n, _p(cp), _p(ri), _p(v), _p(lcp), _p(lri), _p(val), C.byref(bad))
    if rc != ORC_OK:
        raise OracleError(rc, bad.value)
    return val[:nnz]


def factor_extended(B: CscMatrix, lu_colptr: np.ndarray, lu_rowind: np.ndarray) -> np.ndarray:
    """Alg. 1 accumulated in extended precision (C long double), rounded to
    float64 at the end: an accuracy reference for the factors."""
    cp, ri, v = _csc_arrays(B)
    nnz = int(lu_colptr[-1])
    val = np.zeros(max(nnz, 1), np.float64)
    bad = C.c_int32(-1)
    lcp = np.ascontiguousarray(lu_colptr, np.int64)
    lri = np.ascontiguousarray(lu_rowind, np.int32)
    rc = _lib().orc_factor_extended(B.n, _p(cp), _p(ri), _p(v), _p(lcp), _p(lri), _p(val), C.byref(bad))
    if rc != ORC_OK:
        raise OracleError(rc, bad.value)
    return val[:nnz]


def solve(lu_colptr, lu_rowind, lu_val, perm, b: np.ndarray) -> np.ndarray:
    """x with A x = b from the factors of B = P A P^T.  b is (n,) or (n, nrhs)."""
    b2 = np.asfortranarray(b.reshape(b.shape[0], -1), dtype=np.float64)
    n, nrhs = b2.shape
    x = np.zeros_like(b2, order="F")
    lcp = np.ascontiguousarray(lu_colptr, np.int64)
    lri = np.ascontiguousarray(lu_rowind, np.int32)
    lv = np.ascontiguousarray(lu_val, np.float64)
    pm = np.ascontiguousarray(perm, np.int32)
    rc = _lib().orc_solve(n, _p(lcp), _p(lri), _p(lv), _p(pm), nrhs, _p(b2), n, _p(x), n)
    if rc != ORC_OK:
        raise OracleError(rc)
    return x.reshape(b.shape)


def fill_lower(B: CscMatrix, j: int) -> np.ndarray:
    """Rows i >= j of column j of A_s, from the fill-path lemma (a path
    i -> ... -> j in the graph of B through vertices below j)."""
    cp, ri, _ = _csc_arrays(B)
    out = np.zeros(max(B.n, 1), np.int32)
    c = _lib().orc_fill_lower(B.n, _p(cp), _p(ri), int(j), _p(out))
    if c < 0:
        raise OracleError(int(c))
    return out[:c].copy()


def fill_upper(B: CscMatrix, i: int) -> np.ndarray:
    """Columns k >= i of row i of A_s, from the fill-path lemma (a path
    i -> ... -> k in the graph of B through vertices below i)."""
    cp, ri, _ = _csc_arrays(B)
    out = np.zeros(max(B.n, 1), np.int32)
    c = _lib().orc_fill_upper(B.n, _p(cp), _p(ri), int(i), _p(out))
    if c < 0:
        raise OracleError(int(c))
    return out[:c].copy()


@dataclass
class OracleResult:
    perm: np.ndarray
    B: CscMatrix
    lu_colptr: np.ndarray
    lu_rowind: np.ndarray
    dag_ptr: np.ndarray
    dag_idx: np.ndarray
    lev: np.ndarray
    level_ptr: np.ndarray
    level_cols: np.ndarray
    lu_val: np.ndarray | None = None


def analyze(A: CscMatrix, perm: np.ndarray | None = None, numeric: bool = True) -> OracleResult:
    """Run the whole oracle chain for A under the symmetric permutation ``perm``."""
    if perm is None:
        perm = np.arange(A.n, dtype=np.int32)
    B = permute(A, perm)
    lcp, lri = symbolic(B)
    dp, di = dag(A.n, lcp, lri)
    lev, lp, lc = levels(A.n, dp, di)
    r = OracleResult(np.asarray(perm, np.int32), B, lcp, lri, dp, di, lev, lp, lc)
    if numeric:
        r.lu_val = factor(B, lcp, lri)
    return r


def mmd_order(A: CscMatrix) -> np.ndarray:
    """Fill-reducing symmetric ordering (perm[new] = old) from SciPy's SuperLU,
    multiple minimum degree on A + A^T with diagonal pivoting forced."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla

    M = sp.csc_matrix((A.values, A.rowind, A.colptr), shape=(A.n, A.n))
    lu = sla.splu(M, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                  options=dict(SymmetricMode=True))
    return np.argsort(lu.perm_c).astype(np.int32)


def level_stats(n, lu_colptr, lu_rowind, level_ptr, level_cols):
    """Counts used to size the work: nL, nU, MACs and per-level widths."""
    lcp = np.asarray(lu_colptr)
    lri = np.asarray(lu_rowind)
    cols = np.repeat(np.arange(n), np.diff(lcp))
    below = lri > cols
    above = lri < cols
    nL_col = np.bincount(cols[below], minlength=n)
    nU_row = np.bincount(lri[above], minlength=n)
    macs = int((nL_col.astype(np.int64) * nU_row.astype(np.int64)).sum())
    widths = np.diff(np.asarray(level_ptr))
    return dict(nL=int(below.sum()), nU=int(above.sum()), macs=macs, n_levels=int(widths.size),
                widest=int(widths.max()) if widths.size else 0,
                max_L=int(nL_col.max()) if n else 0)
