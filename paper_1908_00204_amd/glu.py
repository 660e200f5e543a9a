"""Thin ctypes binding of the C ABI in ``include/glu.h`` (argument marshalling only).

Every step of the factorization and the solve runs in the HIP library
``libglu_mi355x.so``; this module only converts Python/NumPy/PyTorch arguments
into pointers.  PyTorch is used for device memory and streams when the caller
passes device tensors.  If the library is missing, importing raises -- there
is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libglu_mi355x.so")

GLU_OK = 0
GLU_ERR_ARG = -1
GLU_ERR_STATE = -2
GLU_ERR_ZERO_PIVOT = -3
GLU_ERR_STRUCT_SINGULAR = -4
GLU_ERR_NOMEM = -5
GLU_ERR_DEVICE = -6
GLU_ERR_NONFINITE_INPUT = -7
GLU_ERR_SCRATCH = -8

GLU_ORDER_AMD, GLU_ORDER_NATURAL, GLU_ORDER_USER = 0, 1, 2
GLU_MODE_AUTO, GLU_MODE_SMALL_BLOCK, GLU_MODE_LARGE_BLOCK, GLU_MODE_STREAM = 0, 1, 2, 3

EXPORTED = [
    "glu_create", "glu_analyze", "glu_factor", "glu_refactor", "glu_solve", "glu_query",
    "glu_export_symbolic", "glu_export_factors", "glu_failed_column", "glu_strerror", "glu_destroy",
    "glu_solve_noalloc", "glu_solve_noalloc_capacity",
    "glu_batch_create", "glu_batch_factor", "glu_batch_solve", "glu_batch_query", "glu_batch_destroy",
    "glu_mc64",
]


class glu_options(C.Structure):
    _fields_ = [
        ("ordering", C.c_int32),
        ("force_mode", C.c_int32),
        ("stream_threshold", C.c_int32),
        ("large_threshold", C.c_int32),
        ("max_device_bytes", C.c_int64),
        ("dense_tail", C.c_int32),
        ("gpu_analysis", C.c_int32),
        ("precision", C.c_int32),
        ("refine_max_iters", C.c_int32),
        ("dense_gemm", C.c_int32),
        ("reserved", C.c_int32 * 3),
    ]


class glu_info(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("n_levels", C.c_int32),
        ("nnz_a", C.c_int64),
        ("nnz_lu", C.c_int64),
        ("nnz_l", C.c_int64),
        ("nnz_u", C.c_int64),
        ("n_dag_edges", C.c_int64),
        ("macs", C.c_int64),
        ("n_levels_mode", C.c_int32 * 3),
        ("widest_level", C.c_int32),
        ("n_tasks", C.c_int64),
        ("n_work_items", C.c_int64),
        ("n_solve_levels_l", C.c_int32),
        ("n_solve_levels_u", C.c_int32),
        ("tail_m", C.c_int32),
        ("n_exec_levels", C.c_int32),
        ("device_bytes", C.c_int64),
        ("t_order_ms", C.c_double),
        ("t_symbolic_ms", C.c_double),
        ("t_levels_ms", C.c_double),
        ("t_plan_ms", C.c_double),
        ("t_factor_ms", C.c_double),
        ("t_solve_ms", C.c_double),
        ("t_update_ms", C.c_double),
        ("t_dense_ms", C.c_double),
        ("t_schur_ms", C.c_double),
        ("schur_macs", C.c_int64),
        ("schur_steps", C.c_int64),
        ("schur_tiles", C.c_int64),
        ("level_macs", C.c_int64),
        ("tail_macs", C.c_int64),
        ("level_nl", C.c_int64),
        ("level_nu", C.c_int64),
        ("precision", C.c_int32),
        ("refine_iters", C.c_int32),
        ("fp64_fallback", C.c_int32),
        ("reserved_info", C.c_int32),
        ("refine_berr", C.c_double),
    ]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if name == "n_levels_mode" else v
        return d


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with python -m paper_1908_00204_amd._build "
                "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        i32, i64 = C.c_int32, C.c_int64
        L.glu_create.argtypes = [C.POINTER(P), C.c_int, C.POINTER(glu_options)]
        L.glu_analyze.argtypes = [P, i32, P, P, P]
        L.glu_factor.argtypes = [P, P, C.c_int, P]
        L.glu_refactor.argtypes = [P, P, C.c_int, P]
        L.glu_solve.argtypes = [P, i32, P, i64, P, i64, C.c_int, P]
        L.glu_query.argtypes = [P, C.POINTER(glu_info)]
        L.glu_export_symbolic.argtypes = [P, P, P, P, P, P, P, P]
        L.glu_export_factors.argtypes = [P, P]
        L.glu_failed_column.argtypes = [P]
        L.glu_failed_column.restype = i32
        L.glu_strerror.argtypes = [C.c_int]
        L.glu_strerror.restype = C.c_char_p
        L.glu_destroy.argtypes = [P]
        L.glu_destroy.restype = None
        L.glu_solve_noalloc.argtypes = [P, i32, P, i64, P, i64, P]
        L.glu_solve_noalloc.restype = C.c_int
        L.glu_solve_noalloc_capacity.argtypes = []
        L.glu_solve_noalloc_capacity.restype = i64
        L.glu_batch_create.argtypes = [C.POINTER(P), C.POINTER(P), i32]
        L.glu_batch_create.restype = C.c_int
        L.glu_batch_factor.argtypes = [P, C.POINTER(P), C.c_int, P]
        L.glu_batch_factor.restype = C.c_int
        L.glu_batch_query.argtypes = [P, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                                      C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.glu_batch_solve.argtypes = [P, i32, C.POINTER(P), C.POINTER(i64), C.POINTER(P), C.POINTER(i64), P]
        L.glu_batch_solve.restype = C.c_int
        L.glu_batch_query.restype = C.c_int
        L.glu_batch_destroy.argtypes = [P]
        L.glu_batch_destroy.restype = None
        L.glu_mc64.argtypes = [i32, P, P, P, P, P, P]
        L.glu_mc64.restype = C.c_int
        for f in ("glu_create", "glu_analyze", "glu_factor", "glu_refactor", "glu_solve",
                  "glu_query", "glu_export_symbolic", "glu_export_factors"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


class GluError(RuntimeError):
    def __init__(self, code: int, where: str, column: int = -1):
        msg = lib().glu_strerror(code).decode()
        super().__init__(f"{where}: {msg} (code {code}" + (f", column {column})" if column >= 0 else ")"))
        self.code = code
        self.column = column


def _ptr(a) -> C.c_void_p:
    if a is None:
        return C.c_void_p(0)
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    return C.c_void_p(a.data_ptr())  # torch tensor


def _stream(stream, on_device: bool = False) -> C.c_void_p:
    """A HIP stream handle.  None means torch's current stream when the
    arguments are device tensors (so the call orders after the work that made
    them), else the null stream."""
    if stream is None:
        if not on_device:
            return C.c_void_p(0)
        import torch

        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _check_device_tensor(t, name: str, device: int):
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor when the other arguments are device tensors")
    if not t.is_cuda or t.dtype != torch.float64:
        raise ValueError(f"{name} must be a float64 tensor on the GPU")
    if t.device.index != device:
        raise ValueError(f"{name} is on cuda:{t.device.index}, the handle on cuda:{device}")


class Handle:
    """One analyzed pattern and its factors (``glu_handle``)."""

    def __init__(self, device: int = 0, ordering: int = GLU_ORDER_AMD, force_mode: int = GLU_MODE_AUTO,
                 stream_threshold: int = 0, large_threshold: int = 0, max_device_bytes: int = 0,
                 dense_tail: int = 0, gpu_analysis: bool = False, precision: int = 0,
                 refine_max_iters: int = 0, dense_gemm: int = 0):
        self._h = C.c_void_p()
        opt = glu_options(ordering, force_mode, stream_threshold, large_threshold, max_device_bytes,
                          dense_tail, int(gpu_analysis), precision, refine_max_iters, dense_gemm)
        rc = lib().glu_create(C.byref(self._h), device, C.byref(opt))
        if rc != GLU_OK:
            raise GluError(rc, "glu_create")
        self.device = device
        self.n = 0

    def close(self):
        if self._h:
            lib().glu_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, where: str):
        if rc != GLU_OK:
            col = lib().glu_failed_column(self._h) if rc in (GLU_ERR_ZERO_PIVOT, GLU_ERR_STRUCT_SINGULAR) else -1
            raise GluError(rc, where, col)

    def analyze(self, n: int, colptr, rowind, perm=None):
        cp = np.ascontiguousarray(colptr, dtype=np.int64).reshape(-1)
        ri = np.ascontiguousarray(rowind, dtype=np.int32).reshape(-1)
        if n < 0 or cp.size != n + 1:
            raise ValueError(f"colptr must hold n + 1 = {n + 1} entries, not {cp.size}")
        if n > 0 and (cp[-1] < 0 or ri.size < cp[-1]):
            raise ValueError(f"rowind holds {ri.size} entries, colptr[n] = {cp[-1]}")
        pm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32).reshape(-1)
        if pm is not None and pm.size != n:
            raise ValueError(f"perm must hold n = {n} entries, not {pm.size}")
        self._check(lib().glu_analyze(self._h, n, _ptr(cp), _ptr(ri), _ptr(pm)), "glu_analyze")
        self.n = n
        return self

    def _values(self, values):
        """Values in A's CSC order: a host array, or a float64 tensor on the
        handle's device; exactly nnz(A) of them."""
        nnz = self.query()["nnz_a"]
        if isinstance(values, np.ndarray):
            v = np.ascontiguousarray(values, dtype=np.float64).reshape(-1)
            if v.size != nnz:
                raise ValueError(f"values has {v.size} entries, the analyzed pattern {nnz}")
            return v, 0
        import torch

        if not isinstance(values, torch.Tensor) or values.dtype != torch.float64 or not values.is_contiguous():
            raise ValueError("values must be a NumPy array or a contiguous float64 tensor")
        if values.numel() != nnz:
            raise ValueError(f"values has {values.numel()} entries, the analyzed pattern {nnz}")
        if not values.is_cuda:
            return values.numpy(), 0
        _check_device_tensor(values, "values", self.device)
        return values, 1

    def factor(self, values, stream=None):
        v, on_dev = self._values(values)
        self._check(lib().glu_factor(self._h, _ptr(v), on_dev, _stream(stream, bool(on_dev))), "glu_factor")

    def refactor(self, values, stream=None):
        v, on_dev = self._values(values)
        self._check(lib().glu_refactor(self._h, _ptr(v), on_dev, _stream(stream, bool(on_dev))), "glu_refactor")

    def solve(self, b, x=None, stream=None):
        """Solve A X = B.  b: (n,) or (n, nrhs) float64, NumPy (host) or torch
        tensor on the device (column-major storage, i.e. a transposed view of a
        contiguous (nrhs, n) tensor or a 1-D tensor)."""
        if isinstance(b, np.ndarray):
            if b.shape[0] != self.n:
                raise ValueError(f"b must have n = {self.n} rows")
            bb = np.asfortranarray(b.reshape(b.shape[0], -1), dtype=np.float64)
            n, nrhs = bb.shape
            if x is not None and (not isinstance(x, np.ndarray) or x.dtype != np.float64 or
                                  x.size != n * nrhs or not (x.flags.f_contiguous or x.ndim == 1)):
                raise ValueError("x must be a float64 column-major NumPy array shaped like b")
            xx = np.zeros((n, nrhs), order="F") if x is None else x
            self._check(lib().glu_solve(self._h, nrhs, _ptr(bb), n, _ptr(xx), n, 0, _stream(stream)),
                        "glu_solve")
            return xx.reshape(b.shape)
        import torch

        _check_device_tensor(b, "b", self.device)
        if b.dim() not in (1, 2) or b.shape[0] != self.n:
            raise ValueError(f"b must be (n,) or (n, nrhs) with n = {self.n}")
        if b.dim() == 1:
            if b.stride(0) != 1:
                raise ValueError("a 1-D device right-hand side must be contiguous")
            n, nrhs, ldb = b.shape[0], 1, b.shape[0]
        else:
            n, nrhs = b.shape
            if b.stride(0) != 1 or (nrhs > 1 and b.stride(1) < n):
                raise ValueError("device right-hand sides must be column-major (stride(0) == 1)")
            ldb = max(b.stride(1), n)
        if x is None:
            x = torch.empty((nrhs, n), dtype=torch.float64, device=b.device).t() if b.dim() == 2 else \
                torch.empty(n, dtype=torch.float64, device=b.device)
        _check_device_tensor(x, "x", self.device)
        if tuple(x.shape) != tuple(b.shape):
            raise ValueError(f"x has shape {tuple(x.shape)}, b {tuple(b.shape)}")
        if x.stride(0) != 1 or (x.dim() == 2 and nrhs > 1 and x.stride(1) < n):
            raise ValueError("x must be column-major (stride(0) == 1)")
        ldx = n if x.dim() == 1 else max(x.stride(1), n)
        self._check(lib().glu_solve(self._h, nrhs, _ptr(b), ldb, _ptr(x), ldx, 1, _stream(stream, True)),
                    "glu_solve")
        return x

    def solve_noalloc(self, b, x, stream=None):
        """``glu_solve_noalloc``: the device solve with every scratch buffer in
        the library's static per-GPU array (no allocation).  b, x: float64
        device tensors on the handle's device, (n,) or column-major (n, nrhs)."""
        _check_device_tensor(b, "b", self.device)
        _check_device_tensor(x, "x", self.device)
        if b.dim() not in (1, 2) or b.shape[0] != self.n or tuple(x.shape) != tuple(b.shape):
            raise ValueError(f"b and x must be (n,) or (n, nrhs) with n = {self.n}, equal shapes")
        if b.stride(0) != 1 or x.stride(0) != 1:
            raise ValueError("device right-hand sides must be column-major (stride(0) == 1)")
        nrhs = 1 if b.dim() == 1 else b.shape[1]
        ldb = self.n if b.dim() == 1 else max(b.stride(1), self.n)
        ldx = self.n if x.dim() == 1 else max(x.stride(1), self.n)
        self._check(lib().glu_solve_noalloc(self._h, nrhs, _ptr(b), ldb, _ptr(x), ldx, _stream(stream, True)),
                    "glu_solve_noalloc")
        return x

    @staticmethod
    def noalloc_capacity() -> int:
        return int(lib().glu_solve_noalloc_capacity())

    def query(self) -> dict:
        info = glu_info()
        self._check(lib().glu_query(self._h, C.byref(info)), "glu_query")
        return info.as_dict()

    def export_symbolic(self) -> dict:
        q = self.query()
        n = q["n"]
        out = dict(
            perm=np.zeros(n, np.int32),
            lu_colptr=np.zeros(n + 1, np.int64),
            lu_rowind=np.zeros(max(q["nnz_lu"], 1), np.int32),
            dag_ptr=np.zeros(n + 1, np.int64),
            dag_idx=np.zeros(max(q["n_dag_edges"], 1), np.int32),
            level_ptr=np.zeros(q["n_levels"] + 1, np.int32),
            level_cols=np.zeros(max(n, 1), np.int32),
        )
        self._check(lib().glu_export_symbolic(
            self._h, _ptr(out["perm"]), _ptr(out["lu_colptr"]), _ptr(out["lu_rowind"]), _ptr(out["dag_ptr"]),
            _ptr(out["dag_idx"]), _ptr(out["level_ptr"]), _ptr(out["level_cols"])), "glu_export_symbolic")
        out["lu_rowind"] = out["lu_rowind"][: q["nnz_lu"]]
        out["dag_idx"] = out["dag_idx"][: q["n_dag_edges"]]
        out["level_cols"] = out["level_cols"][:n]
        return out

    def export_factors(self) -> np.ndarray:
        q = self.query()
        v = np.zeros(max(q["nnz_lu"], 1), np.float64)
        self._check(lib().glu_export_factors(self._h, _ptr(v)), "glu_export_factors")
        return v[: q["nnz_lu"]]

    def failed_column(self) -> int:
        return int(lib().glu_failed_column(self._h))


def mc64(n: int, colptr, rowind, values):
    """``glu_mc64``: maximum-product transversal and scalings of A (host).

    Returns (row_perm, row_scale, col_scale): row_perm[j] is the row of A
    matched to column j; diag(row_scale) A diag(col_scale) has magnitudes
    <= 1 with the matched entries 1."""
    cp = np.ascontiguousarray(colptr, dtype=np.int64).reshape(-1)
    ri = np.ascontiguousarray(rowind, dtype=np.int32).reshape(-1)
    v = np.ascontiguousarray(values, dtype=np.float64).reshape(-1)
    if n < 0 or cp.size != n + 1:
        raise ValueError(f"colptr must hold n + 1 = {n + 1} entries, not {cp.size}")
    if n > 0 and (cp[-1] < 0 or ri.size < cp[-1] or v.size < cp[-1]):
        raise ValueError(f"rowind/values hold {ri.size}/{v.size} entries, colptr[n] = {cp[-1]}")
    perm = np.empty(max(n, 1), np.int32)
    dr = np.empty(max(n, 1), np.float64)
    dc = np.empty(max(n, 1), np.float64)
    rc = lib().glu_mc64(n, _ptr(cp), _ptr(ri), _ptr(v), _ptr(perm), _ptr(dr), _ptr(dc))
    if rc != GLU_OK:
        raise GluError(rc, "glu_mc64")
    return perm[:n], dr[:n], dc[:n]


class Batch:
    """``glu_batch``: factorize several analyzed handles together (one launch
    per level wavefront, replayed from a captured graph)."""

    def __init__(self, handles):
        self.handles = list(handles)
        arr = (C.c_void_p * len(self.handles))(*[h._h.value for h in self.handles])
        self._b = C.c_void_p()
        rc = lib().glu_batch_create(C.byref(self._b), arr, len(self.handles))
        if rc != GLU_OK:
            raise GluError(rc, "glu_batch_create")

    def factor(self, values, stream=None):
        """values: one array per handle (NumPy host arrays, or float64 device
        tensors on the handles' device)."""
        if len(values) != len(self.handles):
            raise ValueError("one value array per handle")
        on_dev = 0
        vs = []
        for h, v in zip(self.handles, values):
            vv, od = h._values(v)
            vs.append(vv)
            on_dev |= od
        if on_dev and not all(h._values(v)[1] for h, v in zip(self.handles, values)):
            raise ValueError("values must be all on the host or all on the device")
        arr = (C.c_void_p * len(vs))(*[_ptr(v).value for v in vs])
        rc = lib().glu_batch_factor(self._b, arr, on_dev, _stream(stream, bool(on_dev)))
        if rc != GLU_OK:
            bad = next((i for i, h in enumerate(self.handles) if h.failed_column() >= 0), -1)
            raise GluError(rc, f"glu_batch_factor (handle {bad})" if bad >= 0 else "glu_batch_factor",
                           self.handles[bad].failed_column() if bad >= 0 else -1)

    def solve(self, bs, xs=None, stream=None):
        """Solve every handle's system at once (``glu_batch_solve``).  bs: one
        float64 device tensor per handle, (n_i, nrhs) column-major (a
        transposed view of a contiguous (nrhs, n_i) tensor) with the same nrhs
        for all; xs: outputs of the same shapes (allocated if None)."""
        import torch

        if len(bs) != len(self.handles):
            raise ValueError("one right-hand side per handle")
        nrhs = None
        ldb, ldx, xo = [], [], []
        for i, (h, b) in enumerate(zip(self.handles, bs)):
            _check_device_tensor(b, f"bs[{i}]", h.device)
            if b.dim() != 2 or b.shape[0] != h.n or b.stride(0) != 1:
                raise ValueError(f"bs[{i}] must be ({h.n}, nrhs) column-major")
            if nrhs is None:
                nrhs = b.shape[1]
            elif b.shape[1] != nrhs:
                raise ValueError("every right-hand side block needs the same nrhs")
            if nrhs > 1 and b.stride(1) < h.n:
                raise ValueError(f"bs[{i}] must be column-major")
            ldb.append(max(b.stride(1), h.n))
            x = None if xs is None else xs[i]
            if x is None:
                x = torch.empty((nrhs, h.n), dtype=torch.float64, device=b.device).t()
            _check_device_tensor(x, f"xs[{i}]", h.device)
            if tuple(x.shape) != tuple(b.shape) or x.stride(0) != 1 or (nrhs > 1 and x.stride(1) < h.n):
                raise ValueError(f"xs[{i}] must be ({h.n}, {nrhs}) column-major")
            ldx.append(max(x.stride(1), h.n))
            xo.append(x)
        k = len(self.handles)
        pb = (C.c_void_p * k)(*[b.data_ptr() for b in bs])
        px = (C.c_void_p * k)(*[x.data_ptr() for x in xo])
        lb = (C.c_int64 * k)(*ldb)
        lx = (C.c_int64 * k)(*ldx)
        rc = lib().glu_batch_solve(self._b, nrhs or 0, pb, lb, px, lx, _stream(stream, True))
        if rc != GLU_OK:
            raise GluError(rc, "glu_batch_solve")
        return xo

    def query(self) -> dict:
        cnt, nwf, cap = C.c_int32(), C.c_int32(), C.c_int32()
        tl, tt, ts = C.c_double(), C.c_double(), C.c_double()
        rc = lib().glu_batch_query(self._b, C.byref(cnt), C.byref(nwf), C.byref(cap), C.byref(tl), C.byref(tt),
                                   C.byref(ts))
        if rc != GLU_OK:
            raise GluError(rc, "glu_batch_query")
        return {"count": cnt.value, "n_wavefronts": nwf.value, "captured": bool(cap.value),
                "t_levels_ms": tl.value, "t_total_ms": tt.value, "t_solve_ms": ts.value}

    def close(self):
        if self._b:
            lib().glu_batch_destroy(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
