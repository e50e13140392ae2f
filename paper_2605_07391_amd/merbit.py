"""Python binding of libmerbit.so (include/merbit.h): argument marshalling only.

Every step of the computation runs in the library's HIP kernels; this module
passes device pointers of torch tensors and torch's current HIP stream.  There
is no CPU fallback: if the library is missing or the tensors are not on the
GPU, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch  # imported first so that libmerbit binds to torch's HIP runtime

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmerbit.so")
_lib = None

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, NOT_CONVERGED = 0, -1, -2, -3, -4, 1
F32, F64 = 0, 1
EXPORTED = ("merbit_opts_init", "merbit_plan_create", "merbit_plan_set_values", "merbit_plan_info",
            "merbit_plan_export", "merbit_spmv", "merbit_spmv_dual", "merbit_zero_boundary",
            "merbit_pagerank", "merbit_profile_enable", "merbit_profile_read",
            "merbit_plan_destroy", "merbit_last_error", "merbit_version")


class MerbitError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"merbit error {code}: {msg}")
        self.code = code


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("tile_num", ctypes.c_int64), ("lane_num", ctypes.c_int64),
                ("fast_tiles", ctypes.c_int64), ("chunk_num", ctypes.c_int64),
                ("grid", ctypes.c_int32), ("chunks_per_block", ctypes.c_int32),
                ("hot_columns", ctypes.c_int32), ("omega", ctypes.c_int32),
                ("sigma", ctypes.c_int32), ("block_lanes", ctypes.c_int32),
                ("offset_bits", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("commit", ctypes.c_int32),
                ("hot_coverage", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_int32), ("block_lanes", ctypes.c_int32),
                ("commit", ctypes.c_int32), ("hot_columns", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


COMMIT_AUTO, COMMIT_BLOCK, COMMIT_WAVE = 0, 1, 2
_COMMIT = {"auto": COMMIT_AUTO, "block": COMMIT_BLOCK, "wave": COMMIT_WAVE}


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load libmerbit.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built (python -m paper_2605_07391_amd.build)")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.merbit_plan_create.argtypes = [i64, i64, i64, vp, vp, vp, i32, ctypes.POINTER(Opts), vp,
                                       ctypes.POINTER(vp)]
    lib.merbit_opts_init.argtypes = [ctypes.POINTER(Opts)]
    lib.merbit_opts_init.restype = None
    lib.merbit_plan_set_values.argtypes = [vp, vp]
    lib.merbit_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.merbit_plan_export.argtypes = [vp, vp, vp, vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.merbit_spmv.argtypes = [vp, vp, vp, vp]
    lib.merbit_spmv_dual.argtypes = [vp, vp, vp, vp, vp]
    lib.merbit_zero_boundary.argtypes = [vp, vp, vp]
    lib.merbit_pagerank.argtypes = [vp, dbl, dbl, i32, i32, vp, ctypes.POINTER(i32),
                                    ctypes.POINTER(dbl), vp]
    lib.merbit_profile_enable.argtypes = [vp, i32]
    lib.merbit_profile_read.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(dbl)]
    lib.merbit_plan_destroy.argtypes = [vp]
    lib.merbit_plan_destroy.restype = None
    lib.merbit_last_error.restype = ctypes.c_char_p
    lib.merbit_version.restype = ctypes.c_char_p
    for name in ("merbit_plan_create", "merbit_plan_set_values", "merbit_plan_info",
                 "merbit_plan_export", "merbit_spmv", "merbit_spmv_dual", "merbit_zero_boundary",
                 "merbit_pagerank", "merbit_profile_enable", "merbit_profile_read"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc, allow=(OK,)):
    if rc not in allow:
        raise MerbitError(rc, load().merbit_last_error().decode())
    return rc


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t: torch.Tensor, dtype, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0)


def _vdtype(values: torch.Tensor):
    if values.dtype == torch.float32:
        return F32
    if values.dtype == torch.float64:
        return F64
    raise TypeError("values must be float32 or float64")


class Plan:
    """A reusable MERBIT plan: TILE built once on the GPU from row_ptr, then
    repeated y = A x.  col_ind and values are borrowed (kept referenced)."""

    def __init__(self, row_ptr: torch.Tensor, col_ind: torch.Tensor, values: torch.Tensor,
                 n_cols: int, *, sigma: int = 0, block_lanes: int = 0, hot_columns: int = -1,
                 commit: str = "auto", blocks_per_cu: int = 0, validate: bool = True,
                 stream=None):
        lib = load()
        self.dtype = values.dtype
        self._code = _vdtype(values)
        self.n_rows = row_ptr.numel() - 1
        self.n_cols = int(n_cols)
        self.nnz = col_ind.numel()
        rp = _dev(row_ptr, torch.int32, "row_ptr")
        ci = _dev(col_ind, torch.int32, "col_ind")
        va = _dev(values, values.dtype, "values")
        if values.numel() != self.nnz:
            raise ValueError("values and col_ind differ in length")
        self._keep = [row_ptr, col_ind, values]
        opts = Opts()
        lib.merbit_opts_init(ctypes.byref(opts))
        opts.sigma = sigma
        opts.block_lanes = block_lanes
        opts.commit = _COMMIT[commit]
        opts.hot_columns = hot_columns
        opts.validate = 1 if validate else 0
        opts.blocks_per_cu = blocks_per_cu
        h = ctypes.c_void_p()
        _check(lib.merbit_plan_create(self.n_rows, self.n_cols, self.nnz, rp, ci, va, self._code,
                                      ctypes.byref(opts), _stream(stream), ctypes.byref(h)))
        self._h = h

    # -- lifecycle ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().merbit_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _handle(self):
        if self._h is None:
            raise RuntimeError("plan is closed")
        return self._h

    # -- plan ---------------------------------------------------------------
    def set_values(self, values: torch.Tensor):
        _check(load().merbit_plan_set_values(self._handle(), _dev(values, self.dtype, "values")))
        self._keep[2] = values

    def info(self) -> dict:
        inf = PlanInfo()
        _check(load().merbit_plan_info(self._handle(), ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in PlanInfo._fields_}

    def export(self):
        """Host copies (numpy) of tile_x int32[T+1], tile_y uint32[T+1], lane_desc uint32[lanes]."""
        import numpy as np
        T, lanes = ctypes.c_int64(), ctypes.c_int64()
        lib = load()
        _check(lib.merbit_plan_export(self._handle(), None, None, None, ctypes.byref(T),
                                      ctypes.byref(lanes)))
        tx = np.empty(T.value + 1, np.int32)
        ty = np.empty(T.value + 1, np.uint32)
        ld = np.empty(max(lanes.value, 1), np.uint32)
        _check(lib.merbit_plan_export(self._handle(), tx.ctypes.data_as(ctypes.c_void_p),
                                      ty.ctypes.data_as(ctypes.c_void_p),
                                      ld.ctypes.data_as(ctypes.c_void_p), None, None))
        return tx, ty, ld[:lanes.value]

    # -- SpMV ---------------------------------------------------------------
    def spmv(self, x: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """y = A x (overwrites out)."""
        if out is None:
            out = torch.empty(self.n_rows, dtype=self.dtype, device=x.device)
        if x.numel() != self.n_cols or out.numel() != self.n_rows:
            raise ValueError("x / y length mismatch")
        _check(load().merbit_spmv(self._handle(), _dev(x, self.dtype, "x"),
                                  _dev(out, self.dtype, "y"), _stream(stream)))
        return out

    def spmv_dual(self, x, y, z, stream=None):
        """y = A x with y zero at the boundary rows on entry; leaves z zero there."""
        if x.numel() != self.n_cols or y.numel() != self.n_rows or z.numel() != self.n_rows:
            raise ValueError("x / y / z length mismatch")
        _check(load().merbit_spmv_dual(self._handle(), _dev(x, self.dtype, "x"),
                                       _dev(y, self.dtype, "y"), _dev(z, self.dtype, "z"),
                                       _stream(stream)))
        return y

    def zero_boundary(self, v, stream=None):
        if v.numel() != self.n_rows:
            raise ValueError("length mismatch")
        _check(load().merbit_zero_boundary(self._handle(), _dev(v, self.dtype, "v"),
                                           _stream(stream)))
        return v

    # -- PageRank -----------------------------------------------------------
    def pagerank(self, x: torch.Tensor, alpha: float = 0.85, tol: float = 0.0,
                 max_iter: int = 100, check_every: int = 10, stream=None):
        """In-place power iteration on x (x_0 in, ranks out).
        Returns (iterations, last l1 change, converged)."""
        if x.numel() != self.n_rows:
            raise ValueError("x length mismatch")
        it = ctypes.c_int()
        res = ctypes.c_double()
        rc = _check(load().merbit_pagerank(self._handle(), float(alpha), float(tol),
                                           int(max_iter), int(check_every),
                                           _dev(x, self.dtype, "x"), ctypes.byref(it),
                                           ctypes.byref(res), _stream(stream)),
                    allow=(OK, NOT_CONVERGED))
        return it.value, res.value, rc == OK

    # -- timing -------------------------------------------------------------
    def profile_enable(self, on: bool = True):
        _check(load().merbit_profile_enable(self._handle(), 1 if on else 0))

    def profile_read(self):
        """(number of timed fused-kernel launches, their summed ms); clears."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(load().merbit_profile_read(self._handle(), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value


def version() -> str:
    return load().merbit_version().decode()
