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

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, NOT_CONVERGED, BREAKDOWN = 0, -1, -2, -3, -4, 1, 2
F32, F64 = 0, 1
EXPORTED = ("merbit_opts_init", "merbit_plan_create", "merbit_plan_set_values", "merbit_plan_info",
            "merbit_plan_export", "merbit_spmv", "merbit_spmv_dual", "merbit_zero_boundary",
            "merbit_pagerank", "merbit_pagerank_noalloc", "merbit_spmm", "merbit_spmm_dual",
            "merbit_spmm_zero_boundary",
            "merbit_pagerank_personalized", "merbit_pagerank_multi", "merbit_transpose",
            "merbit_sddmm", "merbit_gather_values", "merbit_column_scale",
            "merbit_pagerank_adjoint", "merbit_bicgstab", "merbit_tune",
            "merbit_profile_enable", "merbit_profile_read",
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
                ("hot_coverage", ctypes.c_double), ("desc_bits", ctypes.c_int32),
                ("stripes", ctypes.c_int32), ("ranges", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("plan_rows", ctypes.c_int64),
                ("graph_captures", ctypes.c_int64), ("graph_replays", ctypes.c_int64)]


class Opts(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_int32), ("block_lanes", ctypes.c_int32),
                ("commit", ctypes.c_int32), ("hot_columns", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("eager_loops", ctypes.c_int32), ("desc_bits", ctypes.c_int32),
                ("stripes", ctypes.c_int32), ("tune_rhs", ctypes.c_int32)]


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
    lib.merbit_pagerank_noalloc.argtypes = [vp, dbl, dbl, i32, i32, vp, ctypes.POINTER(i32),
                                            ctypes.POINTER(dbl), vp]
    lib.merbit_spmm.argtypes = [vp, vp, i64, vp, i64, i32, vp]
    lib.merbit_spmm_dual.argtypes = [vp, vp, i64, vp, i64, vp, i64, i32, vp]
    lib.merbit_spmm_zero_boundary.argtypes = [vp, vp, i64, i32, vp]
    lib.merbit_pagerank_personalized.argtypes = [vp, dbl, dbl, i32, i32, vp, i32, vp,
                                                 ctypes.POINTER(i32), vp, vp]
    lib.merbit_pagerank_multi.argtypes = [vp, vp, i32, dbl, dbl, i32, i32, vp,
                                          ctypes.POINTER(i32), vp, vp]
    lib.merbit_transpose.argtypes = [vp, vp, vp, vp, vp]
    lib.merbit_sddmm.argtypes = [vp, vp, vp, dbl, vp, vp]
    lib.merbit_gather_values.argtypes = [i32, i64, vp, vp, vp, vp, vp]
    lib.merbit_column_scale.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp]
    lib.merbit_pagerank_adjoint.argtypes = [vp, vp, dbl, dbl, i32, i32, vp, vp,
                                            ctypes.POINTER(i32), ctypes.POINTER(dbl), vp]
    lib.merbit_bicgstab.argtypes = [vp, vp, vp, dbl, i32, i32, ctypes.POINTER(i32),
                                    ctypes.POINTER(dbl), vp]
    lib.merbit_tune.argtypes = [i64, i64, i64, vp, vp, vp, i32, vp, i32, vp, i32, i32,
                                ctypes.POINTER(Opts), vp, vp]
    lib.merbit_profile_enable.argtypes = [vp, i32]
    lib.merbit_profile_read.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(dbl)]
    lib.merbit_plan_destroy.argtypes = [vp]
    lib.merbit_plan_destroy.restype = None
    lib.merbit_last_error.restype = ctypes.c_char_p
    lib.merbit_version.restype = ctypes.c_char_p
    for name in ("merbit_plan_create", "merbit_plan_set_values", "merbit_plan_info",
                 "merbit_plan_export", "merbit_spmv", "merbit_spmv_dual", "merbit_zero_boundary",
                 "merbit_pagerank", "merbit_pagerank_noalloc", "merbit_spmm", "merbit_spmm_dual",
                 "merbit_spmm_zero_boundary", "merbit_pagerank_personalized",
                 "merbit_pagerank_multi", "merbit_transpose", "merbit_sddmm",
                 "merbit_gather_values", "merbit_column_scale", "merbit_pagerank_adjoint",
                 "merbit_bicgstab", "merbit_tune", "merbit_profile_enable",
                 "merbit_profile_read"):
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
    repeated y = A x.  col_ind and values are borrowed (kept referenced).
    stripes = S > 1 plans the column-stripe stack of the matrix (the plan then
    copies col_ind and values; set_values re-copies the values)."""

    def __init__(self, row_ptr: torch.Tensor, col_ind: torch.Tensor, values: torch.Tensor,
                 n_cols: int, *, sigma: int = 0, block_lanes: int = 0, hot_columns: int = -1,
                 commit: str = "auto", blocks_per_cu: int = 0, validate: bool = True,
                 eager_loops: bool = False, desc_bits: int = 32, stripes: int = 0,
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
        opts.eager_loops = 1 if eager_loops else 0
        opts.desc_bits = desc_bits
        opts.stripes = stripes
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
        """Host copies (numpy) of tile_x int32[T+1], tile_y uint32[T+1] and
        lane_desc uint32[lanes] (uint64 for a 64-bit-descriptor plan)."""
        import numpy as np
        T, lanes = ctypes.c_int64(), ctypes.c_int64()
        lib = load()
        _check(lib.merbit_plan_export(self._handle(), None, None, None, ctypes.byref(T),
                                      ctypes.byref(lanes)))
        tx = np.empty(T.value + 1, np.int32)
        ty = np.empty(T.value + 1, np.uint32)
        ld = np.empty(max(lanes.value, 1), np.uint64 if self.info()["desc_bits"] == 64
                      else np.uint32)
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

    def pagerank_noalloc(self, x: torch.Tensor, alpha: float = 0.85, tol: float = 0.0,
                         max_iter: int = 100, check_every: int = 10, stream=None):
        """As pagerank(), through merbit_pagerank_noalloc: the library's fixed
        work array instead of plan-owned buffers, no HIP graphs."""
        if x.numel() != self.n_rows:
            raise ValueError("x length mismatch")
        it = ctypes.c_int()
        res = ctypes.c_double()
        rc = _check(load().merbit_pagerank_noalloc(self._handle(), float(alpha), float(tol),
                                                   int(max_iter), int(check_every),
                                                   _dev(x, self.dtype, "x"), ctypes.byref(it),
                                                   ctypes.byref(res), _stream(stream)),
                    allow=(OK, NOT_CONVERGED))
        return it.value, res.value, rc == OK

    # -- batched forms ------------------------------------------------------
    def _mat(self, t, rows, name):
        """Row-major [rows, k] GPU tensor with unit column stride -> (ptr, ld, k)."""
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a GPU tensor")
        if t.dtype != self.dtype:
            raise TypeError(f"{name} must be {self.dtype}, got {t.dtype}")
        if t.dim() != 2 or t.shape[0] != rows:
            raise ValueError(f"{name} must have shape ({rows}, k)")
        if t.shape[1] > 1 and t.stride(1) != 1:
            raise TypeError(f"{name} must have unit column stride")
        ld = t.stride(0) if t.shape[0] > 1 else t.shape[1]
        return ctypes.c_void_p(t.data_ptr() if t.numel() else 0), max(ld, t.shape[1]), t.shape[1]

    def spmm(self, X: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        """Y = A X for X of shape (n_cols, k) (overwrites out, shape (n_rows, k))."""
        if out is None:
            out = torch.empty(self.n_rows, X.shape[1], dtype=self.dtype, device=X.device)
        xp, ldx, k = self._mat(X, self.n_cols, "X")
        yp, ldy, ky = self._mat(out, self.n_rows, "Y")
        if ky != k:
            raise ValueError("X and Y differ in column count")
        _check(load().merbit_spmm(self._handle(), xp, ldx, yp, ldy, k, _stream(stream)))
        return out

    def spmm_dual(self, X, Y, Z, stream=None):
        """Y = A X with Y zero at the boundary rows on entry; leaves Z zero there."""
        xp, ldx, k = self._mat(X, self.n_cols, "X")
        yp, ldy, ky = self._mat(Y, self.n_rows, "Y")
        zp, ldz, kz = self._mat(Z, self.n_rows, "Z")
        if not k == ky == kz:
            raise ValueError("X, Y, Z differ in column count")
        _check(load().merbit_spmm_dual(self._handle(), xp, ldx, yp, ldy, zp, ldz, k,
                                       _stream(stream)))
        return Y

    def spmm_zero_boundary(self, Y, stream=None):
        yp, ldy, k = self._mat(Y, self.n_rows, "Y")
        _check(load().merbit_spmm_zero_boundary(self._handle(), yp, ldy, k, _stream(stream)))
        return Y

    def pagerank_personalized(self, sources, X: torch.Tensor | None = None, alpha: float = 0.85,
                              tol: float = 0.0, max_iter: int = 100, check_every: int = 10,
                              stream=None):
        """Personalised PageRank for up to 64 sources at once.  X (n, k) holds
        the initial vectors (default: column j = e_{sources[j]}) and gets the
        ranks.  Returns (X, iterations, per-column last l1 change, converged)."""
        import numpy as np
        src = np.ascontiguousarray(np.asarray(sources, dtype=np.int64).reshape(-1))
        k = src.size
        # checked here, before any device work touches them
        if not 1 <= k <= 64:
            raise MerbitError(EINVAL, "need 1..64 sources")
        if src.min() < 0 or src.max() >= self.n_rows:
            raise MerbitError(EINVAL, "source out of range")
        src = src.astype(np.int32)
        if X is None:
            X = torch.zeros(self.n_rows, k, dtype=self.dtype, device="cuda")
            X[torch.as_tensor(src, dtype=torch.int64, device="cuda"),
              torch.arange(k, device="cuda")] = 1.0
        if tuple(X.shape) != (self.n_rows, k) or not X.is_contiguous():
            raise ValueError(f"X must be a contiguous ({self.n_rows}, {k}) tensor")
        it = ctypes.c_int()
        res = np.zeros(max(k, 1), np.float64)
        rc = _check(load().merbit_pagerank_personalized(
            self._handle(), float(alpha), float(tol), int(max_iter), int(check_every),
            src.ctypes.data_as(ctypes.c_void_p), int(k), _dev(X, self.dtype, "X"),
            ctypes.byref(it), res.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
            allow=(OK, NOT_CONVERGED))
        return X, it.value, res[:k], rc == OK

    def pagerank_multi(self, graph_ptr, x: torch.Tensor, alpha: float = 0.85, tol: float = 0.0,
                       max_iter: int = 100, check_every: int = 10, stream=None):
        """PageRank of every graph on the diagonal (graph g = rows
        graph_ptr[g] .. graph_ptr[g+1]-1), in place on x.  Returns
        (iterations, per-graph last l1 change, converged)."""
        import numpy as np
        gp = np.ascontiguousarray(np.asarray(graph_ptr, dtype=np.int64).reshape(-1))
        G = gp.size - 1
        if x.numel() != self.n_rows:
            raise ValueError("x length mismatch")
        it = ctypes.c_int()
        res = np.zeros(max(G, 1), np.float64)
        rc = _check(load().merbit_pagerank_multi(
            self._handle(), gp.ctypes.data_as(ctypes.c_void_p), int(G), float(alpha), float(tol),
            int(max_iter), int(check_every), _dev(x, self.dtype, "x"), ctypes.byref(it),
            res.ctypes.data_as(ctypes.c_void_p), _stream(stream)), allow=(OK, NOT_CONVERGED))
        return it.value, res[:max(G, 0)], rc == OK

    # -- adjoint pieces -----------------------------------------------------
    def transpose(self, stream=None):
        """CSR of A^T on the device: (rowT_ptr int32[n_cols+1], colT int32[nnz],
        perm int32[nnz]); A^T's values are values[perm]."""
        dev = self._keep[1].device
        rowT = torch.empty(self.n_cols + 1, dtype=torch.int32, device=dev)
        colT = torch.empty(self.nnz, dtype=torch.int32, device=dev)
        perm = torch.empty(self.nnz, dtype=torch.int32, device=dev)
        _check(load().merbit_transpose(self._handle(), _dev(rowT, torch.int32, "rowT"),
                                       _dev(colT, torch.int32, "colT"),
                                       _dev(perm, torch.int32, "perm"), _stream(stream)))
        return rowT, colT, perm

    def sddmm(self, g: torch.Tensor, x: torch.Tensor, scale: float = 1.0,
              out: torch.Tensor | None = None, stream=None):
        """out[e] = scale g[row(e)] x[col(e)] on the plan's nonzeros."""
        if g.numel() != self.n_rows or x.numel() != self.n_cols:
            raise ValueError("g / x length mismatch")
        if out is None:
            out = torch.empty(self.nnz, dtype=self.dtype, device=g.device)
        if out.numel() != self.nnz:
            raise ValueError("out length mismatch")
        _check(load().merbit_sddmm(self._handle(), _dev(g, self.dtype, "g"),
                                   _dev(x, self.dtype, "x"), float(scale),
                                   _dev(out, self.dtype, "out"), _stream(stream)))
        return out

    def pagerank_adjoint(self, plan_t: "Plan", g: torch.Tensor, lam: torch.Tensor,
                         alpha: float = 0.85, tol: float = 0.0, max_iter: int = 100,
                         check_every: int = 10, stream=None):
        """In place on lam: lambda = g + alpha P^T lambda + (alpha/n)(1^T lambda) d.
        plan_t is the plan of this matrix's transpose.  Returns
        (iterations, last l1 change, converged)."""
        if g.numel() != self.n_rows or lam.numel() != self.n_rows:
            raise ValueError("g / lambda length mismatch")
        it = ctypes.c_int()
        res = ctypes.c_double()
        rc = _check(load().merbit_pagerank_adjoint(
            self._handle(), plan_t._handle(), float(alpha), float(tol), int(max_iter),
            int(check_every), _dev(g, self.dtype, "g"), _dev(lam, self.dtype, "lambda"),
            ctypes.byref(it), ctypes.byref(res), _stream(stream)), allow=(OK, NOT_CONVERGED))
        return it.value, res.value, rc == OK

    # -- BiCGSTAB -----------------------------------------------------------
    def bicgstab(self, b: torch.Tensor, x: torch.Tensor, tol: float = 1e-10,
                 max_iter: int = 20000, check_every: int = 10, stream=None):
        """Solve A x = b in place on x (x_0 in).  Returns (iterations,
        ||r|| / ||b|| at the last test, status) with status one of
        "converged", "iteration cap", "breakdown"."""
        if b.numel() != self.n_rows or x.numel() != self.n_rows:
            raise ValueError("b / x length mismatch")
        it = ctypes.c_int()
        res = ctypes.c_double()
        rc = _check(load().merbit_bicgstab(self._handle(), _dev(b, self.dtype, "b"),
                                           _dev(x, self.dtype, "x"), float(tol), int(max_iter),
                                           int(check_every), ctypes.byref(it), ctypes.byref(res),
                                           _stream(stream)), allow=(OK, NOT_CONVERGED, BREAKDOWN))
        if rc == OK:
            status = "converged" if tol > 0 else "done"
        else:
            status = {NOT_CONVERGED: "iteration cap", BREAKDOWN: "breakdown"}[rc]
        return it.value, res.value, status

    # -- timing -------------------------------------------------------------
    def profile_enable(self, on: bool = True):
        _check(load().merbit_profile_enable(self._handle(), 1 if on else 0))

    def profile_read(self):
        """(number of timed fused-kernel launches, their summed ms); clears."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(load().merbit_profile_read(self._handle(), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value


def gather_values(perm: torch.Tensor, src: torch.Tensor, src2: torch.Tensor | None = None,
                  out: torch.Tensor | None = None, stream=None):
    """out[i] = src[perm[i]] (* src2[perm[i]])."""
    code = _vdtype(src)
    if out is None:
        out = torch.empty(perm.numel(), dtype=src.dtype, device=src.device)
    if src.numel() != perm.numel() or out.numel() != perm.numel() or (
            src2 is not None and src2.numel() != perm.numel()):
        raise ValueError("length mismatch")
    _check(load().merbit_gather_values(
        code, perm.numel(), _dev(perm, torch.int32, "perm"), _dev(src, src.dtype, "src"),
        None if src2 is None else _dev(src2, src.dtype, "src2"), _dev(out, src.dtype, "out"),
        _stream(stream)))
    return out


def column_scale(col: torch.Tensor, a: torch.Tensor, s: torch.Tensor,
                 t: torch.Tensor | None = None, out: torch.Tensor | None = None, stream=None):
    """out[e] = (a[e] - t[col[e]]) / s[col[e]] (t optional)."""
    code = _vdtype(a)
    if out is None:
        out = torch.empty_like(a)
    if a.numel() != col.numel() or out.numel() != col.numel():
        raise ValueError("length mismatch")
    _check(load().merbit_column_scale(
        code, col.numel(), _dev(col, torch.int32, "col"), _dev(a, a.dtype, "a"),
        None if t is None else _dev(t, a.dtype, "t"), _dev(s, a.dtype, "s"),
        _dev(out, a.dtype, "out"), _stream(stream)))
    return out


def tune(row_ptr: torch.Tensor, col_ind: torch.Tensor, values: torch.Tensor, n_cols: int, *,
         sigmas=None, block_lanes=None, reps: int = 20, commit: str = "auto",
         hot_columns: int = -1, desc_bits: int = 32, stripes: int = 0, rhs: int = 0,
         stream=None):
    """Time the fused SpMV (rhs = 0) or the SpMM over rhs right-hand sides
    for every (sigma, block_lanes) candidate on this matrix.  Returns
    ({"sigma": s, "block_lanes": b}, {(s, b): mean us})."""
    import numpy as np
    lib = load()
    code = _vdtype(values)
    n_rows = row_ptr.numel() - 1
    if sigmas is None and desc_bits == 64:
        sigmas = [16, 20, 24, 28, 32] if code == F32 else [14, 16, 20, 24]
    elif sigmas is None:
        sigmas = list(range(7, 13)) if code == F32 else list(range(4, 11))
    if block_lanes is None:
        block_lanes = [256, 512, 1024]
    sg = np.ascontiguousarray(sigmas, np.int32)
    bl = np.ascontiguousarray(block_lanes, np.int32)
    us = np.full(sg.size * bl.size, -1.0, np.float32)
    opts = Opts()
    lib.merbit_opts_init(ctypes.byref(opts))
    opts.commit = _COMMIT[commit]
    opts.hot_columns = hot_columns
    opts.desc_bits = desc_bits
    opts.stripes = stripes
    opts.tune_rhs = rhs
    _check(lib.merbit_tune(n_rows, int(n_cols), col_ind.numel(),
                           _dev(row_ptr, torch.int32, "row_ptr"),
                           _dev(col_ind, torch.int32, "col_ind"),
                           _dev(values, values.dtype, "values"), code,
                           sg.ctypes.data_as(ctypes.c_void_p), int(sg.size),
                           bl.ctypes.data_as(ctypes.c_void_p), int(bl.size), int(reps),
                           ctypes.byref(opts), us.ctypes.data_as(ctypes.c_void_p),
                           _stream(stream)))
    table = {(int(s), int(b)): float(us[i * bl.size + j])
             for i, s in enumerate(sg) for j, b in enumerate(bl)}
    return {"sigma": opts.sigma, "block_lanes": opts.block_lanes}, table


def version() -> str:
    return load().merbit_version().decode()
