"""CPU oracle for the MERBIT hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this module.  The product path never calls it.  It wraps the plain
sequential C in ``merbit_oracle.c`` (built with gcc, no OpenMP) plus a few
numpy helpers that restate the paper's closed forms.

Every function cites the part of the paper ("MERBIT: A GPU-Based SpMV Method
for Iterative Workloads") it follows.  Functions and their pins:

* ``spmv`` (Sec. 3.1) -- pinned by dense brute force and special matrices.
* ``path_coords`` (Sec. 3.3 walk) and ``merge_search`` (Algorithm 1) -- two
  derivations pinned against each other on every diagonal and against the
  step string built row by row.
* ``plan`` (Sec. 4.1) -- pinned by the worked example of Sec. 4.1.1, by the
  closed forms for tile_num / lane_num / field widths, by invariants and by
  ``plan_replay`` reproducing ``spmv`` bit for bit.
* ``plan64`` / ``plan_replay64`` (the same TILE with 64-bit descriptors,
  sigma up to 40) -- pinned by the brute-force TILE built from the step
  string, equality with ``plan`` for sigma <= 12, the fit condition and the
  replay reproducing ``spmv`` bit for bit.
* ``pagerank`` (Sec. 5.5.1) -- pinned by closed-form cases, by a dense direct
  solve of the stationary equation and by the mass / contraction invariants.
* ``spmm`` (Sec. 3.1 per column) -- pinned by dense brute force.
* ``pagerank_teleport`` / ``personalized_pagerank`` (the power method of
  Sec. 5.5.1 with a general teleport vector) -- pinned by a dense direct
  solve, by closed forms and by reducing to ``pagerank`` for a uniform vector.
* ``pagerank_multi`` (independent graphs on the diagonal of one matrix) --
  each graph's PageRank computed on its own slice; pinned by the block
  structure (a graph's ranks do not depend on the other graphs).
* ``bicgstab`` (Sec. 5.5.2, unpreconditioned BiCGSTAB) -- pinned by dense
  solves of well-conditioned systems, exact termination in one iteration on
  a multiple of the identity, the true residual ||b - A x|| at exit, and the
  textbook recurrences checked step by step in numpy.
* ``transpose`` (CSR of A^T, stable) -- pinned by dense transposes, the
  double-transpose identity and the adjoint identity <A x, g> = <x, A^T g>.
* ``pagerank_adjoint``, ``pagerank_value_grad``, ``colnorm`` /
  ``colnorm_backward``, ``pagerank_loss_grad`` (the derivative of the
  PageRank fixed point of Sec. 5.5.1 with respect to the matrix values) --
  pinned by a dense solve of the adjoint equation and by central finite
  differences of the oracle's own converged PageRank.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "merbit_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32 = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_u32 = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_f64 = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def build() -> str:
    """Compile the oracle with gcc (single threaded, -O2), and the benchmark's
    timed CPU baseline beside it (``cpu_baseline.c``, OpenMP)."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC,
                    "-lm"], check=True)
    os.replace(tmp, _LIB)
    from . import cpu_baseline
    cpu_baseline.build()
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    c_i64, c_int, c_dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.or_spmv.restype = None
    lib.or_spmv.argtypes = [c_i64, _i32, _i32, _f64, _f64, _f64]
    lib.or_abs_spmv.restype = None
    lib.or_abs_spmv.argtypes = [c_i64, _i32, _i32, _f64, _f64, _f64]
    lib.or_path_coords.restype = None
    lib.or_path_coords.argtypes = [c_i64, _i32, _i32, _i32]
    lib.or_merge_search.restype = None
    lib.or_merge_search.argtypes = [c_i64, _i32, c_i64, ctypes.POINTER(c_i64),
                                    ctypes.POINTER(c_i64)]
    lib.or_offset_bits.restype = c_int
    lib.or_offset_bits.argtypes = [c_int, c_int]
    lib.or_plan.restype = c_int
    lib.or_plan.argtypes = [c_i64, _i32, c_int, c_int, _i32, _u32, _u32]
    lib.or_plan_replay.restype = c_int
    lib.or_plan_replay.argtypes = [c_i64, c_i64, c_int, c_int, _i32, _u32, _u32, _i32, _f64,
                                   _f64, _f64, ctypes.c_void_p]
    _u64 = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
    lib.or_plan64.restype = c_int
    lib.or_plan64.argtypes = [c_i64, _i32, c_int, c_int, _i32, _u32, _u64]
    lib.or_plan_replay64.restype = c_int
    lib.or_plan_replay64.argtypes = [c_i64, c_i64, c_int, c_int, _i32, _u32, _u64, _i32, _f64,
                                     _f64, _f64]
    lib.or_spmm.restype = None
    lib.or_spmm.argtypes = [c_i64, _i32, _i32, _f64, c_int, _f64, _f64]
    lib.or_pagerank_teleport.restype = c_int
    lib.or_pagerank_teleport.argtypes = [c_i64, _i32, _i32, _f64, c_dbl, c_int, _f64, _f64, _f64,
                                         ctypes.c_void_p]
    lib.or_transpose.restype = c_int
    lib.or_transpose.argtypes = [c_i64, c_i64, _i32, _i32, _i32, _i32, _i32]
    lib.or_pagerank_adjoint.restype = c_int
    lib.or_pagerank_adjoint.argtypes = [c_i64, _i32, _i32, _f64, c_dbl, c_int, _f64, _f64]
    lib.or_bicgstab.restype = c_int
    lib.or_bicgstab.argtypes = [c_i64, _i32, _i32, _f64, _f64, _f64, c_dbl, c_int, _f64,
                                ctypes.c_void_p, ctypes.POINTER(c_int)]
    lib.or_pagerank.restype = c_int
    lib.or_pagerank.argtypes = [c_i64, _i32, _i32, _f64, c_dbl, c_int, _f64, _f64,
                                ctypes.c_void_p, ctypes.c_void_p]
    _lib = lib
    return lib


def _i32a(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64a(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------ SpMV --

def spmv(row_ptr, col, values, x) -> np.ndarray:
    """Sec. 3.1: y = A x with y[r] = sum_k values[k] x[col[k]] (long double)."""
    row_ptr = _i32a(row_ptr)
    n = len(row_ptr) - 1
    y = np.empty(max(n, 1), np.float64)
    _load().or_spmv(n, row_ptr, _i32a(col), _f64a(values), _f64a(x) if len(x) else np.zeros(1),
                    y)
    return y[:n]


def abs_spmv(row_ptr, col, values, x) -> np.ndarray:
    """(|A| |x|)[r]: the per-row scale of the SpMV parity tolerance."""
    row_ptr = _i32a(row_ptr)
    n = len(row_ptr) - 1
    y = np.empty(max(n, 1), np.float64)
    _load().or_abs_spmv(n, row_ptr, _i32a(col), _f64a(values),
                        _f64a(x) if len(x) else np.zeros(1), y)
    return y[:n]


# ------------------------------------------------------------ merge path --

def path_coords(row_ptr):
    """Sec. 3.3: coordinates (xs[d], ys[d]) after d steps, d = 0 .. m + n."""
    row_ptr = _i32a(row_ptr)
    n = len(row_ptr) - 1
    L = int(row_ptr[-1]) + n
    xs = np.empty(L + 1, np.int32)
    ys = np.empty(L + 1, np.int32)
    _load().or_path_coords(n, row_ptr, xs, ys)
    return xs, ys


def merge_search(row_ptr, diag: int):
    """Algorithm 1 (merge_search): path coordinate on diagonal `diag`."""
    row_ptr = _i32a(row_ptr)
    xo, yo = ctypes.c_int64(), ctypes.c_int64()
    _load().or_merge_search(len(row_ptr) - 1, row_ptr, int(diag), ctypes.byref(xo),
                            ctypes.byref(yo))
    return xo.value, yo.value


def offset_bits(omega: int, sigma: int) -> int:
    """Sec. 4.1.1: b = ceil(log2(omega sigma)) bits per offset field."""
    return int(_load().or_offset_bits(omega, sigma))


def plan_sizes(n_rows: int, nnz: int, omega: int, sigma: int):
    """Sec. 4.1.1: (tile_num, lane_num) = (ceil((m+n)/(omega sigma)), ceil((m+n)/sigma))."""
    L = nnz + n_rows
    return -(-L // (omega * sigma)), -(-L // sigma)


def plan(row_ptr, omega: int, sigma: int):
    """Sec. 4.1: TILE = (tile_x int32[T+1], tile_y uint32[T+1], lane_desc uint32[lanes])."""
    row_ptr = _i32a(row_ptr)
    n = len(row_ptr) - 1
    T, lanes = plan_sizes(n, int(row_ptr[-1]), omega, sigma)
    tile_x = np.empty(T + 1, np.int32)
    tile_y = np.empty(T + 1, np.uint32)
    lane_desc = np.empty(max(lanes, 1), np.uint32)
    rc = _load().or_plan(n, row_ptr, omega, sigma, tile_x, tile_y, lane_desc)
    if rc != 0:
        raise ValueError(f"descriptor does not fit: 2*{offset_bits(omega, sigma)}+{sigma} > 32")
    return tile_x, tile_y, lane_desc[:lanes]


def plan64(row_ptr, omega: int, sigma: int):
    """TILE with 64-bit lane descriptors (fit condition 2b + sigma <= 64):
    (tile_x int32[T+1], tile_y uint32[T+1], lane_desc uint64[lanes])."""
    row_ptr = _i32a(row_ptr)
    n = len(row_ptr) - 1
    T, lanes = plan_sizes(n, int(row_ptr[-1]), omega, sigma)
    tile_x = np.empty(T + 1, np.int32)
    tile_y = np.empty(T + 1, np.uint32)
    lane_desc = np.empty(max(lanes, 1), np.uint64)
    rc = _load().or_plan64(n, row_ptr, omega, sigma, tile_x, tile_y, lane_desc)
    if rc != 0:
        raise ValueError(f"descriptor does not fit: 2*{offset_bits(omega, sigma)}+{sigma} > 64")
    return tile_x, tile_y, lane_desc[:lanes]


def plan_replay64(row_ptr, col, values, x, tile, omega: int, sigma: int):
    """Decode + replay of a 64-bit-descriptor TILE; returns y."""
    tile_x, tile_y, lane_desc = tile
    row_ptr = _i32a(row_ptr)
    n = len(row_ptr) - 1
    m = int(row_ptr[-1])
    y = np.empty(max(n, 1), np.float64)
    rc = _load().or_plan_replay64(n, m, omega, sigma, _i32a(tile_x),
                                  np.ascontiguousarray(tile_y, np.uint32),
                                  np.ascontiguousarray(lane_desc if len(lane_desc) else [0],
                                                       np.uint64),
                                  _i32a(col) if m else np.zeros(1, np.int32),
                                  _f64a(values) if m else np.zeros(1),
                                  _f64a(x) if len(x) else np.zeros(1), y)
    if rc != 0:
        raise ValueError(f"plan replay failed ({rc})")
    return y[:n]


def unpack_desc(lane_desc, omega: int, sigma: int):
    """Sec. 4.1.1: split descriptors into (x_offset, y_offset, bit_flag)."""
    b = offset_bits(omega, sigma)
    d = np.asarray(lane_desc, np.uint64)
    mask = (1 << b) - 1
    return (d & mask).astype(np.int64), ((d >> b) & mask).astype(np.int64), (d >> (2 * b)).astype(
        np.int64)


def plan_replay(row_ptr, col, values, x, tile, omega: int, sigma: int):
    """Sec. 4.1.1 decode + replay of every lane; returns (y, row of each nnz)."""
    tile_x, tile_y, lane_desc = tile
    row_ptr = _i32a(row_ptr)
    n = len(row_ptr) - 1
    m = int(row_ptr[-1])
    y = np.empty(max(n, 1), np.float64)
    nnz_row = np.full(max(m, 1), -1, np.int32)
    rc = _load().or_plan_replay(n, m, omega, sigma, _i32a(tile_x),
                                np.ascontiguousarray(tile_y, np.uint32),
                                np.ascontiguousarray(lane_desc if len(lane_desc) else [0],
                                                     np.uint32),
                                _i32a(col) if m else np.zeros(1, np.int32),
                                _f64a(values) if m else np.zeros(1),
                                _f64a(x) if len(x) else np.zeros(1), y,
                                nnz_row.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ValueError(f"plan replay failed ({rc})")
    return y[:n], nnz_row[:m]


def tile_mem_bytes(n_rows: int, nnz: int, omega: int, sigma: int, r_f: float) -> float:
    """Sec. 4.3: mem_sigma = 8 (ceil((m+n)/(omega sigma)) + 1) + 4 ceil((m+n)/sigma) (1 - r_f)."""
    L = nnz + n_rows
    return 8 * (math.ceil(L / (omega * sigma)) + 1) + 4 * math.ceil(L / sigma) * (1 - r_f)


def smem_bytes(block_lanes: int, sigma: int, value_size: int) -> int:
    """Sec. 4.3: smem_sigma = (b + 1) sigma sizeof(value) per block."""
    return (block_lanes + 1) * sigma * value_size


# -------------------------------------------------------------- PageRank --

def pagerank(row_ptr, col, values, alpha: float, iters: int, x0, *, history: bool = False):
    """Sec. 5.5.1: power method, damping alpha, dangling mass spread
    uniformly.  Returns (x_iters, resid[iters], hist or None)."""
    row_ptr = _i32a(row_ptr)
    n = len(row_ptr) - 1
    x_out = np.empty(max(n, 1), np.float64)
    resid = np.empty(max(iters, 1), np.float64)
    hist = np.empty((max(iters, 1), max(n, 1)), np.float64) if history else None
    rc = _load().or_pagerank(n, row_ptr, _i32a(col) if len(col) else np.zeros(1, np.int32),
                             _f64a(values) if len(values) else np.zeros(1), float(alpha),
                             int(iters), _f64a(x0), x_out,
                             hist.ctypes.data_as(ctypes.c_void_p) if history else None,
                             resid.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise MemoryError("or_pagerank failed")
    return x_out[:n], resid[:iters], (hist[:iters, :n] if history else None)


# -------------------------------------------------------------- batched --

def spmm(row_ptr, col, values, X) -> np.ndarray:
    """Y = A X for X of shape (n_cols, k) (Sec. 3.1 per column), long-double sums."""
    row_ptr = _i32a(row_ptr)
    X = np.ascontiguousarray(X, np.float64)
    n = len(row_ptr) - 1
    k = X.shape[1]
    Y = np.empty((max(n, 1), max(k, 1)), np.float64)
    _load().or_spmm(n, row_ptr, _i32a(col) if len(col) else np.zeros(1, np.int32),
                    _f64a(values) if len(values) else np.zeros(1), k,
                    X.ravel() if X.size else np.zeros(1), Y.ravel())
    return Y[:n, :k]


def pagerank_teleport(row_ptr, col, values, alpha: float, iters: int, v, x0):
    """Power method x' = alpha P x + (alpha * dangling mass + 1 - alpha) v.
    Returns (x_iters, resid[iters])."""
    row_ptr = _i32a(row_ptr)
    n = len(row_ptr) - 1
    x_out = np.empty(max(n, 1), np.float64)
    resid = np.empty(max(iters, 1), np.float64)
    rc = _load().or_pagerank_teleport(n, row_ptr, _i32a(col) if len(col) else np.zeros(1, np.int32),
                                      _f64a(values) if len(values) else np.zeros(1), float(alpha),
                                      int(iters), _f64a(v), _f64a(x0), x_out,
                                      resid.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise MemoryError("or_pagerank_teleport failed")
    return x_out[:n], resid[:iters]


def personalized_pagerank(row_ptr, col, values, alpha: float, iters: int, sources):
    """Personalised PageRank for each source s (teleport and x_0 = e_s).
    Returns X of shape (n, len(sources))."""
    n = len(row_ptr) - 1
    out = np.empty((n, len(sources)), np.float64)
    for j, s in enumerate(sources):
        e = np.zeros(n)
        e[s] = 1.0
        out[:, j], _ = pagerank_teleport(row_ptr, col, values, alpha, iters, e, e)
    return out


def pagerank_multi(row_ptr, col, values, graph_ptr, alpha: float, iters: int, x0):
    """PageRank (Sec. 5.5.1) of every graph on the diagonal of a block-diagonal
    matrix: graph g owns rows and columns [graph_ptr[g], graph_ptr[g+1]).
    Each graph is solved on its own slice with its own n, dangling set and
    teleport."""
    row_ptr = np.asarray(row_ptr, np.int64)
    x = np.empty(len(row_ptr) - 1, np.float64)
    for g in range(len(graph_ptr) - 1):
        a, b = int(graph_ptr[g]), int(graph_ptr[g + 1])
        lo, hi = int(row_ptr[a]), int(row_ptr[b])
        sub_ptr = (row_ptr[a:b + 1] - lo).astype(np.int32)
        sub_col = np.asarray(col[lo:hi], np.int64) - a
        if len(sub_col) and (sub_col.min() < 0 or sub_col.max() >= b - a):
            raise ValueError(f"graph {g} has a column outside its block")
        x[a:b], _, _ = pagerank(sub_ptr, sub_col.astype(np.int32), values[lo:hi], alpha, iters,
                                x0[a:b])
    return x


# ------------------------------------------------- adjoint of PageRank --

def transpose(n_cols: int, row_ptr, col):
    """CSR of A^T: (rowT_ptr, colT, perm); row c of A^T lists the nonzeros of
    column c of A in increasing row order, perm[i] = their index in A."""
    row_ptr = _i32a(row_ptr)
    n = len(row_ptr) - 1
    m = int(row_ptr[-1])
    rowT = np.empty(n_cols + 1, np.int32)
    colT = np.empty(max(m, 1), np.int32)
    perm = np.empty(max(m, 1), np.int32)
    rc = _load().or_transpose(n, int(n_cols), row_ptr, _i32a(col) if m else np.zeros(1, np.int32),
                              rowT, colT, perm)
    if rc != 0:
        raise MemoryError("or_transpose failed")
    return rowT, colT[:m], perm[:m]


def pagerank_adjoint(row_ptr, col, values, alpha: float, iters: int, g):
    """lambda = g + M^T lambda for the Jacobian M = alpha P + (alpha/n) 1 d^T
    of the PageRank step (Sec. 5.5.1), by `iters` fixed-point steps from g."""
    row_ptr = _i32a(row_ptr)
    n = len(row_ptr) - 1
    lam = np.empty(max(n, 1), np.float64)
    rc = _load().or_pagerank_adjoint(n, row_ptr, _i32a(col) if len(col) else np.zeros(1, np.int32),
                                     _f64a(values) if len(values) else np.zeros(1), float(alpha),
                                     int(iters), _f64a(g), lam)
    if rc != 0:
        raise MemoryError("or_pagerank_adjoint failed")
    return lam[:n]


def row_index(row_ptr) -> np.ndarray:
    """Row of every nonzero."""
    row_ptr = np.asarray(row_ptr, np.int64)
    return np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))


def pagerank_value_grad(row_ptr, col, lam, x, alpha: float) -> np.ndarray:
    """dL/dP[e] = alpha lambda[row(e)] x*[col(e)] for every nonzero e = (v, u):
    the derivative of the fixed point through the term alpha P x."""
    return alpha * np.asarray(lam)[row_index(row_ptr)] * np.asarray(x)[np.asarray(col)]


def colnorm(col, w, n_cols: int):
    """P[e] = w[e] / s[col(e)], s[c] = sum of w over column c (column
    normalisation of positive edge weights).  Returns (P, s)."""
    col = np.asarray(col, np.int64)
    s = np.bincount(col, weights=np.asarray(w, np.float64), minlength=n_cols)
    return np.asarray(w) / s[col], s


def colnorm_backward(col, w, G, n_cols: int) -> np.ndarray:
    """dL/dw[e] = (G[e] - sum_{e' in col(e)} G[e'] P[e']) / s[col(e)] for
    G = dL/dP, from differentiating P[e'] = w[e'] / s[col(e')]."""
    col = np.asarray(col, np.int64)
    P, s = colnorm(col, w, n_cols)
    t = np.bincount(col, weights=np.asarray(G, np.float64) * P, minlength=n_cols)
    return (np.asarray(G) - t[col]) / s[col]


def pagerank_loss_grad(row_ptr, col, w, target, alpha: float, iters: int):
    """Loss ||x*(P(w)) - target||^2 of the PageRank of the column-normalised
    weights and its gradient with respect to w (adjoint method).  x_0 = 1/n;
    `iters` steps for both the forward and the adjoint fixed point.
    Returns (loss, dL/dw, x*, lambda)."""
    n = len(row_ptr) - 1
    P, _ = colnorm(col, w, n)
    x, _, _ = pagerank(row_ptr, col, P, alpha, iters, np.full(n, 1.0 / n))
    r = x - np.asarray(target)
    lam = pagerank_adjoint(row_ptr, col, P, alpha, iters, 2.0 * r)
    G = pagerank_value_grad(row_ptr, col, lam, x, alpha)
    return float(r @ r), colnorm_backward(col, w, G, n), x, lam


# -------------------------------------------------------------- BiCGSTAB --

BICGSTAB_STATUS = {0: "converged", 1: "iteration cap", 2: "breakdown"}


def bicgstab(row_ptr, col, values, b, x0, tol: float, max_iter: int):
    """Sec. 5.5.2: unpreconditioned BiCGSTAB for A x = b, stopping when the
    updated residual satisfies ||r|| / ||b|| < tol.  Returns
    (x, iterations, status, relative-residual history)."""
    row_ptr = _i32a(row_ptr)
    n = len(row_ptr) - 1
    x = np.empty(max(n, 1), np.float64)
    hist = np.zeros(max(max_iter, 1), np.float64)
    st = ctypes.c_int()
    it = _load().or_bicgstab(n, row_ptr, _i32a(col) if len(col) else np.zeros(1, np.int32),
                             _f64a(values) if len(values) else np.zeros(1), _f64a(b), _f64a(x0),
                             float(tol), int(max_iter), x, hist.ctypes.data_as(ctypes.c_void_p),
                             ctypes.byref(st))
    if it < 0:
        raise MemoryError("or_bicgstab failed")
    return x[:n], it, BICGSTAB_STATUS[st.value], hist[:it]
