"""Seeded synthetic inputs shared by the CPU oracle tests and the HIP library.

This module draws sparse matrices and vectors; it contains none of the
method's arithmetic (no SpMV, no merge path, no PageRank step).  The C source
next to it (``graphgen.c``) documents the counter-based random streams.

Workloads (all int32 CSR, rows = destinations, duplicates merged):

* ``chung_lu_10k`` -- directed Chung-Lu graph, 10,000 vertices, 100,000 edge
  draws, source weights with power-law exponent 2.1, 10 % of vertices with
  target weight 0 (their rows are empty).  Column-stochastic PageRank matrix,
  values 1/outdeg.  Graph seed 1.
* ``rmat<s>`` -- R-MAT with 2^s vertices, 16 * 2^s edge draws,
  (a, b, c) = (0.57, 0.19, 0.19), no noise, no relabelling.  PageRank matrix,
  values 1/outdeg.  Scale 22 uses graph seed 22.
* ``chung_lu_multi256`` -- 256 independent Chung-Lu graphs on the diagonal of
  one matrix (rows and columns of graph g are [graph_ptr[g], graph_ptr[g+1])).
  Vertex counts log-uniform in [1,000, 200,000] (seed 40, stream 22), 8 edge
  draws per vertex, exponent 2.1, 10 % empty rows; graph g uses seed 1000 + g.
  Values 1/outdeg.  The key ``graph_ptr`` holds the offsets.
* ``rmat<s>_sym`` -- the R-MAT pattern above made undirected (A + A^T,
  duplicates merged, self-loops kept) with every value 1: the symmetric 0/1
  systems of the BiCGSTAB workload.  x_true uniform in [-1, 1) (seed s,
  stream 85); b = A x_true is formed on the device by the caller.
* ``stress24`` -- R-MAT scale 24 as above (seed 24), 30 % of rows cleared,
  8 rows replaced by 2,000,000 uniformly chosen distinct columns.  Values
  uniform in (0, 1] (seed 24, stream 20), x uniform in [-1, 1) (seed 25,
  stream 21).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None

STREAM_VALUES = 20
STREAM_X = 21


def build() -> str:
    """Compile the generator library with gcc (OpenMP) next to its source."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                    "-Wall", "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    lib.gg_rmat.restype = ctypes.c_int64
    lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_uint64, i32p, i32p]
    lib.gg_stress.restype = ctypes.c_int64
    lib.gg_stress.argtypes = [ctypes.c_int64, ctypes.c_int64, i32p, i32p, ctypes.c_uint64,
                              ctypes.c_double, ctypes.c_int, ctypes.c_int64, i32p, i32p, i32p]
    lib.gg_chung_lu.restype = ctypes.c_int64
    lib.gg_chung_lu.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_uint64, i32p, i32p]
    lib.gg_uniform.restype = None
    lib.gg_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int, f64p]
    lib.gg_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def num_threads() -> int:
    return int(_load().gg_num_threads())


def rmat_pattern(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
                 c: float = 0.19, seed: int = 22):
    """R-MAT pattern (row_ptr, col) with 2^scale rows; rows = destinations."""
    lib = _load()
    n = 1 << scale
    nedges = edge_factor * n
    row_ptr = np.empty(n + 1, np.int32)
    col = np.empty(max(nedges, 1), np.int32)
    nnz = lib.gg_rmat(scale, nedges, a, b, c, seed, row_ptr, col)
    if nnz < 0:
        raise MemoryError("gg_rmat: allocation failed")
    return row_ptr, np.ascontiguousarray(col[:nnz])


def chung_lu_pattern(n: int, nedges: int, gamma_out: float = 2.1, empty_frac: float = 0.1,
                     seed: int = 1):
    """Directed Chung-Lu pattern (row_ptr, col); rows = destinations."""
    lib = _load()
    row_ptr = np.empty(n + 1, np.int32)
    col = np.empty(max(nedges, 1), np.int32)
    nnz = lib.gg_chung_lu(n, nedges, gamma_out, empty_frac, seed, row_ptr, col)
    if nnz < 0:
        raise MemoryError("gg_chung_lu: allocation failed")
    return row_ptr, np.ascontiguousarray(col[:nnz])


def stress_pattern(row_ptr, col, n_cols: int, seed: int = 24, empty_frac: float = 0.3,
                   n_hubs: int = 8, hub_nnz: int = 2_000_000):
    """Clear a seeded fraction of rows and inject hub rows (see graphgen.c)."""
    lib = _load()
    n = len(row_ptr) - 1
    out_ptr = np.empty(n + 1, np.int32)
    out_col = np.empty(len(col) + n_hubs * hub_nnz + 1, np.int32)
    hubs = np.full(max(n_hubs, 1), -1, np.int32)
    nnz = lib.gg_stress(n, n_cols, np.ascontiguousarray(row_ptr, np.int32),
                        np.ascontiguousarray(col, np.int32), seed, empty_frac, n_hubs, hub_nnz,
                        out_ptr, out_col, hubs)
    if nnz < 0:
        raise MemoryError("gg_stress: allocation failed")
    return out_ptr, np.ascontiguousarray(out_col[:nnz]), hubs[:n_hubs]


def uniform(seed: int, stream: int, count: int, lo: float, hi: float,
            closed_high: bool = False) -> np.ndarray:
    """Counter-based uniform doubles in [lo, hi) or, with closed_high, (lo, hi]."""
    out = np.empty(max(count, 1), np.float64)
    _load().gg_uniform(seed, stream, count, lo, hi, 1 if closed_high else 0, out)
    return out[:count]


def column_stochastic_values(col: np.ndarray, n_cols: int) -> np.ndarray:
    """Values 1/outdeg(u) for every nonzero (v, u): outdeg counts the merged
    nonzeros in column u (self-loops kept)."""
    outdeg = np.bincount(col, minlength=n_cols).astype(np.float64)
    with np.errstate(divide="ignore"):
        inv = np.where(outdeg > 0, 1.0 / np.maximum(outdeg, 1.0), 0.0)
    return inv[col]


class Workload(dict):
    """A named input: keys row_ptr, col, values (float64), n_rows, n_cols,
    nnz, x (float64 or None) and meta (seeds and recipe)."""


def ppr_sources(n: int, k: int = 64, seed: int = 4) -> np.ndarray:
    """k distinct personalised-PageRank source vertices, uniform in [0, n), sorted."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32)


STREAM_SIZES = 22


def multi_graph_sizes(n_graphs: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Vertex counts log-uniform in [lo, hi]."""
    u = uniform(seed, STREAM_SIZES, n_graphs, np.log(lo), np.log(hi + 1.0))
    return np.clip(np.floor(np.exp(u)), lo, hi).astype(np.int64)


def chung_lu_multi(n_graphs: int = 256, lo: int = 1000, hi: int = 200_000, degree: int = 8,
                   seed: int = 40, graph_seed0: int = 1000):
    """Block-diagonal CSR of independent Chung-Lu graphs.  Returns
    (row_ptr, col, graph_ptr); graph g's rows and columns are
    [graph_ptr[g], graph_ptr[g+1])."""
    sizes = multi_graph_sizes(n_graphs, lo, hi, seed)
    graph_ptr = np.zeros(n_graphs + 1, np.int64)
    np.cumsum(sizes, out=graph_ptr[1:])
    parts_ptr, parts_col = [np.zeros(1, np.int64)], []
    nnz = 0
    for g, n in enumerate(sizes):
        rp, cl = chung_lu_pattern(int(n), degree * int(n), 2.1, 0.1, seed=graph_seed0 + g)
        parts_ptr.append(rp[1:].astype(np.int64) + nnz)
        parts_col.append(cl.astype(np.int32) + np.int32(graph_ptr[g]))
        nnz += int(rp[-1])
    row_ptr = np.concatenate(parts_ptr)
    if row_ptr[-1] >= 2**31:
        raise ValueError("too many nonzeros for int32 row_ptr")
    return row_ptr.astype(np.int32), np.concatenate(parts_col), graph_ptr


STREAM_XTRUE = 85


def symmetrize_pattern(row_ptr, col, n: int):
    """Pattern of A + A^T (duplicates merged, columns sorted within rows)."""
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(np.asarray(row_ptr, np.int64)))
    c = np.asarray(col, np.int64)
    keys = np.unique(np.concatenate([rows * n + c, c * n + rows]))
    r2 = keys // n
    out_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(r2, minlength=n), out=out_ptr[1:])
    if out_ptr[-1] >= 2**31:
        raise ValueError("too many nonzeros for int32 row_ptr")
    return out_ptr.astype(np.int32), (keys % n).astype(np.int32)


def workload(name: str) -> Workload:
    """Build one of the named synthetic workloads (see module docstring)."""
    if name.startswith("rmat") and name.endswith("_sym"):
        scale = int(name[4:-4])
        rp, cl = rmat_pattern(scale, 16, 0.57, 0.19, 0.19, seed=scale)
        n = 1 << scale
        row_ptr, col = symmetrize_pattern(rp, cl, n)
        del rp, cl
        meta = {"generator": "rmat_sym", "scale": scale, "edge_factor": 16,
                "abc": [0.57, 0.19, 0.19], "seed": scale, "x_true_seed": scale,
                "x_true_stream": STREAM_XTRUE}
        return Workload(row_ptr=row_ptr, col=col, values=np.ones(len(col)), n_rows=n, n_cols=n,
                        nnz=len(col), x=uniform(scale, STREAM_XTRUE, n, -1.0, 1.0), meta=meta)
    if name.startswith("chung_lu_multi"):
        count = int(name[len("chung_lu_multi"):] or 256)
        row_ptr, col, graph_ptr = chung_lu_multi(count)
        n = int(graph_ptr[-1])
        vals = column_stochastic_values(col, n)
        meta = {"generator": "chung_lu_multi", "graphs": count, "size_range": [1000, 200_000],
                "degree": 8, "gamma_out": 2.1, "empty_frac": 0.1, "seed": 40,
                "graph_seed0": 1000}
        return Workload(row_ptr=row_ptr, col=col, values=vals, n_rows=n, n_cols=n,
                        nnz=len(col), x=None, meta=meta, graph_ptr=graph_ptr)
    if name == "chung_lu_10k":
        row_ptr, col = chung_lu_pattern(10_000, 100_000, 2.1, 0.1, seed=1)
        n = 10_000
        vals = column_stochastic_values(col, n)
        meta = {"generator": "chung_lu", "n": n, "edge_draws": 100_000, "gamma_out": 2.1,
                "empty_frac": 0.1, "seed": 1}
        return Workload(row_ptr=row_ptr, col=col, values=vals, n_rows=n, n_cols=n,
                        nnz=len(col), x=None, meta=meta)
    if name.startswith("rmat"):
        scale = int(name[4:])
        seed = {22: 22, 20: 20}.get(scale, scale)
        row_ptr, col = rmat_pattern(scale, 16, 0.57, 0.19, 0.19, seed=seed)
        n = 1 << scale
        vals = column_stochastic_values(col, n)
        meta = {"generator": "rmat", "scale": scale, "edge_factor": 16,
                "abc": [0.57, 0.19, 0.19], "seed": seed}
        return Workload(row_ptr=row_ptr, col=col, values=vals, n_rows=n, n_cols=n,
                        nnz=len(col), x=None, meta=meta)
    if name.startswith("stress"):
        scale = int(name[6:]) if len(name) > 6 else 24
        hub_nnz = 2_000_000 if scale >= 24 else max(1, (1 << scale) // 8)
        n = 1 << scale
        rp, cl = rmat_pattern(scale, 16, 0.57, 0.19, 0.19, seed=scale)
        row_ptr, col, hubs = stress_pattern(rp, cl, n, seed=scale, empty_frac=0.3,
                                            n_hubs=8, hub_nnz=hub_nnz)
        del rp, cl
        vals = uniform(scale, STREAM_VALUES, len(col), 0.0, 1.0, closed_high=True)
        x = uniform(scale + 1, STREAM_X, n, -1.0, 1.0)
        meta = {"generator": "stress", "scale": scale, "empty_frac": 0.3, "hubs": 8,
                "hub_nnz": hub_nnz, "seed": scale, "x_seed": scale + 1,
                "hub_rows": [int(h) for h in hubs]}
        return Workload(row_ptr=row_ptr, col=col, values=vals, n_rows=n, n_cols=n,
                        nnz=len(col), x=x, meta=meta)
    raise KeyError(name)


def random_csr(n_rows: int, n_cols: int, density: float, seed: int, *,
               empty_frac: float = 0.0, long_rows=()):
    """Small irregular CSR for tests: Bernoulli(density) pattern, a seeded
    fraction of forced-empty rows, and optional dense rows (long_rows).
    Values uniform in [-1, 1).  Returns (row_ptr, col, values)."""
    rng = np.random.default_rng(seed)
    mask = rng.random((n_rows, n_cols)) < density
    if empty_frac > 0:
        mask[rng.random(n_rows) < empty_frac, :] = False
    for r in long_rows:
        mask[r, :] = True
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n_rows + 1, np.int32)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.nonzero(mask)[1].astype(np.int32)
    vals = rng.uniform(-1.0, 1.0, len(col))
    return row_ptr, col, vals


def csr_from_lengths(lengths, n_cols: int, seed: int):
    """CSR with the given row lengths (each <= n_cols), distinct sorted
    columns per row and values uniform in [-1, 1).  Returns
    (row_ptr, col, values)."""
    rng = np.random.default_rng(seed)
    lengths = np.asarray(lengths, np.int64)
    row_ptr = np.zeros(len(lengths) + 1, np.int64)
    np.cumsum(lengths, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), np.int32)
    for r, L in enumerate(lengths):
        if L == 0:
            continue
        if L == n_cols:
            cols = np.arange(n_cols)
        else:
            cols = np.sort(rng.choice(n_cols, size=int(L), replace=False))
        col[row_ptr[r]:row_ptr[r + 1]] = cols
    vals = rng.uniform(-1.0, 1.0, len(col))
    return row_ptr.astype(np.int32), col, vals
