"""Shared helpers for the GPU parity tests (inputs to device, tolerances)."""
import numpy as np
import torch

import graphgen
import oracle

# Parity bars: |y_gpu - y_ref| <= tol * (|A| |x|)[r] per row; rows whose scale
# is 0 must be exactly 0.
SPMV_TOL = {torch.float32: 1e-5, torch.float64: 1e-12}
# PageRank iterate-by-iterate, per-entry relative error
PR_TOL = {torch.float32: 1e-4, torch.float64: 1e-11}
OMEGA = 64
_WORKLOADS = {}


def workload(name):
    """graphgen.workload(name), generated once per test session."""
    if name not in _WORKLOADS:
        _WORKLOADS.clear()  # keep at most one large input alive
        _WORKLOADS[name] = graphgen.workload(name)
    return _WORKLOADS[name]


def require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a GPU")
    return torch.device("cuda:0")


def to_device(row_ptr, col, values, dtype, dev):
    rp = torch.from_numpy(np.ascontiguousarray(row_ptr, np.int32)).to(dev)
    ci = torch.from_numpy(np.ascontiguousarray(col, np.int32)).to(dev)
    va = torch.from_numpy(np.ascontiguousarray(values, np.float64)).to(dtype).to(dev)
    return rp, ci, va


def host_values(values, dtype):
    """The values exactly as the GPU sees them, promoted back to float64."""
    return np.asarray(values, np.float64).astype(
        np.float32 if dtype == torch.float32 else np.float64).astype(np.float64)


def check_spmv(y_gpu, row_ptr, col, vals64, x64, dtype, label=""):
    """Compare a GPU SpMV result (tensor) with the oracle; returns max rel err."""
    y = y_gpu.double().cpu().numpy()
    ref = oracle.spmv(row_ptr, col, vals64, x64)
    scale = oracle.abs_spmv(row_ptr, col, vals64, x64)
    assert not np.isnan(y).any(), f"{label}: NaN in output"
    zero = scale == 0
    assert np.all(y[zero] == 0.0), f"{label}: nonzero output on a row with |A||x| = 0"
    err = np.abs(y - ref)
    rel = np.where(zero, 0.0, err / np.where(zero, 1.0, scale))
    worst = float(rel.max()) if len(rel) else 0.0
    assert worst <= SPMV_TOL[dtype], f"{label}: max rel err {worst:.3e} row {int(rel.argmax())}"
    return worst


def seeded_x(n, seed, dtype):
    x = graphgen.uniform(seed, 77, n, -1.0, 1.0)
    return x.astype(np.float32 if dtype == torch.float32 else np.float64).astype(np.float64)


def spmv_cases():
    """Named row_ptr patterns (with their column counts) for the parity tests:
    degenerate shapes, long rows, random and fuzzed sizes, a Chung-Lu graph."""
    cases = {}
    cases["one_row"] = (np.array([0, 1], np.int32), 3)
    cases["all_rows_empty"] = (np.zeros(301, np.int32), 4)
    cases["single_long_row"] = (np.array([0, 20000], np.int32), 20000)
    cases["long_then_empty"] = (np.array([0, 2000, 2000, 2000, 2001, 4500] + [4500] * 700,
                                         np.int32), 3000)
    for seed, (n, nc, dens, emp) in enumerate([(50, 40, 0.3, 0.2), (700, 300, 0.02, 0.5),
                                               (1200, 800, 0.02, 0.1), (333, 64, 0.02, 0.0),
                                               (200, 3000, 0.01, 0.3), (3000, 50, 0.05, 0.2)]):
        rp, _, _ = graphgen.random_csr(n, nc, dens, seed, empty_frac=emp, long_rows=(n // 3,))
        cases[f"random{seed}_{n}x{nc}"] = (rp, nc)
    cases["one_column"] = (np.arange(1001, dtype=np.int32), 1)
    rp, _ = graphgen.chung_lu_pattern(10_000, 100_000, 2.1, 0.1, seed=1)
    cases["chung_lu_10k"] = (rp, 10_000)
    # fuzz: random sizes, densities, empty fractions
    rng = np.random.default_rng(2024)
    for f in range(6):
        n = int(rng.integers(1, 4000))
        nc = int(rng.integers(1, 4000))
        dens = float(rng.uniform(0.0005, 0.02))
        rp, _, _ = graphgen.random_csr(n, nc, dens, 100 + f, empty_frac=float(rng.uniform(0, .7)))
        cases[f"fuzz{f}_{n}x{nc}"] = (rp, nc)
    return cases


def case_matrix(cases, name, seed=0):
    """Seeded columns and values in [-1, 1) on the named pattern."""
    rp, nc = cases[name]
    m = int(rp[-1])
    rng = np.random.default_rng(seed)
    col = rng.integers(0, nc, m).astype(np.int32)
    # columns need not be sorted within a row
    vals = rng.uniform(-1, 1, m)
    return rp, col, vals, nc


def stacked_row_ptr(row_ptr, col, n_cols, stripes):
    """Row pointer of the stacked matrix, written from its definition: the
    stripe of column c is c >> max(0, ceil(log2 n_cols) - log2 S); the
    nonzeros are ordered by (stripe, row, position in the row) and every
    distinct (stripe, row) pair is a row."""
    n = len(row_ptr) - 1
    m = int(row_ptr[-1])
    cbits = int(np.ceil(np.log2(n_cols))) if n_cols > 1 else 0
    shift = max(0, cbits - int(np.log2(stripes)))
    stripe = np.asarray(col, np.int64) >> shift
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    order = np.lexsort((np.arange(m), rows, stripe))
    key = stripe[order] * (n + 1) + rows[order]
    starts = np.flatnonzero(np.r_[True, key[1:] != key[:-1]]) if m else np.zeros(0, np.int64)
    return np.r_[starts, m].astype(np.int32), order
