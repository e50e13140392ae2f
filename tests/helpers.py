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
