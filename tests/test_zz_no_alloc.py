"""merbit_pagerank_noalloc (the PageRank entry point that allocates nothing)
against merbit_pagerank on the same plans and inputs, called through the C
ABI: two calls in a row, the second on a smaller input, in FP32 and FP64, on
plain and column-stripe plans, before and after the plan has a dangling mask
of its own; plus the size limit of its work array."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from helpers import PR_TOL, host_values, require_gpu, to_device, workload

pytestmark = pytest.mark.gpu
ALPHA = 0.85


def _plan(w, dtype, dev, **kw):
    import paper_2605_07391_amd as pkg
    r, c, v = to_device(w["row_ptr"], w["col"], w["values"], dtype, dev)
    return pkg.Plan(r, c, v, w["n_cols"], **kw), (r, c, v)


def _x0(n, dtype, dev):
    return torch.full((n,), 1.0 / n, dtype=dtype, device=dev)


def _compare(got, ref, dtype, label):
    g = got.double().cpu().numpy()
    r = ref.double().cpu().numpy()
    rel = np.abs(g - r) / np.abs(r)
    assert rel.max() <= PR_TOL[dtype], f"{label}: max rel diff {rel.max():.3e}"
    assert abs(g.sum() - 1.0) <= (1e-5 if dtype == torch.float32 else 1e-12), label


def _run_pair(plan, n, dtype, dev, iters, tol=0.0, check_every=10, label=""):
    """noalloc then the plan-owned driver from the same x0; both must agree."""
    xa = _x0(n, dtype, dev)
    ia, ra, ca = plan.pagerank_noalloc(xa, ALPHA, tol=tol, max_iter=iters,
                                       check_every=check_every)
    xb = _x0(n, dtype, dev)
    ib, rb, cb = plan.pagerank(xb, ALPHA, tol=tol, max_iter=iters, check_every=check_every)
    assert (ia, ca) == (ib, cb), f"{label}: iterations {ia} / {ib}, converged {ca} / {cb}"
    # the residual is the l1 change of the last step, so by the triangle
    # inequality two runs' residuals differ by at most the l1 differences of
    # their last two iterates: rows that span tiles are finished with float
    # atomics, whose order varies, and in FP32 near convergence the residual
    # is of the size of those rounding differences
    slack = 4.0 * float((xa.double() - xb.double()).abs().sum())
    assert abs(ra - rb) <= 1e-3 * rb + slack + 1e-12, f"{label}: residual {ra} / {rb}"
    _compare(xa, xb, dtype, label)
    return xa


@pytest.mark.parametrize("stripes", [0, 8], ids=["plain", "striped8"])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_noalloc_matches_pagerank_two_calls_second_smaller(dtype, stripes):
    dev = require_gpu()
    big = workload("rmat18")
    plan_big, keep_big = _plan(big, dtype, dev, stripes=stripes)
    n_big = big["n_rows"]
    print(f"noalloc: rmat18 {dtype} stripes={stripes}", flush=True)
    # first call builds its own dangling mask in the work array
    x_big = _run_pair(plan_big, n_big, dtype, dev, 25, label="rmat18 first")
    # the plan now has its own mask (from pagerank): the second form
    _run_pair(plan_big, n_big, dtype, dev, 13, label="rmat18 plan mask")
    w = workload("chung_lu_10k")
    plan_small, keep_small = _plan(w, dtype, dev, stripes=stripes)
    n = w["n_rows"]
    # second call, smaller input, right after the larger one on the same array
    x_small = _run_pair(plan_small, n, dtype, dev, 20, label="chung_lu_10k after rmat18")
    # and against the oracle, iterate 20
    x0 = np.full(n, 1.0 / n).astype(np.float32 if dtype == torch.float32 else np.float64)
    ref, _, _ = oracle.pagerank(w["row_ptr"], w["col"], host_values(w["values"], dtype), ALPHA,
                                20, x0.astype(np.float64))
    got = x_small.double().cpu().numpy()
    assert (np.abs(got - ref) / ref).max() <= PR_TOL[dtype]
    assert torch.isfinite(x_big).all()
    plan_small.close()
    plan_big.close()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_noalloc_convergence_status(dtype):
    dev = require_gpu()
    w = workload("chung_lu_10k")
    plan, keep = _plan(w, dtype, dev)
    n = w["n_rows"]
    tol = 1e-6 if dtype == torch.float32 else 1e-13
    _run_pair(plan, n, dtype, dev, 500, tol=tol, check_every=5, label="converged")
    x = _x0(n, dtype, dev)
    it, res, conv = plan.pagerank_noalloc(x, ALPHA, tol=1e-30, max_iter=3, check_every=1)
    assert it == 3 and not conv
    plan.close()


def test_noalloc_rejects_a_plan_beyond_its_array():
    import paper_2605_07391_amd.merbit as mb
    dev = require_gpu()
    # FP64, n = 3,000,000: 3 n 8 bytes = 72 MB > 64 MiB
    n = 3_000_000
    r = torch.arange(n + 1, dtype=torch.int32, device=dev)
    c = torch.arange(n, dtype=torch.int32, device=dev)
    v = torch.ones(n, dtype=torch.float64, device=dev)
    plan = mb.Plan(r, c, v, n)
    x = _x0(n, torch.float64, dev)
    it = ctypes.c_int(-1)
    res = ctypes.c_double(-1.0)
    rc = mb.load().merbit_pagerank_noalloc(plan._handle(), 0.85, 0.0, 5, 10,
                                           ctypes.c_void_p(x.data_ptr()), ctypes.byref(it),
                                           ctypes.byref(res), None)
    assert rc == mb.EINVAL
    assert b"work space" in mb.load().merbit_last_error()
    assert it.value == 0
    # rejected before any launch: x is untouched
    assert torch.equal(x, _x0(n, torch.float64, dev))
    plan.close()
