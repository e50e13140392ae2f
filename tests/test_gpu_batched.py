"""GPU parity of the batched forms through the C ABI: Y = A X for many
right-hand sides, personalised PageRank for many sources at once, and
PageRank of many graphs on the diagonal of one matrix, against the oracle."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from helpers import (PR_TOL, SPMV_TOL, case_matrix, host_values, require_gpu, spmv_cases,
                     to_device, workload)

pytestmark = pytest.mark.gpu

DTYPES = [torch.float32, torch.float64]
CASES = spmv_cases()
ALPHA = 0.85


def _np_dtype(dtype):
    return np.float32 if dtype == torch.float32 else np.float64


def seeded_X(n, k, seed, dtype):
    X = graphgen.uniform(seed, 78, n * k, -1.0, 1.0).reshape(n, k)
    return X.astype(_np_dtype(dtype)).astype(np.float64)


def check_spmm(Y_gpu, row_ptr, col, vals64, X64, dtype, label=""):
    """|Y - A X| <= tol (|A| |X|) entry by entry; entries with scale 0 exactly 0."""
    Y = Y_gpu.double().cpu().numpy()
    ref = oracle.spmm(row_ptr, col, vals64, X64)
    scale = oracle.spmm(row_ptr, col, np.abs(vals64), np.abs(X64))
    assert not np.isnan(Y).any(), f"{label}: NaN in output"
    zero = scale == 0
    assert np.all(Y[zero] == 0.0), f"{label}: nonzero entry where |A||X| = 0"
    rel = np.where(zero, 0.0, np.abs(Y - ref) / np.where(zero, 1.0, scale))
    worst = float(rel.max()) if rel.size else 0.0
    assert worst <= SPMV_TOL[dtype], f"{label}: max rel err {worst:.3e}"
    return worst


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("k", [1, 13, 33, 64])
@pytest.mark.parametrize("sigma", [3, 12])
@pytest.mark.parametrize("name", list(CASES))
def test_spmm_parity(name, sigma, k, dtype):
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, vals, nc = case_matrix(CASES, name, seed=k)
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, nc, sigma=sigma)
    X64 = seeded_X(nc, k, sigma + k, dtype)
    X = torch.from_numpy(X64).to(dtype).to(dev)
    Y = torch.full((len(rp) - 1, k), float("nan"), dtype=dtype, device=dev)
    plan.spmm(X, out=Y)
    torch.cuda.synchronize()
    check_spmm(Y, rp, col, host_values(vals, dtype), X64, dtype, f"{name} s{sigma} k{k}")
    plan.close()


@pytest.mark.parametrize("k", [64, 13])
@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_spmm_x_beyond_2gib(dtype, k):
    """X of more than 2 GiB (the kernel's 64-bit row-address path instead of
    the buffer path): 2^23 + 5 (FP32) or 2^22 + 5 (FP64) rows of 64 values,
    1,000 rows of A with columns spread over all of X, the last rows
    included.  Checked against the oracle on the X rows A uses."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    n_cols = (1 << 23) + 5 if dtype == torch.float32 else (1 << 22) + 5
    ldx = 64
    assert n_cols * ldx * (4 if dtype == torch.float32 else 8) >= 1 << 31
    rng = np.random.default_rng(31)
    lens = rng.integers(0, 120, 1000)
    lens[::97] = 0
    rp = np.r_[0, np.cumsum(lens)].astype(np.int32)
    m = int(rp[-1])
    col = rng.integers(0, n_cols, m).astype(np.int32)
    col[:20] = n_cols - 1 - np.arange(20)          # the last rows of X
    vals = rng.uniform(-1, 1, m)
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, n_cols, sigma=7)
    X = torch.empty((n_cols, ldx), dtype=dtype, device=dev)
    X.uniform_(-1.0, 1.0, generator=torch.Generator(device=dev).manual_seed(5))
    Y = torch.full((len(rp) - 1, k), float("nan"), dtype=dtype, device=dev)
    plan.spmm(X[:, :k], out=Y)
    torch.cuda.synchronize()
    used, remap = np.unique(col, return_inverse=True)
    X_used = X[torch.from_numpy(used.astype(np.int64)).to(dev), :k].double().cpu().numpy()
    del X
    check_spmm(Y, rp, remap.astype(np.int32), host_values(vals, dtype), X_used, dtype,
               f"X > 2 GiB k{k}")
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_spmm_strided_and_many_slabs(dtype):
    """k = 150 runs as four slabs of 32 columns and one of 22; X and Y are
    column windows of wider row-major buffers (leading dimensions > k)."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, vals, nc = case_matrix(CASES, "chung_lu_10k", seed=3)
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, nc)
    k = 150
    X64 = seeded_X(nc, k, 9, dtype)
    Xbuf = torch.full((nc, 170), float("nan"), dtype=dtype, device=dev)
    Xbuf[:, 7:7 + k] = torch.from_numpy(X64).to(dtype).to(dev)
    Ybuf = torch.full((len(rp) - 1, 201), float("nan"), dtype=dtype, device=dev)
    Y = Ybuf[:, 40:40 + k]
    plan.spmm(Xbuf[:, 7:7 + k], out=Y)
    torch.cuda.synchronize()
    check_spmm(Y, rp, col, host_values(vals, dtype), X64, dtype, "strided")
    # the columns outside the window are untouched
    assert torch.isnan(Ybuf[:, :40]).all() and torch.isnan(Ybuf[:, 40 + k:]).all()
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_spmm_columns_equal_single_vector(dtype):
    """Each column of the SpMM equals the single-vector SpMV on the same plan
    within the SpMV tolerance."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, vals, nc = case_matrix(CASES, "random2_1200x800", seed=4)
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, nc)
    k = 64
    X64 = seeded_X(nc, k, 10, dtype)
    X = torch.from_numpy(X64).to(dtype).to(dev)
    Y = plan.spmm(X)
    scale = oracle.spmm(rp, col, np.abs(host_values(vals, dtype)), np.abs(X64))
    for j in (0, 1, 31, 63):
        y = plan.spmv(X[:, j].contiguous())
        torch.cuda.synchronize()
        d = (Y[:, j].double() - y.double()).abs().cpu().numpy()
        assert np.all(d <= 2 * SPMV_TOL[dtype] * scale[:, j])
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_spmm_dual_chain(dtype):
    """Alternating outputs: Y zero at the boundary rows on entry, Z left zero."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, vals, nc = case_matrix(CASES, "long_then_empty", seed=6)
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, nc, sigma=5)
    n, k = len(rp) - 1, 33
    bufs = [torch.full((n, k), float("nan"), dtype=dtype, device=dev) for _ in range(2)]
    plan.spmm_zero_boundary(bufs[0])
    for it in range(4):
        X64 = seeded_X(nc, k, 20 + it, dtype)
        X = torch.from_numpy(X64).to(dtype).to(dev)
        plan.spmm_dual(X, bufs[it % 2], bufs[(it + 1) % 2])
        torch.cuda.synchronize()
        check_spmm(bufs[it % 2], rp, col, host_values(vals, dtype), X64, dtype, f"iter {it}")
    plan.close()


def test_spmm_argument_errors():
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, vals, nc = case_matrix(CASES, "random0_50x40", seed=1)
    r, c, v = to_device(rp, col, vals, torch.float32, dev)
    plan = pkg.Plan(r, c, v, nc)
    X = torch.zeros(nc, 4, device=dev)
    with pytest.raises(ValueError):
        plan.spmm(torch.zeros(nc + 1, 4, device=dev))
    with pytest.raises(TypeError):
        plan.spmm(X.double())
    with pytest.raises(ValueError):
        plan.spmm(X, out=torch.zeros(len(rp) - 1, 5, device=dev))
    Yb = torch.zeros(len(rp) - 1, 4, device=dev)
    with pytest.raises(pkg.MerbitError):  # Y and Z alias
        plan.spmm_dual(X, Yb, Yb)
    plan.close()


# ------------------------------------------------------ personalised PageRank


def _ppr_check(X_gpu, ref, dtype, label):
    """Per entry relative error (all terms are nonnegative, so no
    cancellation); in FP32 entries below 1e-30 are compared absolutely."""
    X = X_gpu.double().cpu().numpy()
    assert not np.isnan(X).any(), label
    assert np.all((X == 0) == (ref == 0)) or dtype == torch.float32, f"{label}: zero pattern"
    floor = 1e-30 if dtype == torch.float32 else 0.0
    big = ref > floor
    rel = np.abs(X[big] - ref[big]) / ref[big]
    worst = float(rel.max()) if rel.size else 0.0
    assert worst <= PR_TOL[dtype], f"{label}: max rel err {worst:.3e}"
    if floor:
        assert np.all(np.abs(X[~big] - ref[~big]) <= 1e-34), f"{label}: tiny entries"
    return worst


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("k", [1, 17, 40, 64])
def test_personalized_pagerank_chung_lu(k, dtype):
    """k sources on the Chung-Lu 10K graph, 20 iterations from x_0 = e_s:
    every column against the oracle entry by entry, and mass 1 per column."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    w = workload("chung_lu_10k")
    rp, col, vals, n = w["row_ptr"], w["col"], w["values"], w["n_rows"]
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, n)
    src = graphgen.ppr_sources(n, k, seed=4)
    X, iters, resid, _ = plan.pagerank_personalized(src, alpha=ALPHA, max_iter=20)
    torch.cuda.synchronize()
    assert iters == 20 and resid.shape == (k,)
    ref = oracle.personalized_pagerank(rp, col, host_values(vals, dtype), ALPHA, 20, src)
    _ppr_check(X, ref, dtype, f"k={k}")
    mass = X.double().sum(0).cpu().numpy()
    assert np.all(np.abs(mass - 1.0) <= (1e-5 if dtype == torch.float32 else 1e-12))
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("k", [8, 45])
def test_personalized_pagerank_convergence_and_reuse(k, dtype):
    """tol stops the iteration; a second call on the same plan (buffers kept)
    continues from the returned vectors and agrees with one long run (k = 45:
    the iterates are converted to and from two column slabs on every call)."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    w = workload("chung_lu_10k")
    rp, col, vals, n = w["row_ptr"], w["col"], w["values"], w["n_rows"]
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, n)
    src = graphgen.ppr_sources(n, k, seed=5)
    tol = 1e-5 if dtype == torch.float32 else 1e-10
    X, iters, resid, conv = plan.pagerank_personalized(src, tol=tol, max_iter=500,
                                                       check_every=5)
    assert conv and iters < 500 and iters % 5 == 0 and np.all(resid < tol)
    X1, _, _, _ = plan.pagerank_personalized(src, max_iter=7)
    X1, _, _, _ = plan.pagerank_personalized(src, X=X1, max_iter=6)
    X2, _, _, _ = plan.pagerank_personalized(src, max_iter=13)
    torch.cuda.synchronize()
    ref = oracle.personalized_pagerank(rp, col, host_values(vals, dtype), ALPHA, 13, src)
    _ppr_check(X1, ref, dtype, "7+6")
    _ppr_check(X2, ref, dtype, "13")
    with pytest.raises(pkg.MerbitError):
        plan.pagerank_personalized([n], max_iter=1)
    with pytest.raises(pkg.MerbitError):
        plan.pagerank_personalized(np.arange(65), max_iter=1)
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("n,density,empty_frac,long_rows,sigma",
                         [(1, 1.0, 0.0, (), 1), (2, 0.5, 0.0, (), 2), (7, 0.3, 0.2, (), 3),
                          (65, 0.05, 0.2, (), 5), (200, 0.01, 0.3, (), 4),
                          (300, 0.02, 0.2, (17,), 12)],
                         ids=["n1", "n2", "n7", "n65", "n200", "n300"])
def test_personalized_pagerank_tiny_graphs(n, density, empty_frac, long_rows, sigma, dtype):
    """Tiny square graphs (empty rows, dangling vertices, a dense row that
    fills single-row tiles, tiles of a few rows) with 33 and then 64 sources
    on the same plan (slabs of 32 + 1 and 32 + 32 columns; sources repeat
    when n < k), 13 iterations in chunks of 4, every entry against the
    oracle."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, _ = graphgen.random_csr(n, n, density, seed=n, empty_frac=empty_frac,
                                     long_rows=long_rows)
    assert len(col) > 0
    vals = graphgen.column_stochastic_values(col, n)
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, n, sigma=sigma)
    vh = host_values(vals, dtype)
    for k in (33, 64):
        src = ((np.arange(k) * 7 + 3) % n).astype(np.int32)
        X, iters, resid, _ = plan.pagerank_personalized(src, alpha=ALPHA, max_iter=13,
                                                        check_every=4)
        torch.cuda.synchronize()
        assert iters == 13 and resid.shape == (k,)
        ref = oracle.personalized_pagerank(rp, col, vh, ALPHA, 13, src)
        _ppr_check(X, ref, dtype, f"n={n} k={k}")
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_personalized_pagerank_rmat22(dtype):
    """64 sources on R-MAT scale 22 (the benchmark's workload: two compact
    32-column slabs of 4.19M rows), 5 iterations; four sampled columns, two
    in each slab, are checked in full against the oracle, all 64 columns for
    mass 1."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    w = workload("rmat22")
    rp, col, vals, n = w["row_ptr"], w["col"], w["values"], w["n_rows"]
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, n)
    src = graphgen.ppr_sources(n, 64, seed=4)
    X, iters, _, _ = plan.pagerank_personalized(src, alpha=ALPHA, max_iter=5)
    torch.cuda.synchronize()
    assert iters == 5
    mass = X.double().sum(0).cpu().numpy()
    assert np.all(np.abs(mass - 1.0) <= (1e-5 if dtype == torch.float32 else 1e-12))
    vh = host_values(vals, dtype)
    for j in (0, 21, 42, 63):
        ref = oracle.personalized_pagerank(rp, col, vh, ALPHA, 5, [src[j]])[:, 0]
        _ppr_check(X[:, j:j + 1], ref[:, None], dtype, f"column {j}")
    plan.close()


# ----------------------------------------------------- many graphs, one plan


def _multi_x0(graph_ptr, dtype):
    sizes = np.diff(graph_ptr)
    return np.repeat(1.0 / sizes, sizes).astype(_np_dtype(dtype)).astype(np.float64)


def _small_multi(seed, count):
    """count small Chung-Lu graphs of uneven size on one diagonal."""
    return graphgen.chung_lu_multi(count, 1, 3000, 8, seed=seed, graph_seed0=100 * seed)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("seed,count", [(1, 1), (2, 7), (3, 40)])
def test_pagerank_multi_parity(seed, count, dtype):
    """20 iterations of every graph at once against the oracle solving each
    graph on its own; per graph mass 1."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, gp = _small_multi(seed, count)
    n = int(gp[-1])
    vals = graphgen.column_stochastic_values(col, n)
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, n)
    x064 = _multi_x0(gp, dtype)
    x = torch.from_numpy(x064).to(dtype).to(dev)
    iters, resid, _ = plan.pagerank_multi(gp, x, alpha=ALPHA, max_iter=20)
    torch.cuda.synchronize()
    assert iters == 20 and resid.shape == (count,)
    ref = oracle.pagerank_multi(rp, col, host_values(vals, dtype), gp, ALPHA, 20, x064)
    xg = x.double().cpu().numpy()
    rel = np.abs(xg - ref) / ref
    assert rel.max() <= PR_TOL[dtype], rel.max()
    for g in range(count):
        s = xg[gp[g]:gp[g + 1]].sum()
        assert abs(s - 1.0) <= (1e-5 if dtype == torch.float32 else 1e-12)
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_pagerank_multi_single_graph_is_plain(dtype):
    """With one graph the multi-graph driver computes the plain PageRank."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    w = workload("chung_lu_10k")
    rp, col, vals, n = w["row_ptr"], w["col"], w["values"], w["n_rows"]
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, n)
    x1 = torch.full((n,), 1.0 / n, dtype=dtype, device=dev)
    x2 = x1.clone()
    plan.pagerank(x1, max_iter=20)
    plan.pagerank_multi([0, n], x2, max_iter=20)
    torch.cuda.synchronize()
    rel = ((x1.double() - x2.double()).abs() / x1.double()).max().item()
    assert rel <= PR_TOL[dtype]
    plan.close()


def test_pagerank_multi_convergence_and_errors():
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, gp = _small_multi(4, 12)
    n = int(gp[-1])
    vals = graphgen.column_stochastic_values(col, n)
    r, c, v = to_device(rp, col, vals, torch.float64, dev)
    plan = pkg.Plan(r, c, v, n)
    x = torch.from_numpy(_multi_x0(gp, torch.float64)).to(dev)
    iters, resid, conv = plan.pagerank_multi(gp, x, tol=1e-10, max_iter=400, check_every=4)
    assert conv and iters % 4 == 0 and np.all(resid < 1e-10)
    ref = oracle.pagerank_multi(rp, col, vals, gp, ALPHA, 300, _multi_x0(gp, torch.float64))
    assert np.abs(x.cpu().numpy() - ref).max() <= 1e-9
    bad = gp.copy()
    bad[1] = bad[0]
    for g in (bad, gp[:-1], np.concatenate([gp, [n + 1]])):
        with pytest.raises(pkg.MerbitError):
            plan.pagerank_multi(g, x, max_iter=1)
    plan.close()


@pytest.mark.parametrize("stripes", [0, 8], ids=["plain", "striped8"])
@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_pagerank_multi_partial_hot_cache(dtype, stripes):
    """A partial hot-column cache on the many-graph plan: the update writes
    the next SpMV's hot values (each with its own graph's teleport), and only
    each call's first chunk gathers them (a graph of its own).  Chunks of 4
    iterations are recorded and replayed over repeated calls, each result
    against the per-graph oracle."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, gp = _small_multi(5, 24)
    n = int(gp[-1])
    vals = graphgen.column_stochastic_values(col, n)
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, n, commit="wave", hot_columns=300, stripes=stripes)
    info = plan.info()
    assert 0 < info["hot_columns"] < n and info["hot_coverage"] < 1.0
    x064 = _multi_x0(gp, dtype)
    vh = host_values(vals, dtype)
    for iters in (12, 10, 12, 12):
        x = torch.from_numpy(x064).to(dtype).to(dev)
        got_iters, _, _ = plan.pagerank_multi(gp, x, alpha=ALPHA, max_iter=iters, check_every=4)
        y = plan.spmv(x)  # eager work on the same plan (its own hot gather) between calls
        torch.cuda.synchronize()
        assert got_iters == iters and torch.isfinite(y).all()
        ref = oracle.pagerank_multi(rp, col, vh, gp, ALPHA, iters, x064)
        rel = np.abs(x.double().cpu().numpy() - ref) / ref
        assert rel.max() <= PR_TOL[dtype], f"{iters} iterations: {rel.max():.3e}"
    plan.close()


def test_pagerank_multi_256_graphs_full_size():
    """The 256-graph workload (log-uniform sizes 1,000 .. 200,000, degree 8),
    FP32, 10 iterations, on a plain plan and on an 8-stripe plan of the kind
    the benchmark tunes (64-bit descriptors, sigma 28, 512 lanes; partial hot
    sets, so the update writes the hot values): every vertex against the
    per-graph oracle."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    w = workload("chung_lu_multi256")
    rp, col, vals, n, gp = w["row_ptr"], w["col"], w["values"], w["n_rows"], w["graph_ptr"]
    r, c, v = to_device(rp, col, vals, torch.float32, dev)
    x064 = _multi_x0(gp, torch.float32)
    ref = oracle.pagerank_multi(rp, col, host_values(vals, torch.float32), gp, ALPHA, 10, x064)
    for kw in ({}, {"stripes": 8, "desc_bits": 64, "sigma": 28, "block_lanes": 512,
                    "commit": "wave"}):
        plan = pkg.Plan(r, c, v, n, **kw)
        x = torch.from_numpy(x064).float().to(dev)
        plan.pagerank_multi(gp, x, max_iter=10)
        torch.cuda.synchronize()
        rel = np.abs(x.double().cpu().numpy() - ref) / ref
        print(f"multi256 {kw or 'plain'}: max rel {rel.max():.3e}", flush=True)
        assert rel.max() <= PR_TOL[torch.float32], (kw, rel.max())
        plan.close()


def test_batched_graph_replays_match_eager():
    """Personalised and multi-graph drivers with HIP-graph chunks against the
    same drivers launching every kernel directly, over repeated calls."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    w = workload("chung_lu_10k")
    rp, col, vals, n = w["row_ptr"], w["col"], w["values"], w["n_rows"]
    r, c, v = to_device(rp, col, vals, torch.float64, dev)
    g_plan = pkg.Plan(r, c, v, n)
    e_plan = pkg.Plan(r, c, v, n, eager_loops=True)
    src = graphgen.ppr_sources(n, 9, seed=6)
    ref = oracle.personalized_pagerank(rp, col, vals, ALPHA, 9, src)
    gp = np.array([0, 1234, 5000, n], np.int64)
    for rep in range(3):
        Xg, _, _, _ = g_plan.pagerank_personalized(src, max_iter=9, check_every=3)
        Xe, _, _, _ = e_plan.pagerank_personalized(src, max_iter=9, check_every=3)
        torch.cuda.synchronize()
        _ppr_check(Xg, ref, torch.float64, f"graph replay {rep}")
        _ppr_check(Xe, ref, torch.float64, f"eager {rep}")
        xg = torch.full((n,), 1.0 / n, dtype=torch.float64, device=dev)
        xe = xg.clone()
        g_plan.pagerank_multi(gp, xg, max_iter=6, check_every=2)
        e_plan.pagerank_multi(gp, xe, max_iter=6, check_every=2)
        torch.cuda.synchronize()
        d = ((xg - xe).abs() / xe).max().item()
        assert d <= 2 * PR_TOL[torch.float64], f"multi replay {rep}: {d:.3e}"
    g_plan.close()
    e_plan.close()
