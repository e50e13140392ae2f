"""GPU parity of column-stripe plans (the matrix stacked by column stripe,
rows = non-empty (stripe, row) pairs, tiles split into one range per XCD)
against the oracle: the plan of the stacked matrix bit exact, y = A x within
the SpMV tolerance, PageRank iterate by iterate, BiCGSTAB and the
multi-graph PageRank on such plans, graph replays, set_values, and the entry
points that refuse a striped plan."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from helpers import (workload, OMEGA, PR_TOL, case_matrix, check_spmv, host_values,
                     require_gpu, seeded_x, spmv_cases, stacked_row_ptr, to_device)

pytestmark = pytest.mark.gpu
DTYPES = [torch.float32, torch.float64]
CASES = spmv_cases()
ALPHA = 0.85


def _plan(rp, col, vals, nc, dtype, dev, **kw):
    import paper_2605_07391_amd as pkg
    r, c, v = to_device(rp, col, vals, dtype, dev)
    return pkg.Plan(r, c, v, nc, **kw), (r, c, v)


@pytest.mark.parametrize("sigma", [4, 12])
@pytest.mark.parametrize("stripes", [2, 8, 32])
@pytest.mark.parametrize("name", list(CASES))
def test_stacked_plan_bit_exact(name, stripes, sigma):
    dev = require_gpu()
    rp, col, vals, nc = case_matrix(CASES, name)
    plan, keep = _plan(rp, col, vals, nc, torch.float32, dev, sigma=sigma, stripes=stripes)
    info = plan.info()
    if len(col) == 0:
        assert info["stripes"] == 1 and info["plan_rows"] == len(rp) - 1
        plan.close()
        return
    vrp, _ = stacked_row_ptr(rp, col, nc, stripes)
    assert info["stripes"] == stripes and info["plan_rows"] == len(vrp) - 1
    tx, ty, ld = plan.export()
    ox, oy, od = oracle.plan(vrp, OMEGA, sigma)
    assert np.array_equal(tx, ox) and np.array_equal(ty, oy) and np.array_equal(ld, od)
    plan.close()


# (stripes, hot_columns, block_lanes): 0 lanes = the default (1024 FP32, 512 FP64)
STRIPED = [(2, -1, 0), (8, 0, 256), (8, -1, 0), (8, 37, 256), (32, -1, 256), (32, 37, 0)]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("stripes,hot,block_lanes", STRIPED,
                         ids=[f"S{a}h{b}b{c}" for a, b, c in STRIPED])
@pytest.mark.parametrize("name", list(CASES))
def test_striped_spmv_parity(name, stripes, hot, block_lanes, dtype):
    dev = require_gpu()
    rp, col, vals, nc = case_matrix(CASES, name, seed=stripes)
    plan, keep = _plan(rp, col, vals, nc, dtype, dev, stripes=stripes, hot_columns=hot,
                       block_lanes=block_lanes)
    info = plan.info()
    if hot == 0:
        assert info["hot_columns"] == 0
    if hot == 37 and len(col):
        # at most 37 per range
        assert 0 < info["hot_columns"] <= 37 * info["ranges"]
    assert info["grid"] % info["ranges"] == 0
    x64 = seeded_x(nc, stripes + hot, dtype)
    x = torch.from_numpy(x64).to(dtype).to(dev)
    for rep in range(3):  # the plan alternates its two buffers of A' x
        y = torch.full((len(rp) - 1,), float("nan"), dtype=dtype, device=dev)
        plan.spmv(x, out=y)
        torch.cuda.synchronize()
        check_spmv(y, rp, col, host_values(vals, dtype), x64, dtype,
                   f"{name} S={stripes} hot={hot} rep={rep}")
    plan.close()


def test_ranges_used_on_a_larger_matrix():
    """chung_lu_10k with 256 lanes per block gives a grid of at least 8
    blocks: the tiles are split into 8 ranges."""
    dev = require_gpu()
    rp, col, vals, nc = case_matrix(CASES, "chung_lu_10k", seed=1)
    plan, keep = _plan(rp, col, vals, nc, torch.float32, dev, stripes=8, block_lanes=256)
    info = plan.info()
    assert info["ranges"] == 8 and info["grid"] % 8 == 0 and info["grid"] >= 8
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_striped_dual_and_set_values(dtype):
    dev = require_gpu()
    rp, col, vals, nc = case_matrix(CASES, "chung_lu_10k", seed=4)
    plan, keep = _plan(rp, col, vals, nc, dtype, dev, stripes=8, block_lanes=256)
    n = len(rp) - 1
    z = torch.full((n,), 5.0, dtype=dtype, device=dev)
    for it in range(4):
        x64 = seeded_x(nc, 30 + it, dtype)
        x = torch.from_numpy(x64).to(dtype).to(dev)
        y = torch.full((n,), float("nan"), dtype=dtype, device=dev)
        plan.spmv_dual(x, y, z)
        torch.cuda.synchronize()
        check_spmv(y, rp, col, host_values(vals, dtype), x64, dtype, f"dual {it}")
    # z is not touched by a striped plan, and zero_boundary does nothing
    plan.zero_boundary(z)
    torch.cuda.synchronize()
    assert bool((z == 5.0).all())
    vals2 = vals * -1.5 + 0.25
    v2 = torch.from_numpy(vals2).to(dtype).to(dev)
    plan.set_values(v2)
    x64 = seeded_x(nc, 40, dtype)
    y = plan.spmv(torch.from_numpy(x64).to(dtype).to(dev))
    torch.cuda.synchronize()
    check_spmv(y, rp, col, host_values(vals2, dtype), x64, dtype, "set_values")
    plan.close()


@pytest.mark.parametrize("hot", [-1, 37])
@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_striped_pagerank_iterates(dtype, hot):
    dev = require_gpu()
    w = workload("chung_lu_10k")
    n = w["n_rows"]
    plan, keep = _plan(w["row_ptr"], w["col"], w["values"], n, dtype, dev, stripes=8,
                       block_lanes=256, hot_columns=hot)
    x0 = np.full(n, 1.0 / n).astype(np.float32 if dtype == torch.float32 else np.float64)
    x0_64 = x0.astype(np.float64)
    vals = host_values(w["values"], dtype)
    _, resid_ref, hist = oracle.pagerank(w["row_ptr"], w["col"], vals, ALPHA, 25, x0_64,
                                         history=True)
    for t in (1, 2, 7, 10, 11, 20, 25):
        x = torch.from_numpy(x0).to(dev)
        iters, resid, conv = plan.pagerank(x, ALPHA, tol=0.0, max_iter=t)
        assert iters == t and conv
        got = x.double().cpu().numpy()
        rel = np.abs(got - hist[t - 1]) / hist[t - 1]
        assert rel.max() <= PR_TOL[dtype], f"iteration {t}: {rel.max():.3e}"
        assert abs(resid - resid_ref[t - 1]) <= 1e-3 * resid_ref[t - 1] + 1e-7
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_striped_pagerank_graph_replays_match_eager(dtype):
    """The iteration chunks are replayed from HIP graphs keyed on the stacked
    buffers' parity too: several calls (odd and even chunk lengths) agree
    with eager launches."""
    dev = require_gpu()
    w = workload("chung_lu_10k")
    n = w["n_rows"]
    pg, keep = _plan(w["row_ptr"], w["col"], w["values"], n, dtype, dev, stripes=8,
                     block_lanes=256)
    pe, keep2 = _plan(w["row_ptr"], w["col"], w["values"], n, dtype, dev, stripes=8,
                      block_lanes=256, eager_loops=True)
    x0 = torch.full((n,), 1.0 / n, dtype=dtype, device=dev)
    for max_iter, every in ((10, 5), (13, 5), (9, 3), (10, 5), (7, 7), (30, 10)):
        xg, xe = x0.clone(), x0.clone()
        pg.pagerank(xg, ALPHA, max_iter=max_iter, check_every=every)
        pe.pagerank(xe, ALPHA, max_iter=max_iter, check_every=every)
        torch.cuda.synchronize()
        rel = ((xg.double() - xe.double()).abs() / xe.double()).max().item()
        assert rel <= PR_TOL[dtype], (max_iter, every, rel)
        # plain SpMV calls between drivers flip the stacked buffers
        pg.spmv(x0)
    pg.close()
    pe.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_striped_multi_graph_pagerank(dtype):
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, gp = graphgen.chung_lu_multi(40, 1, 3000, 8, seed=3, graph_seed0=300)
    n = int(gp[-1])
    vals = graphgen.column_stochastic_values(col, n)
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, n, stripes=8, block_lanes=256)
    x064 = np.repeat(1.0 / np.diff(gp), np.diff(gp))
    x064 = x064.astype(np.float32 if dtype == torch.float32 else np.float64).astype(np.float64)
    x = torch.from_numpy(x064).to(dtype).to(dev)
    iters, resid, _ = plan.pagerank_multi(gp, x, alpha=ALPHA, max_iter=20)
    torch.cuda.synchronize()
    ref = oracle.pagerank_multi(rp, col, host_values(vals, dtype), gp, ALPHA, 20, x064)
    rel = np.abs(x.double().cpu().numpy() - ref) / ref
    assert iters == 20 and rel.max() <= PR_TOL[dtype]
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_striped_bicgstab_iterates(dtype):
    import scipy.sparse as sp
    dev = require_gpu()
    n = 3000
    rng = np.random.default_rng(5)
    A = sp.random(n, n, density=0.003, random_state=rng, format="csr")
    A.data = rng.uniform(-1, 1, A.nnz)
    A = (A + sp.diags(np.asarray(abs(A).sum(axis=1)).ravel() + 1.0)).tocsr()
    A.sort_indices()
    rp, col = A.indptr.astype(np.int32), A.indices.astype(np.int32)
    npd = np.float32 if dtype == torch.float32 else np.float64
    vals = A.data.astype(npd).astype(np.float64)
    plan, keep = _plan(rp, col, vals, n, dtype, dev, stripes=4, block_lanes=256)
    b = graphgen.uniform(5, 86, n, -1.0, 1.0).astype(npd).astype(np.float64)
    bt = torch.from_numpy(b).to(dtype).to(dev)
    for k in (1, 3, 8):
        x = torch.zeros(n, dtype=dtype, device=dev)
        it, res, status = plan.bicgstab(bt, x, tol=0.0, max_iter=k, check_every=3)
        ref, _, _, hist = oracle.bicgstab(rp, col, vals, b, np.zeros(n), 1e-300, k)
        err = np.abs(x.double().cpu().numpy() - ref).max() / np.abs(ref).max()
        assert it == k and err <= (1e-4 if dtype == torch.float32 else 1e-10) * k, err
    plan.close()


def test_striped_plan_refuses_tile_level_entry_points():
    import paper_2605_07391_amd.merbit as pkg
    dev = require_gpu()
    rp, col, vals, nc = case_matrix(CASES, "random2_1200x800", seed=2)
    plan, keep = _plan(rp, col, vals, nc, torch.float32, dev, stripes=4)
    n = len(rp) - 1
    X = torch.zeros(nc, 4, device=dev)
    for call in (lambda: plan.spmm(X), lambda: plan.transpose(),
                 lambda: plan.sddmm(torch.zeros(n, device=dev), torch.zeros(nc, device=dev))):
        with pytest.raises(pkg.MerbitError) as e:
            call()
        assert e.value.code == pkg.EUNSUPPORTED
    plan.close()
    with pytest.raises(pkg.MerbitError) as e:  # block commit
        _plan(rp, col, vals, nc, torch.float32, dev, stripes=4, commit="block")
    assert e.value.code == pkg.EUNSUPPORTED
    for bad in (3, 64, -2):
        with pytest.raises(pkg.MerbitError) as e:
            _plan(rp, col, vals, nc, torch.float32, dev, stripes=bad)
        assert e.value.code == pkg.EINVAL


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_striped_rmat22_full_size(dtype):
    """R-MAT scale 22 with 8 stripes in the benchmark's launch configuration:
    the stacked plan bit exact and every row of y within tolerance."""
    dev = require_gpu()
    w = workload("rmat22")
    rp, col, vals, n = w["row_ptr"], w["col"], w["values"], w["n_rows"]
    plan, keep = _plan(rp, col, vals, n, dtype, dev, stripes=8)
    info = plan.info()
    assert info["stripes"] == 8 and info["ranges"] == 8 and info["hot_coverage"] > 0.5
    sigma = info["sigma"]
    vrp, _ = stacked_row_ptr(rp, col, n, 8)
    assert info["plan_rows"] == len(vrp) - 1
    tx, ty, ld = plan.export()
    ox, oy, od = oracle.plan(vrp, OMEGA, sigma)
    assert np.array_equal(tx, ox) and np.array_equal(ty, oy) and np.array_equal(ld, od)
    for k, x64 in enumerate([np.full(n, 1.0 / n), seeded_x(n, 22, dtype)]):
        x64 = x64.astype(np.float32 if dtype == torch.float32 else np.float64).astype(np.float64)
        x = torch.from_numpy(x64).to(dtype).to(dev)
        for rep in range(2):
            y = torch.full((n,), float("nan"), dtype=dtype, device=dev)
            plan.spmv(x, out=y)
            torch.cuda.synchronize()
            check_spmv(y, rp, col, host_values(vals, dtype), x64, dtype, f"rmat22 S8 x{k}")
    plan.close()


def test_striped_stress24_fp64_full_size():
    dev = require_gpu()
    w = workload("stress24")
    rp, col, vals, n = w["row_ptr"], w["col"], w["values"], w["n_rows"]
    plan, keep = _plan(rp, col, vals, n, torch.float64, dev, stripes=8)
    assert plan.info()["ranges"] == 8
    x64 = w["x"]
    x = torch.from_numpy(x64).to(dev)
    y = plan.spmv(x)
    torch.cuda.synchronize()
    check_spmv(y, rp, col, np.asarray(vals, np.float64), x64, torch.float64, "stress24 S8")
    plan.close()


def test_striped_stress24_fp64_bench_configuration():
    """The FP64 stress matrix at exactly the configuration the benchmark
    times (64-bit descriptors, sigma 20, 512 lanes, 8 stripes; its long hub
    rows span thousands of tiles): every row within 1e-12 of |A||x|, for a
    standalone SpMV and for a chain of dual-buffer launches (the benchmark's
    timed form, whose tile queues reset between launches)."""
    import bench
    dev = require_gpu()
    w = workload("stress24")
    rp, col, vals, n = w["row_ptr"], w["col"], w["values"], w["n_rows"]
    cfg = bench.STRESS_CONFIG
    plan, keep = _plan(rp, col, vals, n, torch.float64, dev, sigma=cfg["sigma"],
                       block_lanes=cfg["block_lanes"], desc_bits=cfg["desc_bits"],
                       stripes=cfg["stripes"])
    info = plan.info()
    assert (info["sigma"], info["desc_bits"], info["stripes"], info["ranges"]) == \
        (cfg["sigma"], cfg["desc_bits"], cfg["stripes"], 8)
    assert info["fast_tiles"] > 0
    vals64 = np.asarray(vals, np.float64)
    x = torch.from_numpy(w["x"]).to(dev)
    y = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    plan.spmv(x, out=y)
    torch.cuda.synchronize()
    check_spmv(y, rp, col, vals64, w["x"], torch.float64, "stress24 bench config")
    ys = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(2)]
    plan.zero_boundary(ys[0])
    for k in range(3):
        plan.spmv_dual(x, ys[k % 2], ys[(k + 1) % 2])
    torch.cuda.synchronize()
    check_spmv(ys[0], rp, col, vals64, w["x"], torch.float64, "stress24 dual chain")
    plan.close()


DESC64 = [(torch.float32, 24, 512), (torch.float32, 16, 256), (torch.float32, 28, 512),
          (torch.float32, 32, 512), (torch.float64, 16, 512), (torch.float64, 14, 256),
          (torch.float64, 20, 512)]


@pytest.mark.parametrize("dtype,sigma,block_lanes", DESC64,
                         ids=[f"{'f32' if d == torch.float32 else 'f64'}s{s}b{b}"
                              for d, s, b in DESC64])
@pytest.mark.parametrize("name", ["random1_700x300", "single_long_row", "long_then_empty",
                                  "chung_lu_10k", "one_column", "fuzz1_3634x3198"])
def test_striped_desc64(name, dtype, sigma, block_lanes):
    """64-bit descriptors on a column-stripe plan: the stacked plan bit exact
    against the oracle's 64-bit TILE, y within tolerance."""
    dev = require_gpu()
    rp, col, vals, nc = case_matrix(CASES, name, seed=sigma)
    plan, keep = _plan(rp, col, vals, nc, dtype, dev, sigma=sigma, block_lanes=block_lanes,
                       desc_bits=64, stripes=8)
    info = plan.info()
    assert info["desc_bits"] == 64 and info["stripes"] == 8
    vrp, _ = stacked_row_ptr(rp, col, nc, 8)
    tx, ty, ld = plan.export()
    ox, oy, od = oracle.plan64(vrp, OMEGA, sigma)
    assert np.array_equal(tx, ox) and np.array_equal(ty, oy) and np.array_equal(ld, od)
    x64 = seeded_x(nc, sigma, dtype)
    for rep in range(2):
        y = torch.full((len(rp) - 1,), float("nan"), dtype=dtype, device=dev)
        plan.spmv(torch.from_numpy(x64).to(dtype).to(dev), out=y)
        torch.cuda.synchronize()
        check_spmv(y, rp, col, host_values(vals, dtype), x64, dtype, f"{name} desc64 S8")
    plan.close()


@pytest.mark.parametrize("dtype,sigma", [(torch.float32, 24), (torch.float32, 28),
                                         (torch.float32, 32), (torch.float64, 16),
                                         (torch.float64, 20)],
                         ids=["f32s24", "f32s28", "f32s32", "f64s16", "f64s20"])
def test_striped_desc64_rmat22_pagerank(dtype, sigma):
    """The 64-bit-descriptor column-stripe configurations at full size (the
    benchmark's autotuner picks among them; their tile queues are in use):
    20 PageRank iterations, replayed from HIP graphs, against the oracle."""
    dev = require_gpu()
    w = workload("rmat22")
    n = w["n_rows"]
    plan, keep = _plan(w["row_ptr"], w["col"], w["values"], n, dtype, dev, sigma=sigma,
                       block_lanes=512, desc_bits=64, stripes=8)
    x0 = np.full(n, 1.0 / n).astype(np.float32 if dtype == torch.float32 else np.float64)
    x = torch.from_numpy(x0).to(dev)
    iters, resid, conv = plan.pagerank(x, ALPHA, tol=0.0, max_iter=20)
    ref, _, _ = oracle.pagerank(w["row_ptr"], w["col"], host_values(w["values"], dtype), ALPHA,
                                20, x0.astype(np.float64))
    rel = np.abs(x.double().cpu().numpy() - ref) / ref
    assert iters == 20 and rel.max() <= PR_TOL[dtype], rel.max()
    plan.close()


@pytest.mark.parametrize("dtype,sigma", [(torch.float32, 32), (torch.float32, 28),
                                         (torch.float64, 20), (torch.float64, 16)],
                         ids=["f32s32", "f32s28", "f64s20", "f64s16"])
def test_striped_desc64_rmat22_mixed_sign_spmv(dtype, sigma):
    """The benchmark's tuned R-MAT 22 configurations (64-bit descriptors,
    512 lanes, 8 stripes, the tile queue in use) on a mixed-sign x: one
    standalone SpMV and a dual-buffer chain, every row within the SpMV
    tolerance of |A||x|."""
    dev = require_gpu()
    w = workload("rmat22")
    rp, col, vals, n = w["row_ptr"], w["col"], w["values"], w["n_rows"]
    plan, keep = _plan(rp, col, vals, n, dtype, dev, sigma=sigma, block_lanes=512,
                       desc_bits=64, stripes=8)
    info = plan.info()
    waves = info["grid"] * info["block_lanes"] // OMEGA
    assert info["tile_num"] >= 12 * waves  # the tile queue's threshold
    x64 = seeded_x(n, 7 + sigma, dtype)
    x = torch.from_numpy(x64).to(dtype).to(dev)
    vh = host_values(vals, dtype)
    y = torch.full((n,), float("nan"), dtype=dtype, device=dev)
    plan.spmv(x, out=y)
    torch.cuda.synchronize()
    check_spmv(y, rp, col, vh, x64, dtype, f"rmat22 s{sigma} mixed sign")
    ys = [torch.empty(n, dtype=dtype, device=dev) for _ in range(2)]
    plan.zero_boundary(ys[0])
    for k in range(4):
        plan.spmv_dual(x, ys[k % 2], ys[(k + 1) % 2])
    torch.cuda.synchronize()
    check_spmv(ys[1], rp, col, vh, x64, dtype, f"rmat22 s{sigma} dual chain")
    plan.close()
