"""GPU parity of the plan (bit exact) and of y = A x (|A||x|-normalised
tolerance) against the CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from helpers import (workload, OMEGA, SPMV_TOL, case_matrix, check_spmv, host_values, require_gpu,
                     seeded_x, spmv_cases, to_device)

pytestmark = pytest.mark.gpu

DTYPES = [torch.float32, torch.float64]


def _boundary_rows(sigma, block_lanes):
    """Row lengths that make rows end exactly at lane, tile and block ends
    (a row of length k takes k + 1 merge-path steps)."""
    lens = [sigma - 1] * 70 + [OMEGA * sigma - 1] * 3 + [block_lanes * sigma - 1] * 2
    lens += [0, 0, 1, sigma, OMEGA * sigma, block_lanes * sigma + 5]
    return lens


CASES = spmv_cases()


def _matrix(name, seed=0):
    return case_matrix(CASES, name, seed)


@pytest.mark.parametrize("sigma", [1, 4, 7, 12])
@pytest.mark.parametrize("name", list(CASES))
def test_plan_bit_exact(name, sigma):
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, vals, nc = _matrix(name)
    r, c, v = to_device(rp, col, vals, torch.float32, dev)
    plan = pkg.Plan(r, c, v, nc, sigma=sigma)
    tx, ty, ld = plan.export()
    ox, oy, od = oracle.plan(rp, OMEGA, sigma)
    assert np.array_equal(tx, ox)
    assert np.array_equal(ty, oy)
    assert np.array_equal(ld, od)
    info = plan.info()
    assert info["tile_num"] == len(ox) - 1 and info["lane_num"] == len(od)
    assert info["fast_tiles"] == int((oy[:-1] >> 31).sum())
    plan.close()


# hot: 0 = no LDS x cache, -1 = automatic (off for matrices this small: too
# few tiles per wavefront to amortise the fill), 37 = a partial cache of the
# 37 most frequent columns, 4096 = every column of a matrix with at most
# 4096 columns (the x-copy form), the 4096 most frequent otherwise
# commit: "block" = b lanes buffered per block (the paper's layout), "wave" =
# one commit unit per tile (b = 64), persistent blocks
CONFIGS = [(1, 256, 0, "block"), (4, 128, -1, "block"), (7, 256, 37, "block"),
           (12, 256, -1, "block"), (12, 512, 0, "block"), (12, 1024, 37, "block"),
           (3, 128, 0, "block"), (2, 512, 37, "block"),
           (1, 256, 0, "wave"), (4, 256, -1, "wave"), (7, 1024, 37, "wave"),
           (12, 1024, 4096, "wave"), (12, 512, 0, "wave"), (5, 1024, -1, "wave"),
           (12, 256, 37, "wave"), (7, 512, 0, "wave")]


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("sigma,block_lanes,hot,commit", CONFIGS,
                         ids=[f"s{a}b{b}h{c}{d}" for a, b, c, d in CONFIGS])
@pytest.mark.parametrize("name", list(CASES))
def test_spmv_parity(name, sigma, block_lanes, hot, commit, dtype):
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, vals, nc = _matrix(name, seed=sigma)
    r, c, v = to_device(rp, col, vals, dtype, dev)
    x64 = seeded_x(nc, sigma, dtype)
    x = torch.from_numpy(x64).to(dtype).to(dev)
    plan = pkg.Plan(r, c, v, nc, sigma=sigma, block_lanes=block_lanes, hot_columns=hot,
                    commit=commit)
    info = plan.info()
    assert info["commit"] == {"block": 1, "wave": 2}[commit]
    if hot in (0, -1) or block_lanes == 128 or len(col) == 0:
        assert info["hot_columns"] == 0  # automatic sizing: these plans are too small
    elif hot == 37:
        assert 0 < info["hot_columns"] <= 37 or nc <= 37
    elif nc <= hot:
        assert info["hot_columns"] == nc  # every column fits in LDS
    else:
        assert 0 < info["hot_columns"] <= hot  # partial cache of the most frequent columns
    y = torch.full((len(rp) - 1,), float("nan"), dtype=dtype, device=dev)
    plan.spmv(x, out=y)
    torch.cuda.synchronize()
    check_spmv(y, rp, col, host_values(vals, dtype), x64, dtype,
               f"{name} sigma={sigma} b={block_lanes}")
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("commit", ["block", "wave"])
@pytest.mark.parametrize("hot", [0, -1, 5])
@pytest.mark.parametrize("sigma", [4, 7, 12])
def test_rows_ending_on_lane_tile_block_boundaries(sigma, hot, commit, dtype):
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    sizes = (256, 512, 1024) if (hot or commit == "wave") else (128, 256, 512, 1024)
    for block_lanes in sizes:
        lens = _boundary_rows(sigma, block_lanes)
        nc = max(lens) + 1
        rp, col, vals = graphgen.csr_from_lengths(lens, nc, seed=sigma + block_lanes)
        r, c, v = to_device(rp, col, vals, dtype, dev)
        x64 = seeded_x(nc, 3, dtype)
        x = torch.from_numpy(x64).to(dtype).to(dev)
        plan = pkg.Plan(r, c, v, nc, sigma=sigma, block_lanes=block_lanes, hot_columns=hot,
                        commit=commit)
        tx, ty, ld = plan.export()
        ox, oy, od = oracle.plan(rp, OMEGA, sigma)
        assert np.array_equal(ty, oy) and np.array_equal(ld, od) and np.array_equal(tx, ox)
        y = plan.spmv(x)
        torch.cuda.synchronize()
        check_spmv(y, rp, col, host_values(vals, dtype), x64, dtype, f"b={block_lanes}")
        plan.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("commit", ["block", "wave"])
@pytest.mark.parametrize("hot", [0, -1, 300])
def test_dual_buffer_chain(dtype, hot, commit):
    """Alternating outputs: each call needs y zero at the boundary rows and
    leaves z zero there (Sec. 4.2, optimisation (3))."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, vals, nc = _matrix("chung_lu_10k", seed=5)
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, nc, hot_columns=hot, commit=commit)
    n = len(rp) - 1
    bufs = [torch.full((n,), float("nan"), dtype=dtype, device=dev) for _ in range(2)]
    plan.zero_boundary(bufs[0])
    for it in range(5):
        x64 = seeded_x(nc, 10 + it, dtype)
        x = torch.from_numpy(x64).to(dtype).to(dev)
        plan.spmv_dual(x, bufs[it % 2], bufs[(it + 1) % 2])
        torch.cuda.synchronize()
        check_spmv(bufs[it % 2], rp, col, host_values(vals, dtype), x64, dtype, f"iter {it}")
    plan.close()


@pytest.mark.parametrize("stripes", [0, 8], ids=["plain", "striped8"])
def test_smaller_hot_set_later_keeps_earlier_plan_launchable(stripes):
    """Two plans of one kernel instance: the second, built later with a much
    smaller hot set, must not shrink the dynamic-LDS allowance the first one
    launches with (the allowance belongs to the kernel, not to a plan)."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    dtype = torch.float32
    rp, col, vals, nc = _matrix("chung_lu_10k", seed=3)
    r, c, v = to_device(rp, col, vals, dtype, dev)
    big = pkg.Plan(r, c, v, nc, commit="wave", stripes=stripes, hot_columns=8192)
    rp2, col2, vals2, nc2 = _matrix("random2_1200x800", seed=4)
    r2, c2, v2 = to_device(rp2, col2, vals2, dtype, dev)
    small = pkg.Plan(r2, c2, v2, nc2, commit="wave", stripes=stripes, hot_columns=64)
    ib, isml = big.info(), small.info()
    assert (ib["sigma"], ib["block_lanes"], ib["desc_bits"]) == \
        (isml["sigma"], isml["block_lanes"], isml["desc_bits"])
    assert ib["lds_bytes"] > isml["lds_bytes"]
    x64 = seeded_x(nc, 21, dtype)
    y = big.spmv(torch.from_numpy(x64).to(dtype).to(dev))
    torch.cuda.synchronize()
    check_spmv(y, rp, col, host_values(vals, dtype), x64, dtype, "earlier plan")
    x64b = seeded_x(nc2, 22, dtype)
    y2 = small.spmv(torch.from_numpy(x64b).to(dtype).to(dev))
    torch.cuda.synchronize()
    check_spmv(y2, rp2, col2, host_values(vals2, dtype), x64b, dtype, "later plan")
    big.close()
    small.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_set_values_and_repeat(dtype):
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, vals, nc = _matrix("random2_1200x800", seed=1)
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, nc)
    x64 = seeded_x(nc, 4, dtype)
    x = torch.from_numpy(x64).to(dtype).to(dev)
    y1 = plan.spmv(x)
    y2 = plan.spmv(x, out=torch.full_like(y1, 7.0))
    torch.cuda.synchronize()
    check_spmv(y1, rp, col, host_values(vals, dtype), x64, dtype)
    check_spmv(y2, rp, col, host_values(vals, dtype), x64, dtype)
    vals2 = vals * -2.5
    v2 = torch.from_numpy(vals2).to(dtype).to(dev)
    plan.set_values(v2)
    y3 = plan.spmv(x)
    torch.cuda.synchronize()
    check_spmv(y3, rp, col, host_values(vals2, dtype), x64, dtype)
    plan.close()


def test_validation_and_degenerate_shapes():
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    f = torch.float32
    # decreasing row_ptr
    r, c, v = to_device(np.array([0, 3, 2, 4], np.int32), np.zeros(4, np.int32), np.ones(4), f,
                        dev)
    with pytest.raises(pkg.MerbitError):
        pkg.Plan(r, c, v, 2)
    # column out of range
    r, c, v = to_device(np.array([0, 2], np.int32), np.array([0, 5], np.int32), np.ones(2), f,
                        dev)
    with pytest.raises(pkg.MerbitError):
        pkg.Plan(r, c, v, 3)
    # row_ptr[n] != nnz
    r, c, v = to_device(np.array([0, 1], np.int32), np.array([0, 0], np.int32), np.ones(2), f,
                        dev)
    with pytest.raises(pkg.MerbitError):
        pkg.Plan(r, c, v, 3)
    # no rows at all
    r, c, v = to_device(np.array([0], np.int32), np.zeros(0, np.int32), np.zeros(0), f, dev)
    plan = pkg.Plan(r, c, v, 5)
    y = plan.spmv(torch.ones(5, dtype=f, device=dev))
    assert y.numel() == 0
    tx, ty, ld = plan.export()
    assert list(tx) == [0] and list(ty) == [0] and len(ld) == 0
    plan.close()
    # rows but no nonzeros: y = 0 whatever it held
    r, c, v = to_device(np.zeros(1000, np.int32), np.zeros(0, np.int32), np.zeros(0), f, dev)
    plan = pkg.Plan(r, c, v, 0)
    y = plan.spmv(torch.zeros(0, dtype=f, device=dev),
                  out=torch.full((999,), float("nan"), dtype=f, device=dev))
    torch.cuda.synchronize()
    assert torch.all(y == 0)
    plan.close()


def test_profile_counts_launches():
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, vals, nc = _matrix("chung_lu_10k")
    r, c, v = to_device(rp, col, vals, torch.float32, dev)
    plan = pkg.Plan(r, c, v, nc)
    x = torch.ones(nc, device=dev)
    plan.profile_enable(True)
    for _ in range(3):
        plan.spmv(x)
    n, ms = plan.profile_read()
    assert n == 3 and ms > 0
    plan.profile_enable(False)
    plan.spmv(x)
    assert plan.profile_read()[0] == 0
    plan.close()


@pytest.mark.parametrize("dtype,sigma", [(torch.float32, 12), (torch.float64, 7)],
                         ids=["f32s12", "f64s7"])
@pytest.mark.parametrize("hot,block_lanes,commit",
                         [(-1, 0, "auto"), (0, 0, "wave"), (0, 0, "block"), (8192, 1024, "block")],
                         ids=["auto", "wave_nohot", "block_nohot", "block_hot_b1024"])
def test_rmat22_full_size(dtype, sigma, hot, block_lanes, commit):
    """R-MAT scale 22 (the benchmark matrix) at full size: plan bit exact and
    every row of y within tolerance, in the benchmark's launch configuration."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    w = workload("rmat22")
    rp, col, vals, n = w["row_ptr"], w["col"], w["values"], w["n_rows"]
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, n, sigma=sigma, hot_columns=hot, block_lanes=block_lanes,
                    commit=commit)
    info = plan.info()
    if hot == 0:
        assert info["hot_columns"] == 0
    elif hot < 0:
        # the most frequent columns hold well over the automatic threshold
        assert info["hot_columns"] > 1000 and info["hot_coverage"] > 0.3
    else:
        # the 8192 most frequent columns hold ~33 % of the nonzeros
        assert 1000 < info["hot_columns"] <= hot and info["hot_coverage"] > 0.25
    tx, ty, ld = plan.export()
    ox, oy, od = oracle.plan(rp, OMEGA, sigma)
    assert np.array_equal(tx, ox) and np.array_equal(ty, oy) and np.array_equal(ld, od)
    # x: a PageRank-like positive vector plus a mixed-sign one
    for k, x64 in enumerate([np.full(n, 1.0 / n), seeded_x(n, 22, dtype)]):
        x64 = x64.astype(np.float32 if dtype == torch.float32 else np.float64).astype(np.float64)
        x = torch.from_numpy(x64).to(dtype).to(dev)
        y = torch.full((n,), float("nan"), dtype=dtype, device=dev)
        plan.spmv(x, out=y)
        torch.cuda.synchronize()
        check_spmv(y, rp, col, host_values(vals, dtype), x64, dtype, f"rmat22 x{k}")
    plan.close()


@pytest.mark.parametrize("commit,hot", [("wave", -1), ("block", 0)], ids=["wave_hot", "block"])
def test_stress24_fp64_full_size(commit, hot):
    """The irregular stress matrix at full size (R-MAT scale 24, 30 % of rows
    cleared, 8 rows of 2,000,000 nonzeros, values in (0, 1], x in [-1, 1)),
    FP64, sigma 7: plan bit exact, every row of y within 1e-12 |A||x|.  Hub
    rows span thousands of tiles, so their partial sums cross thousands of
    commit units."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    w = workload("stress24")
    rp, col, vals, n, x64 = w["row_ptr"], w["col"], w["values"], w["n_rows"], w["x"]
    r, c, v = to_device(rp, col, vals, torch.float64, dev)
    plan = pkg.Plan(r, c, v, n, sigma=7, commit=commit, hot_columns=hot)
    if commit == "wave":
        tx, ty, ld = plan.export()
        ox, oy, od = oracle.plan(rp, OMEGA, 7)
        assert np.array_equal(tx, ox) and np.array_equal(ty, oy) and np.array_equal(ld, od)
        del tx, ty, ld, ox, oy, od
    x = torch.from_numpy(x64).to(dev)
    y = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    plan.spmv(x, out=y)
    torch.cuda.synchronize()
    check_spmv(y, rp, col, vals, x64, torch.float64, f"stress24 {commit}")
    # a hub row is a sum of 2,000,000 products
    hub = w["meta"]["hub_rows"][0]
    assert rp[hub + 1] - rp[hub] == 2_000_000
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_autotuner_picks_a_measured_candidate(dtype):
    """The tuner times every built (sigma, block size) pair, reports -1 for a
    pair the kernels do not build, and returns the fastest; a plan with its
    choice is exact against the oracle."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, vals, nc = _matrix("chung_lu_10k", seed=2)
    r, c, v = to_device(rp, col, vals, dtype, dev)
    best, table = pkg.tune(r, c, v, nc, sigmas=[5, 12, 13], block_lanes=[256, 1024, 192],
                           reps=5)
    assert table[(13, 256)] == -1.0 and table[(12, 192)] == -1.0
    measured = {k: t for k, t in table.items() if t >= 0}
    assert len(measured) == 4 and all(t > 0 for t in measured.values())
    assert (best["sigma"], best["block_lanes"]) == min(measured, key=measured.get)
    plan = pkg.Plan(r, c, v, nc, **best)
    x64 = seeded_x(nc, 1, dtype)
    y = plan.spmv(torch.from_numpy(x64).to(dtype).to(dev))
    torch.cuda.synchronize()
    check_spmv(y, rp, col, host_values(vals, dtype), x64, dtype, "tuned")
    plan.close()
    # default candidate sets
    best, table = pkg.tune(r, c, v, nc, reps=3)
    assert len(table) == (6 if dtype == torch.float32 else 7) * 3
    assert best["sigma"] in {s for s, _ in table}


# 64-bit lane descriptors: (dtype, sigma) pairs the wave kernel builds
DESC64 = [(torch.float32, 16), (torch.float32, 20), (torch.float32, 24), (torch.float32, 28),
          (torch.float32, 32), (torch.float64, 14), (torch.float64, 16), (torch.float64, 20),
          (torch.float64, 24)]


@pytest.mark.parametrize("block_lanes,hot", [(256, 0), (512, -1), (512, 37)])
@pytest.mark.parametrize("dtype,sigma", DESC64, ids=[f"{'f32' if d == torch.float32 else 'f64'}s{s}"
                                                     for d, s in DESC64])
@pytest.mark.parametrize("name", ["one_row", "all_rows_empty", "single_long_row", "long_then_empty",
                                  "random1_700x300", "random4_200x3000", "chung_lu_10k",
                                  "fuzz2_3471x315", "one_column"])
def test_desc64_plan_and_spmv(name, dtype, sigma, block_lanes, hot):
    """Plans with 64-bit descriptors are bit exact against the oracle's
    64-bit TILE and give y = A x within the SpMV tolerance."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, vals, nc = _matrix(name, seed=sigma)
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, nc, sigma=sigma, block_lanes=block_lanes, hot_columns=hot,
                    desc_bits=64)
    info = plan.info()
    assert info["desc_bits"] == 64 and info["sigma"] == sigma and info["commit"] == 2
    tx, ty, ld = plan.export()
    ox, oy, od = oracle.plan64(rp, OMEGA, sigma)
    assert ld.dtype == np.uint64
    assert np.array_equal(tx, ox) and np.array_equal(ty, oy) and np.array_equal(ld, od)
    x64 = seeded_x(nc, sigma, dtype)
    y = torch.full((len(rp) - 1,), float("nan"), dtype=dtype, device=dev)
    plan.spmv(torch.from_numpy(x64).to(dtype).to(dev), out=y)
    torch.cuda.synchronize()
    check_spmv(y, rp, col, host_values(vals, dtype), x64, dtype, f"{name} desc64 s{sigma}")
    if len(col):
        with pytest.raises(pkg.MerbitError):  # SpMM walks 32-bit descriptors only
            plan.spmm(torch.zeros(nc, 2, dtype=dtype, device=dev))
    plan.close()


@pytest.mark.parametrize("dtype,sigma", [(torch.float32, 24), (torch.float64, 16)],
                         ids=["f32s24", "f64s16"])
def test_desc64_rmat22_full_size(dtype, sigma):
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    w = workload("rmat22")
    rp, col, vals, n = w["row_ptr"], w["col"], w["values"], w["n_rows"]
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, n, sigma=sigma, desc_bits=64)
    tx, ty, ld = plan.export()
    ox, oy, od = oracle.plan64(rp, OMEGA, sigma)
    assert np.array_equal(tx, ox) and np.array_equal(ty, oy) and np.array_equal(ld, od)
    del tx, ty, ld, ox, oy, od
    x64 = seeded_x(n, 22, dtype)
    y = plan.spmv(torch.from_numpy(x64).to(dtype).to(dev))
    torch.cuda.synchronize()
    check_spmv(y, rp, col, host_values(vals, dtype), x64, dtype, f"rmat22 desc64 s{sigma}")
    # PageRank on the 64-bit plan, a few iterations against the oracle
    x = torch.full((n,), 1.0 / n, dtype=dtype, device=dev)
    plan.pagerank(x, 0.85, max_iter=4)
    x0 = np.full(n, 1.0 / n).astype(np.float32 if dtype == torch.float32 else np.float64)
    ref, _, _ = oracle.pagerank(rp, col, host_values(vals, dtype), 0.85, 4, x0.astype(np.float64))
    rel = np.abs(x.double().cpu().numpy() - ref) / ref
    assert rel.max() <= (1e-4 if dtype == torch.float32 else 1e-11)
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("stripes", [0, 8])
def test_wave_tile_queue_across_launches(stripes, dtype):
    """On a striped plan with at least 12 tiles per wavefront the wave kernel
    deals each wavefront one tile and hands out the rest from a per-range
    counter that the launch's last wavefront resets (R-MAT scale 17, sigma 2,
    256 lanes, one block per CU: about 18 tiles per wavefront); without
    stripes every wavefront takes a fixed sequence.  Consecutive launches,
    dual-buffer launches and a PageRank chain in between must each produce
    the oracle's y."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col = graphgen.rmat_pattern(17, 16, seed=17)
    nc = len(rp) - 1
    vals = np.random.default_rng(17).uniform(-1, 1, len(col))
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, nc, sigma=2, block_lanes=256, blocks_per_cu=1, commit="wave",
                    stripes=stripes)
    info = plan.info()
    waves = info["grid"] * 4
    assert info["tile_num"] >= 12 * waves  # the striped plan uses its tile queues
    vals64 = host_values(vals, dtype)
    for rep in range(4):
        x64 = seeded_x(nc, 40 + rep, dtype)
        x = torch.from_numpy(x64).to(dtype).to(dev)
        y = torch.full((nc,), float("nan"), dtype=dtype, device=dev)
        plan.spmv(x, out=y)
        torch.cuda.synchronize()
        check_spmv(y, rp, col, vals64, x64, dtype, f"S={stripes} launch {rep}")
        if rep == 1:
            xp = torch.full((nc,), 1.0 / nc, dtype=dtype, device=dev)
            plan.pagerank(xp, 0.85, tol=0.0, max_iter=7)
    if stripes == 0:
        bufs = [torch.full((nc,), float("nan"), dtype=dtype, device=dev) for _ in range(2)]
        plan.zero_boundary(bufs[0])
        for it in range(3):
            x64 = seeded_x(nc, 60 + it, dtype)
            x = torch.from_numpy(x64).to(dtype).to(dev)
            plan.spmv_dual(x, bufs[it % 2], bufs[(it + 1) % 2])
            torch.cuda.synchronize()
            check_spmv(bufs[it % 2], rp, col, vals64, x64, dtype, f"dual {it}")
    plan.close()
