"""Benchmark: repeated merge-path SpMV inside PageRank power iterations on one
MI355X, R-MAT scale 22 (4,194,304 rows, ~65.2M nonzeros after merging).

A step is one PageRank iteration: the SpMV (y = P x) plus the update kernel
(x' = alpha y + teleport, dangling mass and l1 change); with a column-stripe
plan the SpMV is the fused kernel on the stacked matrix plus the kernel that
adds each row's stripes.  The plan is built once and timed separately.
`value` is nonzeros processed per second over the timed steps (GNZ/s).  The
roofline block reports the SpMV: algorithmic bytes per SpMV / mean SpMV time
from HIP events around its launches (a separate pass of standalone SpMVs),
against the MI355X HBM peak.  The CPU baseline is the oracle (single thread)
timed on a bounded number of iterations of the same workload.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SpMV GNZ/s and % of HBM peak (FP32/FP64); batched + adjoint vs plain"
CSRC = os.path.join(ROOT, "paper_2605_07391_amd", "csrc")
# fused SpMV kernel of each commit family: (kernel name, source file)
KERNELS = {1: ("merbit::spmv_kernel", "merbit_spmv.hip"),
           2: ("merbit::spmv_wave_kernel", "merbit_spmv_wave.hip")}
# a striped plan's SpMV is the wave kernel on the stacked matrix plus the
# kernel that sums each row's stripes
COMBINE = ("merbit::stripe_combine_kernel", "merbit_stripes.hip")


def spmv_kernels(commit: int, stripes: int):
    return [KERNELS[commit]] + ([COMBINE] if stripes > 1 else [])


def spmv_source_hash(commit: int, stripes: int = 1) -> str:
    h = hashlib.sha256()
    for _, src in spmv_kernels(commit, stripes):
        with open(os.path.join(CSRC, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(info: dict, value_size: int) -> float:
    """Bytes one SpMV must move: values + col_ind once, x once, y once, the
    tile starts and the descriptors of the non-fast tiles (paper Sec. 4.3's
    TILE footprint), each descriptor at its own width (4 or 8 bytes)."""
    m, n_rows, n_cols = info["nnz"], info["n_rows"], info["n_cols"]
    T, lanes = info["tile_num"], info["lane_num"]
    r_f = info["fast_tiles"] / T if T else 0.0
    desc_bytes = info.get("desc_bits", 32) // 8
    return (m * (value_size + 4) + n_cols * value_size + n_rows * value_size + 8 * (T + 1)
            + desc_bytes * lanes * (1.0 - r_f))


def timed_prep_calls(steps: int) -> int:
    """Untimed PageRank calls of exactly the timed call's shape (max_iter =
    steps) run before the clock starts.  Each call records the HIP graphs of
    its chunks for the dual-buffer state it starts from; a call of odd length
    flips that state, so the second call puts it back and the timed call
    starts from a state whose graphs exist, whatever the warm-up did."""
    return 1 + (steps & 1)


def kernel_instance(info: dict) -> str:
    """Name of the fused kernel's template instance a plan launches."""
    v = "float" if info["dtype"] == 0 else "double"
    hot = "true" if info["hot_columns"] else "false"
    waves = info["block_lanes"] // 64
    if info["commit"] == 1:
        return f"merbit::spmv_kernel<{v}, {info['sigma']}, {waves}, {hot}>"
    word = "unsigned long" if info["desc_bits"] == 64 else "unsigned int"
    return f"merbit::spmv_wave_kernel<{v}, {info['sigma']}, {waves}, {hot}, {word}>"


def load_traffic(workload: str, dtype: str, info: dict):
    """Measured HBM bytes per SpMV from the committed rocprofv3 counter
    summary, if it was taken on the same kernel instance, stripe count and
    kernel sources."""
    import glob
    commit, stripes = info["commit"], info["stripes"]
    # one record per measured configuration (the tuned one and near ties)
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", f"spmv_traffic_{workload}_{dtype}*.json")))
    for path in paths:
        with open(path) as f:
            rec = json.load(f)
        if (rec.get("kernel") == kernel_instance(info)
                and rec.get("stripes", 1) == stripes
                and rec.get("spmv_source_sha256_16") == spmv_source_hash(commit, stripes)):
            return rec.get("hbm_bytes_per_launch")
    return None


def traffic_record(workload: str, dtype: str, info: dict, alg_bytes: float, fetch_dir: str,
                   write_dir: str, copy_fetch_dir: str, copy_write_dir: str) -> dict:
    """HBM bytes of one SpMV (fused launch + stripe sum) from four rocprofv3
    --pmc runs (FETCH_SIZE and WRITE_SIZE of the bench at this configuration,
    and of --copy-calibration-mib 1024), each counter scaled by what it reads
    for the plain 1 GiB copy; the record load_traffic() matches against."""
    import collections
    import csv

    def per_dispatch(d, counter):
        acc = collections.defaultdict(lambda: collections.defaultdict(float))
        with open(os.path.join(d, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    acc[r["Kernel_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
        return acc

    def mean_of(acc, name):
        keys = [k for k in acc if name in k]
        if len(keys) != 1:
            raise RuntimeError(f"{name}: {len(keys)} matching kernels")
        vals = list(acc[keys[0]].values())
        return sum(vals) / len(vals), len(vals)

    stripes = info["stripes"]
    names = [kernel_instance(info)] + (
        [f"merbit::stripe_combine_kernel<{'float' if info['dtype'] == 0 else 'double'}, "
         f"{stripes}>"] if stripes > 1 else [])
    fetch, write = per_dispatch(fetch_dir, "FETCH_SIZE"), per_dispatch(write_dir, "WRITE_SIZE")
    f_kib = [mean_of(fetch, k) for k in names]
    w_kib = [mean_of(write, k) for k in names]
    copy_f, _ = mean_of(per_dispatch(copy_fetch_dir, "FETCH_SIZE"), "copyBuffer")
    copy_w, _ = mean_of(per_dispatch(copy_write_dir, "WRITE_SIZE"), "copyBuffer")
    nbytes = 1 << 30
    ff, wf = nbytes / 1024 / copy_f, nbytes / 1024 / copy_w
    f_raw, w_raw = sum(v for v, _ in f_kib), sum(v for v, _ in w_kib)
    rec = {"kernel": names[0], "workload": workload, "dtype": dtype, "stripes": stripes,
           "combine_kernel": names[1] if stripes > 1 else None,
           "spmv_source_files": [src for _, src in spmv_kernels(info["commit"], stripes)],
           "spmv_source_sha256_16": spmv_source_hash(info["commit"], stripes),
           "fetch_size_kib_per_spmv_raw": round(f_raw, 1),
           "write_size_kib_per_spmv_raw": round(w_raw, 1),
           "launches_counted": [f_kib[0][1], w_kib[0][1]],
           "copy_calibration": {"bytes_copied": nbytes, "fetch_kib_raw": round(copy_f, 1),
                                "write_kib_raw": round(copy_w, 1), "fetch_factor": round(ff, 5),
                                "write_factor": round(wf, 5)},
           "hbm_fetch_bytes_per_launch": int(f_raw * 1024 * ff),
           "hbm_write_bytes_per_launch": int(w_raw * 1024 * wf)}
    rec["hbm_bytes_per_launch"] = rec["hbm_fetch_bytes_per_launch"] + rec["hbm_write_bytes_per_launch"]
    rec["algorithmic_bytes_per_launch"] = int(alg_bytes)
    return rec


def run_gpu(w, dtype_name: str, steps: int, warmup: int, sigma: int, block_lanes: int,
            alpha: float, hot_columns: int = -1, commit: str = "auto", blocks_per_cu: int = 0,
            tune: bool = False, stripes: int = 0, desc_bits: int = 32):
    import numpy as np
    import torch

    import paper_2605_07391_amd as pkg

    dev = torch.device("cuda:0")
    dtype = torch.float32 if dtype_name == "f32" else torch.float64
    vsize = 4 if dtype == torch.float32 else 8
    n = w["n_rows"]
    r = torch.from_numpy(w["row_ptr"]).to(dev)
    c = torch.from_numpy(w["col"]).to(dev)
    v = torch.from_numpy(w["values"]).to(dtype).to(dev)
    torch.cuda.synchronize()
    tuning = None
    if tune:
        # sigma, block size, commit family, column stripes and descriptor
        # width by measurement on this matrix (untimed); every table is kept
        # in the output
        def cands_of(table, commit_name, stripes_, bits):
            return [(t, a, b, commit_name, stripes_, bits) for (a, b), t in table.items() if t > 0]

        best, table = pkg.tune(r, c, v, n, reps=10, commit=commit, hot_columns=hot_columns)
        cands = cands_of(table, "wave" if commit == "auto" else commit, 0, 32)
        table_block = table_striped = table64s = None
        if commit == "auto":
            # the paper's block-commit layout, b = 128 .. 1024 lanes, swept as well
            _, table_block = pkg.tune(r, c, v, n, reps=10, commit="block",
                                      hot_columns=hot_columns, block_lanes=[128, 256, 512, 1024])
            cands += cands_of(table_block, "block", 0, 32)
        best64, table64 = pkg.tune(r, c, v, n, reps=10, hot_columns=hot_columns, desc_bits=64,
                                   block_lanes=[256, 512])
        if commit in ("auto", "wave"):
            cands += cands_of(table64, "wave", 0, 64)
        if commit in ("auto", "wave") and stripes < 0:
            # the column-stripe plan (8 stripes, one tile range per XCD), with
            # 32- and 64-bit descriptors; its time includes the launch that
            # adds each row's stripes
            _, table_striped = pkg.tune(r, c, v, n, reps=10, commit="wave",
                                        hot_columns=hot_columns, stripes=8)
            cands += cands_of(table_striped, "wave", 8, 32)
            _, table64s = pkg.tune(r, c, v, n, reps=10, hot_columns=hot_columns, desc_bits=64,
                                   block_lanes=[256, 512], stripes=8)
            cands += cands_of(table64s, "wave", 8, 64)
        # the library default (sigma 12 / 7, 1024 / 512 lanes, wave commit, no
        # stripes, 32-bit descriptors) unless a candidate is more than 2 %
        # faster: near-ties do not flip the configuration from run to run
        d_sigma, d_lanes = (12, 1024) if dtype == torch.float32 else (7, 512)
        t_best, b_sigma, b_lanes, b_commit, b_stripes, b_bits = min(cands)
        t_def = table.get((d_sigma, d_lanes), -1.0)
        if t_def > 0 and t_best >= 0.98 * t_def:
            sigma, block_lanes, commit, stripes, desc_bits = d_sigma, d_lanes, "wave", 0, 32
        else:
            sigma, block_lanes, commit, stripes, desc_bits = (b_sigma, b_lanes, b_commit,
                                                              b_stripes, b_bits)

        def fmt(t):
            return None if t is None else {f"s{a}_b{b}": round(x, 1) for (a, b), x in t.items()}

        tuning = {"chosen": {"sigma": sigma, "block_lanes": block_lanes, "commit": commit,
                             "stripes": stripes, "desc_bits": desc_bits},
                  "rule": "fastest candidate if more than 2 % faster than the default "
                          "(sigma, lanes) of the wave kernel, else the default",
                  "us_per_spmv": fmt(table),
                  "block_commit_us_per_spmv": fmt(table_block),
                  "striped8_us_per_spmv": fmt(table_striped),
                  "desc64": {"best": best64, "us_per_spmv": fmt(table64),
                             "striped8_us_per_spmv": fmt(table64s),
                             "vs_32bit": round(min(t for t in table.values() if t > 0)
                                               / min(t for t in table64.values() if t > 0), 3)}}
    stripes = max(stripes, 0)
    # plan build, timed on its own (kernel + allocation of TILE)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    plan = pkg.Plan(r, c, v, n, sigma=sigma, block_lanes=block_lanes, hot_columns=hot_columns,
                    commit=commit, blocks_per_cu=blocks_per_cu, validate=False,
                    stripes=max(stripes, 0), desc_bits=desc_bits)
    e1.record()
    torch.cuda.synchronize()
    plan_ms = e0.elapsed_time(e1)
    info = plan.info()
    pagerank = w["meta"]["generator"] != "stress"
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    if pagerank:
        # a step is one PageRank iteration: fused SpMV + update kernel
        x = torch.full((n,), 1.0 / n, dtype=dtype, device=dev)
        if warmup > 0:
            plan.pagerank(x, alpha, tol=0.0, max_iter=warmup)
        # the timed call's own chunk shape, untimed: its HIP graphs are
        # recorded before t0 whatever --warmup was
        for _ in range(timed_prep_calls(steps)):
            x.fill_(1.0 / n)
            plan.pagerank(x, alpha, tol=0.0, max_iter=steps)
        x.fill_(1.0 / n)
        torch.cuda.synchronize()
        g_before = plan.info()
        wall0 = time.perf_counter()
        t0.record()
        iters, resid, _ = plan.pagerank(x, alpha, tol=0.0, max_iter=steps)
        t1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        g_after = plan.info()
        graphs = {"captured_in_timed_call": g_after["graph_captures"] - g_before["graph_captures"],
                  "replayed_in_timed_call": g_after["graph_replays"] - g_before["graph_replays"],
                  "prep_calls": timed_prep_calls(steps)}
        mass = float(x.double().sum().item())
        # roofline pass: `steps` standalone SpMVs y = A x on the ranks just
        # computed (the same launches as in a PageRank step), each bracketed
        # by HIP events
        ys = [torch.empty(n, dtype=dtype, device=dev) for _ in range(2)]
        plan.zero_boundary(ys[0])
        plan.spmv_dual(x, ys[0], ys[1])
        plan.profile_enable(True)
        for k in range(steps):
            plan.spmv_dual(x, ys[(k + 1) % 2], ys[k % 2])
    else:
        # a step is one y = A x with the workload's x (dual output buffers)
        x = torch.from_numpy(w["x"]).to(dtype).to(dev)
        ys = [torch.empty(n, dtype=dtype, device=dev) for _ in range(2)]
        plan.zero_boundary(ys[0])
        for k in range(warmup):
            plan.spmv_dual(x, ys[k % 2], ys[(k + 1) % 2])
        base = warmup
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        t0.record()
        for k in range(steps):
            plan.spmv_dual(x, ys[(base + k) % 2], ys[(base + k + 1) % 2])
        t1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        iters, resid, mass = steps, None, None
        graphs = None
        plan.profile_enable(True)
        base += steps
        for k in range(steps):
            plan.spmv_dual(x, ys[(base + k) % 2], ys[(base + k + 1) % 2])
    step_ms = t0.elapsed_time(t1) / steps
    launches, kernel_ms = plan.profile_read()
    plan.profile_enable(False)
    spmv_ms = kernel_ms / max(launches, 1)
    abytes = algorithmic_bytes(info, vsize)
    achieved = abytes / (spmv_ms * 1e-3) / 1e9
    plan.close()
    nnz = info["nnz"]
    return {
        "iters": iters, "resid": resid, "mass": mass, "step_ms": step_ms, "wall_s": wall,
        "plan_ms": plan_ms, "spmv_ms": spmv_ms, "launches": launches, "info": info,
        "tuning": tuning, "graphs": graphs,
        "alg_bytes": abytes, "achieved_gbs": achieved,
        "value_gnzs": nnz * steps / (step_ms * steps * 1e-3) / 1e9,
        "spmv_gnzs": nnz / (spmv_ms * 1e-3) / 1e9,
    }


def run_ppr(w, k: int, steps: int, warmup: int, alpha: float, sigma: int = 0):
    """Personalised PageRank for k sources at once on the workload graph
    (FP32): a step is one SpMM over k right-hand sides plus the per-column
    update, on a plan whose sigma the autotuner measured fastest for the SpMM
    (sigma > 0: that sigma, no tuning; the tuned sigmas are within a few
    percent of each other, so a profile that must see one kernel fixes it).
    Returns step and SpMM-kernel times and the SpMM's bandwidth against its
    compulsory bytes (A once, X once, Y once, the plan's tiles and
    descriptors)."""
    import torch

    import graphgen
    import paper_2605_07391_amd as pkg
    dev = torch.device("cuda:0")
    n = w["n_rows"]
    r = torch.from_numpy(w["row_ptr"]).to(dev)
    c = torch.from_numpy(w["col"]).to(dev)
    v = torch.from_numpy(w["values"]).float().to(dev)
    # sigma of the SpMM by measurement on this matrix (untimed)
    if sigma > 0:
        best, table = {"sigma": sigma}, {}
    else:
        best, table = pkg.tune(r, c, v, n, sigmas=list(range(4, 13)), block_lanes=[256],
                               reps=5, rhs=k)
    plan = pkg.Plan(r, c, v, n, validate=False, sigma=best["sigma"])
    src = graphgen.ppr_sources(n, k, seed=4)
    # untimed: warm-up iterations in the timed run's chunk shape, so its HIP
    # graph is recorded before the clock starts
    X, _, _, _ = plan.pagerank_personalized(src, alpha=alpha, max_iter=max(warmup, steps))
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    X0 = torch.zeros_like(X)
    X0[torch.as_tensor(src, dtype=torch.int64, device=dev), torch.arange(k, device=dev)] = 1.0
    X.copy_(X0)
    t0.record()
    plan.pagerank_personalized(src, X=X, alpha=alpha, max_iter=steps)
    t1.record()
    torch.cuda.synchronize()
    step_ms = t0.elapsed_time(t1) / steps
    mass_err = float((X.double().sum(0) - 1.0).abs().max().item())
    X.copy_(X0)
    plan.profile_enable(True)
    plan.pagerank_personalized(src, X=X, alpha=alpha, max_iter=steps)
    launches, kernel_ms = plan.profile_read()
    info = plan.info()
    plan.close()
    spmm_ms = kernel_ms / max(launches, 1)
    nnz = w["nnz"]
    # compulsory bytes: the single-vector count with x and y widened to k columns
    alg = algorithmic_bytes(info, 4) + (k - 1) * 4 * (info["n_cols"] + info["n_rows"])
    ach = alg / (spmm_ms * 1e-3) / 1e9
    return {"k": k, "steps": steps, "ms_per_step": round(step_ms, 4),
            "spmm_us": round(spmm_ms * 1e3, 1), "sigma": best["sigma"],
            "tuning_spmm_us": {f"s{a}": round(t, 1) for (a, _), t in table.items()},
            "gnz_rhs_per_s": round(nnz * k / (spmm_ms * 1e-3) / 1e9, 2),
            "step_gnz_rhs_per_s": round(nnz * k / (step_ms * 1e-3) / 1e9, 2),
            "max_mass_error": mass_err, "sources_seed": 4,
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                         # the SpMM of the step, fused with the update of the
                         # rows inside tiles: one launch per 32-column slab
                         # (128 bytes of X row), timed together
                         "kernel": f"merbit::spmm_kernel<float, {best['sigma']}, true>",
                         "launches_per_spmm": -(-k // 32),
                         "alg_bytes_per_spmm": int(alg),
                         "mean_spmm_us": round(spmm_ms * 1e3, 1)}}


def run_multi(steps: int, warmup: int, alpha: float, stripes: int = 0, plan_kw=None,
              tune: bool = False):
    """PageRank of the 256 Chung-Lu graphs stored on one diagonal, FP32, one
    plan: a step is one fused SpMV over all graphs plus the per-graph update.
    tune: sigma and block size of the striped plan with 64-bit descriptors
    measured on this matrix (the autotuner, untimed) instead of plan_kw."""
    import numpy as np
    import torch

    import graphgen
    import paper_2605_07391_amd as pkg
    dev = torch.device("cuda:0")
    w = graphgen.workload("chung_lu_multi256")
    n, gp = w["n_rows"], w["graph_ptr"]
    r = torch.from_numpy(w["row_ptr"]).to(dev)
    c = torch.from_numpy(w["col"]).to(dev)
    v = torch.from_numpy(w["values"]).float().to(dev)
    tuning = None
    if tune:
        best, table = pkg.tune(r, c, v, n, reps=10, commit="wave", desc_bits=64,
                               block_lanes=[256, 512], stripes=stripes)
        plan_kw = {"sigma": best["sigma"], "block_lanes": best["block_lanes"], "desc_bits": 64,
                   "commit": "wave"}
        tuning = {f"s{a}_b{b}": round(t, 1) for (a, b), t in table.items()}
    plan = pkg.Plan(r, c, v, n, validate=False, stripes=stripes, **(plan_kw or {}))
    sizes = np.diff(gp)
    x0 = torch.from_numpy(np.repeat(1.0 / sizes, sizes)).float().to(dev)
    x = x0.clone()
    plan.pagerank_multi(gp, x, alpha=alpha, max_iter=max(warmup, steps))  # records the graphs
    x.copy_(x0)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    plan.pagerank_multi(gp, x, alpha=alpha, max_iter=steps)
    t1.record()
    torch.cuda.synchronize()
    step_ms = t0.elapsed_time(t1) / steps
    x.copy_(x0)
    plan.profile_enable(True)
    plan.pagerank_multi(gp, x, alpha=alpha, max_iter=steps)
    launches, kernel_ms = plan.profile_read()
    plan.close()
    spmv_ms = kernel_ms / max(launches, 1)
    nnz = w["nnz"]
    return {"graphs": len(sizes), "n": int(n), "nnz": int(nnz), "steps": steps,
            "ms_per_step": round(step_ms, 4), "spmv_us": round(spmv_ms * 1e3, 1),
            "gnzs": round(nnz / (step_ms * 1e-3) / 1e9, 3),
            "spmv_gnzs": round(nnz / (spmv_ms * 1e-3) / 1e9, 3),
            "stripes": stripes, "plan": plan_kw or "default", "tuning_us_per_spmv": tuning,
            "seed": w["meta"]["seed"]}


def tuned_kw(info) -> dict:
    """Plan options of a tuned striped run, for the other striped workloads."""
    if info["stripes"] <= 1 or {1: "block", 2: "wave"}[info["commit"]] != "wave":
        return {}
    return {"sigma": info["sigma"], "block_lanes": info["block_lanes"],
            "desc_bits": info["desc_bits"], "commit": "wave"}


def run_bicgstab(scale: int, steps: int, stripes: int = 0, plan_kw=None):
    """BiCGSTAB (Sec. 5.5.2) on the symmetric 0/1 R-MAT system of the given
    scale, FP64, b = A x_true: `steps` iterations (two fused SpMVs and five
    vector kernels each) after 20 warm-up iterations.  Returns per-iteration
    time, the SpMV share and the residual reached."""
    import torch

    import graphgen
    import paper_2605_07391_amd as pkg
    dev = torch.device("cuda:0")
    w = graphgen.workload(f"rmat{scale}_sym")
    n = w["n_rows"]
    r = torch.from_numpy(w["row_ptr"]).to(dev)
    c = torch.from_numpy(w["col"]).to(dev)
    v = torch.from_numpy(w["values"]).to(dev)
    plan = pkg.Plan(r, c, v, n, validate=False, stripes=stripes, **(plan_kw or {}))
    b = plan.spmv(torch.from_numpy(w["x"]).to(dev))
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    # two chunks of the timed run's shape: both of its HIP graphs are recorded
    plan.bicgstab(b, x, tol=0.0, max_iter=20, check_every=10)
    x.zero_()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    it, res, _ = plan.bicgstab(b, x, tol=0.0, max_iter=steps, check_every=10)
    t1.record()
    torch.cuda.synchronize()
    it_ms = t0.elapsed_time(t1) / steps
    x.zero_()
    plan.profile_enable(True)
    plan.bicgstab(b, x, tol=0.0, max_iter=steps, check_every=10)
    launches, kernel_ms = plan.profile_read()
    plan.close()
    spmv_ms = kernel_ms / max(launches, 1)
    nnz = w["nnz"]
    return {"workload": f"rmat{scale}_sym_bicgstab", "dtype": "f64", "n": n, "nnz": int(nnz),
            "iterations": it, "ms_per_iteration": round(it_ms, 4),
            "spmv_us": round(spmv_ms * 1e3, 1),
            "spmv_share": round(2 * spmv_ms / it_ms, 3),
            "gnzs": round(2 * nnz / (it_ms * 1e-3) / 1e9, 3),
            "rel_residual": res, "stripes": stripes, "plan": plan_kw or "default", "seed": scale}


def measured_copy_gbs(mib: int = 1024, reps: int = 5) -> float:
    """Device-to-device copy bandwidth (read + write bytes / time), a measured
    second denominator beside the published HBM peak."""
    import torch
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * (mib << 20) / (ms * 1e-3) / 1e9


def run_adjoint(scale: int, iters: int, alpha: float, stripes: int = 0):
    """Differentiable PageRank on R-MAT (scale 20 by default), FP32: weights in
    (0.5, 1.5] column-normalised, loss ||pr(w) - t||^2.  Times the forward
    power method and the backward pass (adjoint fixed point on the transposed
    plan + per-nonzero value gradient + column-normalisation backward), both
    with `iters` iterations, and the transposed SpMV against the forward one."""
    import numpy as np
    import torch

    import graphgen
    import paper_2605_07391_amd.autograd as ag
    dev = torch.device("cuda:0")
    w = graphgen.workload(f"rmat{scale}")
    n, m = w["n_rows"], w["nnz"]
    r = torch.from_numpy(w["row_ptr"]).to(dev)
    c = torch.from_numpy(w["col"]).to(dev)
    op = ag.DiffPageRank(r, c, n, dtype=torch.float32, alpha=alpha, tol=0.0, max_iter=iters,
                         stripes=stripes)
    w0 = torch.from_numpy(graphgen.uniform(5, 83, m, 0.5, 1.5, closed_high=True)).float().to(dev)
    t0 = graphgen.uniform(6, 84, n, 0.0, 1.0)
    tgt = torch.from_numpy(t0 / t0.sum()).float().to(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def step():
        wt = w0.clone().requires_grad_(True)
        ev[0].record()
        x = op(wt)
        loss = ((x - tgt) ** 2).sum()
        ev[1].record()
        ev[2].record()
        loss.backward()
        ev[3].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3]), wt.grad

    step()
    fwd, bwd, grad = step()
    # kernel time of the forward and the transposed SpMV over one more step
    op.plan_fwd.profile_enable(True)
    op.plan_t.profile_enable(True)
    step()
    nf, tf = op.plan_fwd.profile_read()
    nt, tt = op.plan_t.profile_read()
    op.plan_fwd.profile_enable(False)
    op.plan_t.profile_enable(False)
    op.close()
    spmv_f = tf / max(nf, 1)
    spmv_t = tt / max(nt, 1)
    return {"workload": f"rmat{scale}_diff_pagerank", "dtype": "f32", "n": n, "nnz": int(m),
            "iterations": iters, "forward_ms": round(fwd, 3), "backward_ms": round(bwd, 3),
            "backward_vs_forward": round(bwd / fwd, 3),
            "forward_spmv_us": round(spmv_f * 1e3, 1),
            "transposed_spmv_us": round(spmv_t * 1e3, 1),
            "transposed_vs_forward_spmv": round(spmv_t / spmv_f, 3),
            "grad_finite": bool(torch.isfinite(grad).all().item()),
            "stripes": stripes, "seeds": {"graph": scale, "w": 5, "target": 6}}


def run_c1(steps: int, alpha: float):
    """PageRank on the 10,000-vertex Chung-Lu graph (FP32, 20 power
    iterations per call, x0 = 1/n; paper Sec. 5.5.1): the matrix is cache
    resident, so this reports time per iteration and per 20-iteration call
    (HIP graphs recorded before the clock), not a bandwidth fraction.  The
    plan takes the sigma and block size the autotuner measures fastest on
    this matrix."""
    import torch

    import graphgen
    import paper_2605_07391_amd as pkg
    dev = torch.device("cuda:0")
    w = graphgen.workload("chung_lu_10k")
    n = w["n_rows"]
    r = torch.from_numpy(w["row_ptr"]).to(dev)
    c = torch.from_numpy(w["col"]).to(dev)
    v = torch.from_numpy(w["values"]).float().to(dev)
    # sigma and block size by measurement on this matrix (the tuner's
    # candidates, untimed; the plan build is timed on its own below)
    best, table = pkg.tune(r, c, v, n, sigmas=list(range(2, 13)), block_lanes=[256, 512, 1024],
                           reps=20)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    plan = pkg.Plan(r, c, v, n, validate=False, sigma=best["sigma"],
                    block_lanes=best["block_lanes"])
    e1.record()
    torch.cuda.synchronize()
    plan_ms = e0.elapsed_time(e1)
    x = torch.empty(n, dtype=torch.float32, device=dev)
    iters = 20
    for _ in range(2):  # records the graphs of the timed call's chunks
        x.fill_(1.0 / n)
        plan.pagerank(x, alpha, tol=0.0, max_iter=iters)
    calls = max(1, steps)
    times = []
    g0 = plan.info()
    for _ in range(calls):
        x.fill_(1.0 / n)
        torch.cuda.synchronize()
        e0.record()
        plan.pagerank(x, alpha, tol=0.0, max_iter=iters)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    g1 = plan.info()
    mass = float(x.double().sum().item())
    x.fill_(1.0 / n)
    plan.profile_enable(True)
    plan.pagerank(x, alpha, tol=0.0, max_iter=iters)
    launches, kernel_ms = plan.profile_read()
    info = plan.info()
    plan.close()
    times.sort()
    med = times[len(times) // 2]
    return {"workload": "chung_lu_10k_pagerank", "dtype": "f32", "n": n, "nnz": int(w["nnz"]),
            "iterations_per_call": iters, "calls_timed": calls,
            "call_ms_median": round(med, 4), "call_ms_min": round(times[0], 4),
            "us_per_iteration": round(med * 1e3 / iters, 2),
            "spmv_us": round(kernel_ms * 1e3 / max(launches, 1), 2),
            "plan_ms": round(plan_ms, 3), "sigma": info["sigma"],
            "block_lanes": info["block_lanes"], "hot_columns": info["hot_columns"],
            "tuning_us_per_spmv": {f"s{a}_b{b}": round(t, 2) for (a, b), t in table.items()},
            "rank_mass": round(mass, 7),
            "graph_replays_in_timed_calls": g1["graph_replays"] - g0["graph_replays"],
            "graph_captures_in_timed_calls": g1["graph_captures"] - g0["graph_captures"],
            "seed": w["meta"]["seed"]}


# the FP64 stress matrix is measured at one fixed configuration (the one its
# full-size parity test checks): 64-bit descriptors, sigma 20, 512 lanes,
# 8 column stripes
STRESS_CONFIG = {"sigma": 20, "block_lanes": 512, "desc_bits": 64, "stripes": 8}


def run_stress(steps: int, warmup: int):
    """y = A x on the FP64 stress matrix (R-MAT scale 24, 30 % of rows empty,
    8 hub rows of 2,000,000 nonzeros; x in [-1, 1)): mean SpMV time from HIP
    events around every fused launch, against its algorithmic bytes."""
    import graphgen
    w = graphgen.workload("stress24")
    cfg = STRESS_CONFIG
    res = run_gpu(w, "f64", steps, warmup, cfg["sigma"], cfg["block_lanes"], 0.85, -1, "wave",
                  0, False, cfg["stripes"], cfg["desc_bits"])
    info = res["info"]
    ach = res["achieved_gbs"]
    return {"workload": "stress24_spmv", "dtype": "f64", "n": info["n_rows"],
            "nnz": info["nnz"], "steps": steps, "spmv_us": round(res["spmv_ms"] * 1e3, 2),
            "ms_per_step": round(res["step_ms"], 5), "spmv_gnzs": round(res["spmv_gnzs"], 3),
            "plan_ms": round(res["plan_ms"], 3), "plan": dict(cfg),
            "hot_columns": info["hot_columns"], "hot_coverage": round(info["hot_coverage"], 4),
            "fast_tile_fraction": round(info["fast_tiles"] / max(info["tile_num"], 1), 4),
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                         "traffic": load_traffic("stress24", "f64", info),
                         "kernel": kernel_instance(info)
                         + f" + merbit::stripe_combine_kernel<double, {info['stripes']}>",
                         "alg_bytes_per_launch": int(res["alg_bytes"]),
                         "mean_launch_us": round(res["spmv_ms"] * 1e3, 2),
                         "launches_timed": res["launches"]},
            "seeds": {"graph": w["meta"]["seed"], "x": w["meta"]["x_seed"]}}


def cpu_baseline(w, iters: int, alpha: float, dtype_name: str = "f32"):
    import numpy as np

    import oracle
    n = w["n_rows"]
    if w["meta"]["generator"] == "stress":
        t = time.perf_counter()
        for _ in range(iters):
            oracle.spmv(w["row_ptr"], w["col"], w["values"], w["x"])
        dt = time.perf_counter() - t
        return {"value": round(w["nnz"] * iters / dt / 1e9, 5), "unit": "GNZ/s", "cores": 1,
                "kind": "oracle",
                "sample": f"{iters} SpMVs of the full workload matrix "
                          f"(single-threaded C, long-double sums), {dt:.1f} s"}
    from oracle import cpu_baseline as cb
    vals = w["values"].astype(np.float32).astype(np.float64)
    x0 = np.full(n, np.float32(1.0 / n), np.float64)
    t = time.perf_counter()
    oracle.pagerank(w["row_ptr"], w["col"], vals, alpha, iters, x0)
    dt = time.perf_counter() - t
    # the timed variants: plain double sums, one thread and then every thread
    # OpenMP gives this process
    rows = []
    for threads in (1, 0):
        t = time.perf_counter()
        _, used = cb.pagerank(w["row_ptr"], w["col"], vals, alpha, iters, x0, threads)
        dtv = time.perf_counter() - t
        rows.append({"value": round(w["nnz"] * iters / dtv / 1e9, 5), "unit": "GNZ/s",
                     "cores": used, "kind": "plain_f64" + ("_openmp" if used > 1 else ""),
                     "sample": f"{iters} PageRank iterations of the full workload matrix "
                               f"({used} thread{'s' if used > 1 else ''}, double sums), "
                               f"{dtv:.2f} s"})
    return {"value": round(w["nnz"] * iters / dt / 1e9, 5), "unit": "GNZ/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{iters} PageRank iterations of the full workload matrix "
                      f"(single-threaded C, long-double sums), {dt:.1f} s",
            "rows": rows, "cpu_model": cb.cpu_model(), "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20,
                    help="untimed PageRank iterations first (20 = two chunks between "
                         "convergence checks, so both HIP graphs of the loop are recorded)")
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--sigma", type=int, default=0,
                    help="steps per lane; 0 = chosen by the autotuner (with --block-lanes 0)")
    ap.add_argument("--block-lanes", type=int, default=0)
    ap.add_argument("--hot-columns", type=int, default=-1,
                    help="LDS x cache size in columns: -1 automatic, 0 off")
    ap.add_argument("--commit", default="auto", choices=["auto", "block", "wave"])
    ap.add_argument("--desc-bits", type=int, default=32, choices=[32, 64])
    ap.add_argument("--stripes", type=int, default=-1,
                    help="column stripes: -1 = the autotuner also tries 8, 0 = none, S = S")
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--alpha", type=float, default=0.85)
    ap.add_argument("--cpu-iters", type=int, default=15)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 companion run")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched runs (64-source PPR, 256 graphs)")
    ap.add_argument("--no-multi", action="store_true",
                    help="skip the 256-graph block of the batched runs (keep the 64-source PPR)")
    ap.add_argument("--batched-steps", type=int, default=10)
    ap.add_argument("--spmm-sigma", type=int, default=0,
                    help="sigma of the 64-source PPR's SpMM instead of tuning it (4..12)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the differentiable-PageRank run (R-MAT scale 20)")
    ap.add_argument("--adjoint-scale", type=int, default=20)
    ap.add_argument("--no-bicgstab", action="store_true",
                    help="skip the BiCGSTAB run on the symmetric 0/1 R-MAT system")
    ap.add_argument("--bicgstab-scale", type=int, default=21)
    ap.add_argument("--no-c1", action="store_true",
                    help="skip the 10,000-vertex Chung-Lu PageRank timing")
    ap.add_argument("--no-stress", action="store_true",
                    help="skip the FP64 stress-matrix SpMV (R-MAT scale 24 with hub rows)")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the default sigma / block size instead of the autotuner")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (5 times), used to "
                         "scale rocprofv3 FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--traffic-record", nargs=5,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR", "OUT"),
                    help="only build the plan of the given configuration and write its HBM "
                         "traffic record from four rocprofv3 --pmc output directories")
    args = ap.parse_args()
    if args.traffic_record:
        import torch

        import graphgen
        import paper_2605_07391_amd as pkg
        w = graphgen.workload(args.workload)
        dt = torch.float32 if args.dtype == "f32" else torch.float64
        dev = torch.device("cuda:0")
        plan = pkg.Plan(torch.from_numpy(w["row_ptr"]).to(dev), torch.from_numpy(w["col"]).to(dev),
                        torch.from_numpy(w["values"]).to(dt).to(dev), w["n_rows"],
                        sigma=args.sigma, block_lanes=args.block_lanes, commit=args.commit,
                        hot_columns=args.hot_columns, stripes=max(args.stripes, 0),
                        desc_bits=args.desc_bits, validate=False)
        info = plan.info()
        plan.close()
        rec = traffic_record(args.workload, args.dtype, info,
                             algorithmic_bytes(info, 4 if args.dtype == "f32" else 8),
                             *args.traffic_record[:4])
        with open(args.traffic_record[4], "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec), flush=True)
        return
    if args.copy_calibration_mib > 0:
        import torch
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 5}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import graphgen
    t = time.perf_counter()
    w = graphgen.workload(args.workload)
    gen_s = time.perf_counter() - t
    print(f"[bench] workload {args.workload}: n={w['n_rows']} nnz={w['nnz']} "
          f"generated in {gen_s:.1f}s", file=sys.stderr, flush=True)

    tune = not args.no_tune and args.sigma == 0 and args.block_lanes == 0
    main_run = run_gpu(w, args.dtype, args.steps, args.warmup, args.sigma, args.block_lanes,
                       args.alpha, args.hot_columns, args.commit, args.blocks_per_cu, tune,
                       args.stripes, args.desc_bits)
    info = main_run["info"]
    print(f"[bench] {args.dtype}: step {main_run['step_ms'] * 1e3:.1f} us, spmv "
          f"{main_run['spmv_ms'] * 1e3:.1f} us", file=sys.stderr, flush=True)
    extra = None
    if not args.no_f64 and args.dtype == "f32" and w["meta"]["generator"] != "stress":
        r64 = run_gpu(w, "f64", args.steps, args.warmup, 0, args.block_lanes, args.alpha,
                      args.hot_columns, args.commit, args.blocks_per_cu, tune, args.stripes,
                      args.desc_bits)
        extra = {
            "value": round(r64["value_gnzs"], 3), "ms_per_step": round(r64["step_ms"], 5),
            "spmv_us": round(r64["spmv_ms"] * 1e3, 2), "spmv_gnzs": round(r64["spmv_gnzs"], 3),
            "achieved_gbs": round(r64["achieved_gbs"], 1),
            "pct_hbm_peak": round(100 * r64["achieved_gbs"] / HBM_PEAK_GBS, 2),
            "plan_ms": round(r64["plan_ms"], 3), "sigma": r64["info"]["sigma"],
            "hot_columns": r64["info"]["hot_columns"],
            "hot_coverage": round(r64["info"]["hot_coverage"], 4),
            "traffic": load_traffic(args.workload, "f64", r64["info"]),
            "stripes": r64["info"]["stripes"], "desc_bits": r64["info"]["desc_bits"],
            "block_lanes": r64["info"]["block_lanes"],
            "commit": {1: "block", 2: "wave"}[r64["info"]["commit"]], "tuning": r64["tuning"],
            "alg_bytes_per_launch": int(r64["alg_bytes"]), "timed_graphs": r64["graphs"],
        }
        print(f"[bench] f64: step {r64['step_ms'] * 1e3:.1f} us, spmv "
              f"{r64['spmv_ms'] * 1e3:.1f} us", file=sys.stderr, flush=True)
    batched = None
    if not args.no_batched and w["meta"]["generator"] == "rmat":
        ppr = run_ppr(w, 64, args.batched_steps, 2, args.alpha, sigma=args.spmm_sigma)
        ppr["vs_plain_spmv"] = round(ppr["gnz_rhs_per_s"] / main_run["spmv_gnzs"], 3)
        print(f"[bench] ppr64: step {ppr['ms_per_step']:.3f} ms, spmm {ppr['spmm_us']:.1f} us",
              file=sys.stderr, flush=True)
        batched = {"ppr64_" + args.workload + "_f32": ppr}
        if not args.no_multi:
            # the striped plan of the 256 graphs is tuned on its own matrix
            multi = run_multi(args.batched_steps, 2, args.alpha, stripes=8, tune=True)
            multi_plain = run_multi(args.batched_steps, 2, args.alpha)
            multi["one_plan_without_stripes"] = {k: multi_plain[k] for k in
                                                 ("ms_per_step", "spmv_us", "gnzs",
                                                  "spmv_gnzs")}
            multi["vs_plain"] = round(multi["gnzs"] / main_run["value_gnzs"], 3)
            print(f"[bench] multi256: step {multi['ms_per_step']:.3f} ms", file=sys.stderr,
                  flush=True)
            batched["chung_lu_multi256_f32"] = multi
    adj = None
    if not args.no_adjoint and w["meta"]["generator"] == "rmat":
        adj = run_adjoint(args.adjoint_scale, 50, args.alpha, stripes=8)
        adj_plain = run_adjoint(args.adjoint_scale, 50, args.alpha)
        adj["one_plan_without_stripes"] = {k: adj_plain[k] for k in
                                           ("forward_ms", "backward_ms", "forward_spmv_us",
                                            "transposed_spmv_us")}
        print(f"[bench] adjoint: forward {adj['forward_ms']:.2f} ms, backward "
              f"{adj['backward_ms']:.2f} ms", file=sys.stderr, flush=True)
    bicg = None
    if not args.no_bicgstab and w["meta"]["generator"] == "rmat":
        bicg = run_bicgstab(args.bicgstab_scale, args.batched_steps * 10, stripes=8,
                            plan_kw=tuned_kw(r64["info"]) if extra is not None else None)
        bicg_plain = run_bicgstab(args.bicgstab_scale, args.batched_steps * 10)
        bicg["one_plan_without_stripes"] = {k: bicg_plain[k] for k in
                                            ("ms_per_iteration", "spmv_us", "spmv_share", "gnzs")}
        print(f"[bench] bicgstab: {bicg['ms_per_iteration']:.3f} ms / iteration", file=sys.stderr,
              flush=True)
    c1 = None
    if not args.no_c1 and w["meta"]["generator"] == "rmat":
        c1 = run_c1(5, args.alpha)
        print(f"[bench] chung_lu_10k: {c1['us_per_iteration']:.1f} us / iteration",
              file=sys.stderr, flush=True)
    stress = None
    if not args.no_stress and w["meta"]["generator"] == "rmat":
        stress = run_stress(args.steps, args.warmup)
        print(f"[bench] stress24 f64: spmv {stress['spmv_us']:.1f} us "
              f"({100 * stress['roofline']['frac']:.1f} % of 8 TB/s)", file=sys.stderr,
              flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_iters, args.alpha, args.dtype)
    ach = main_run["achieved_gbs"]
    copy_gbs = measured_copy_gbs()
    out = {
        "metric": METRIC,
        "value": round(main_run["value_gnzs"], 3),
        "unit": "GNZ/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["step_ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": ("synthetic (seeded R-MAT, values 1/outdeg)"
                 if w["meta"]["generator"] != "stress" else
                 "synthetic (seeded R-MAT scale 24, 30% rows cleared, 8 hub rows of 2M nnz, "
                 "values in (0,1], x in [-1,1))"),
        "config": {"workload": (f"{args.workload}_pagerank" if w["meta"]["generator"] != "stress"
                                else f"{args.workload}_spmv"), "n": info["n_rows"],
                   "nnz": info["nnz"], "sigma": info["sigma"],
                   "block_lanes": info["block_lanes"],
                   "commit": {1: "block", 2: "wave"}[info["commit"]],
                   "hot_columns": info["hot_columns"],
                   "hot_coverage": round(info["hot_coverage"], 4), "grid": info["grid"],
                   "stripes": info["stripes"], "ranges": info["ranges"],
                   "desc_bits": info["desc_bits"],
                   "plan_rows": info["plan_rows"],
                   "alpha": args.alpha,
                   "seed": w["meta"].get("seed"), "x0": "1/n"},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic(args.workload, args.dtype, info),
                     "kernel": kernel_instance(info) + (
                         f" + merbit::stripe_combine_kernel<{'float' if info['dtype'] == 0 else 'double'}, "
                         f"{info['stripes']}>" if info["stripes"] > 1 else ""),
                     "alg_bytes_per_launch": int(main_run["alg_bytes"]),
                     "mean_launch_us": round(main_run["spmv_ms"] * 1e3, 2),
                     "measured_copy_gbs": round(copy_gbs, 1),
                     "frac_of_measured_copy": round(ach / copy_gbs, 4),
                     "launches_timed": main_run["launches"]},
        "cpu_baseline": cpu,
        "spmv_gnzs": round(main_run["spmv_gnzs"], 3),
        "plan_ms": round(main_run["plan_ms"], 3),
        "fast_tile_fraction": round(info["fast_tiles"] / max(info["tile_num"], 1), 4),
        "rank_mass": None if main_run["mass"] is None else round(main_run["mass"], 7),
        "timed_graphs": main_run["graphs"],
        "tuning": main_run["tuning"],
        "f64": extra,
        "batched": batched,
        "bicgstab": bicg,
        "adjoint": adj,
        "chung_lu_10k": c1,
        "stress24_f64": stress,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
