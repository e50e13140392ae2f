"""GPU parity of the adjoint pieces (transpose, per-nonzero products,
gathers, column scaling, adjoint fixed point) against the oracle, and of the
differentiable PageRank's gradients against finite differences and the FP64
oracle gradient."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from helpers import (OMEGA, SPMV_TOL, case_matrix, check_spmv, host_values, require_gpu,
                     spmv_cases, to_device, workload)

pytestmark = pytest.mark.gpu

DTYPES = [torch.float32, torch.float64]
CASES = spmv_cases()
ALPHA = 0.85
ADJ_TOL = {torch.float32: 1e-4, torch.float64: 1e-11}


def _np(dtype):
    return np.float32 if dtype == torch.float32 else np.float64


@pytest.mark.parametrize("sigma", [3, 12])
@pytest.mark.parametrize("name", list(CASES))
def test_transpose_bit_exact(name, sigma):
    """rowT_ptr, colT and perm equal the oracle's stable transpose; the plan
    of the transpose is bit exact and its SpMV is A^T g."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, vals, nc = case_matrix(CASES, name, seed=sigma)
    r, c, v = to_device(rp, col, vals, torch.float64, dev)
    plan = pkg.Plan(r, c, v, nc, sigma=sigma)
    rt, ct, perm = plan.transpose()
    ort, oct_, operm = oracle.transpose(nc, rp, col)
    assert np.array_equal(rt.cpu().numpy(), ort)
    assert np.array_equal(ct.cpu().numpy(), oct_)
    assert np.array_equal(perm.cpu().numpy(), operm)
    vt = pkg.gather_values(perm, v)
    assert np.array_equal(vt.cpu().numpy(), vals[operm])
    plan_t = pkg.Plan(rt, ct, vt, len(rp) - 1, sigma=sigma)
    tx, ty, ld = plan_t.export()
    ox, oy, od = oracle.plan(ort, OMEGA, sigma)
    assert np.array_equal(tx, ox) and np.array_equal(ty, oy) and np.array_equal(ld, od)
    g64 = graphgen.uniform(5, 79, len(rp) - 1, -1.0, 1.0)
    y = plan_t.spmv(torch.from_numpy(g64).to(dev))
    torch.cuda.synchronize()
    check_spmv(y, ort, oct_, vals[operm], g64, torch.float64, f"{name} A^T g")
    plan.close()
    plan_t.close()


@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
@pytest.mark.parametrize("name", ["random1_700x300", "single_long_row", "long_then_empty",
                                  "chung_lu_10k", "all_rows_empty", "one_column"])
def test_sddmm_gather_column_scale(name, dtype):
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    rp, col, vals, nc = case_matrix(CASES, name, seed=1)
    n = len(rp) - 1
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, nc, sigma=7)
    g = graphgen.uniform(6, 80, n, -1.0, 1.0).astype(_np(dtype)).astype(np.float64)
    x = graphgen.uniform(7, 81, nc, -1.0, 1.0).astype(_np(dtype)).astype(np.float64)
    out = plan.sddmm(torch.from_numpy(g).to(dtype).to(dev), torch.from_numpy(x).to(dtype).to(dev),
                     0.85)
    ref = oracle.pagerank_value_grad(rp, col, g, x, 0.85)
    got = out.double().cpu().numpy()
    eps = 2.5e-7 if dtype == torch.float32 else 5e-16
    assert np.all(np.abs(got - ref) <= 3 * eps * np.abs(ref))
    if len(col):
        # gather with a product, column scaling (with and without t)
        perm = torch.from_numpy(oracle.transpose(nc, rp, col)[2]).to(dev)
        a = torch.from_numpy(vals).to(dtype).to(dev)
        b = torch.from_numpy(vals[::-1].copy()).to(dtype).to(dev)
        gv = pkg.gather_values(perm, a, b).double().cpu().numpy()
        ah, bh = host_values(vals, dtype), host_values(vals[::-1].copy(), dtype)
        pm = perm.cpu().numpy()
        assert np.all(np.abs(gv - ah[pm] * bh[pm]) <= eps * np.abs(ah[pm] * bh[pm]))
        s = torch.from_numpy(1.5 + x).to(dtype).to(dev)
        t = torch.from_numpy(x[::-1].copy()).to(dtype).to(dev)
        sh, th = (1.5 + x).astype(_np(dtype)).astype(np.float64), host_values(x[::-1].copy(), dtype)
        cs = pkg.column_scale(c, a, s).double().cpu().numpy()
        assert np.all(np.abs(cs - ah / sh[col]) <= 2 * eps * np.abs(ah / sh[col]))
        cs2 = pkg.column_scale(c, a, s, t).double().cpu().numpy()
        ref2 = (ah - th[col]) / sh[col]
        assert np.all(np.abs(cs2 - ref2) <= 4 * eps * (np.abs(ah) + np.abs(th[col])) / sh[col])
    plan.close()


def _diff_setup(w, dtype, dev, **kw):
    import paper_2605_07391_amd.autograd as ag
    rp, col, n = w["row_ptr"], w["col"], w["n_rows"]
    r = torch.from_numpy(np.ascontiguousarray(rp, np.int32)).to(dev)
    c = torch.from_numpy(np.ascontiguousarray(col, np.int32)).to(dev)
    return ag.DiffPageRank(r, c, n, dtype=dtype, **kw)


@pytest.mark.parametrize("stripes", [0, 8])
@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_adjoint_fixed_point_chung_lu(dtype, stripes):
    """20 adjoint iterations against the oracle's, normwise (P^T on a plain
    and on a column-stripe plan)."""
    dev = require_gpu()
    w = workload("chung_lu_10k")
    rp, col, vals, n = w["row_ptr"], w["col"], w["values"], w["n_rows"]
    op = _diff_setup(w, dtype, dev, stripes=stripes)
    assert op.plan_t.info()["stripes"] == max(stripes, 1)
    vh = host_values(vals, dtype)
    P = torch.from_numpy(vh).to(dtype).to(dev)
    import paper_2605_07391_amd as pkg
    pkg.gather_values(op.perm, P, out=op.values_t)
    op.refresh_transpose_values()
    g64 = graphgen.uniform(8, 82, n, -1.0, 1.0).astype(_np(dtype)).astype(np.float64)
    g = torch.from_numpy(g64).to(dtype).to(dev)
    for iters in (1, 7, 20):
        lam = g.clone()
        it, res, _ = op.plan.pagerank_adjoint(op.plan_t, g, lam, ALPHA, 0.0, iters, 10)
        torch.cuda.synchronize()
        assert it == iters
        ref = oracle.pagerank_adjoint(rp, col, vh, ALPHA, iters, g64)
        err = np.abs(lam.double().cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err <= ADJ_TOL[dtype], f"{iters} iterations: {err:.3e}"
    lam = g.clone()
    it, res, conv = op.plan.pagerank_adjoint(op.plan_t, g, lam, ALPHA,
                                             1e-3 if dtype == torch.float32 else 1e-10, 500, 5)
    assert conv and it % 5 == 0
    op.close()


@pytest.mark.parametrize("stripes", [0, 8], ids=["plain", "striped8"])
@pytest.mark.parametrize("dtype", DTYPES, ids=["f32", "f64"])
def test_adjoint_partial_hot_cache(dtype, stripes):
    """P^T's plan with a partial hot-column cache: the adjoint update writes
    the next SpMV's hot values, and only each call's first chunk gathers them
    (a graph of its own).  Chunks of 4 iterations are recorded and replayed
    over repeated calls, each result against the oracle."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    w = workload("chung_lu_10k")
    rp, col, vals, n = w["row_ptr"], w["col"], w["values"], w["n_rows"]
    op = _diff_setup(w, dtype, dev)
    vh = host_values(vals, dtype)
    P = torch.from_numpy(vh).to(dtype).to(dev)
    pkg.gather_values(op.perm, P, out=op.values_t)
    pt = pkg.Plan(op.row_t, op.col_t, op.values_t, n, commit="wave", hot_columns=100,
                  stripes=stripes)
    info = pt.info()
    assert 0 < info["hot_columns"] < n and info["hot_coverage"] < 1.0
    g64 = graphgen.uniform(8, 83, n, -1.0, 1.0).astype(_np(dtype)).astype(np.float64)
    g = torch.from_numpy(g64).to(dtype).to(dev)
    for iters in (12, 9, 12, 12):
        lam = g.clone()
        it, _, _ = op.plan.pagerank_adjoint(pt, g, lam, ALPHA, 0.0, iters, 4)
        y = pt.spmv(g)  # eager work on the same plan (its own hot gather) between calls
        torch.cuda.synchronize()
        assert it == iters and torch.isfinite(y).all()
        ref = oracle.pagerank_adjoint(rp, col, vh, ALPHA, iters, g64)
        err = np.abs(lam.double().cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err <= ADJ_TOL[dtype], f"{iters} iterations: {err:.3e}"
    pt.close()
    op.close()


def _tiny_graph(n, seed):
    rng = np.random.default_rng(seed)
    edges = {(int(rng.integers(n)), int(rng.integers(n))) for _ in range(3 * n)}
    edges = sorted({(u, v) for u, v in edges if u != n - 1}, key=lambda e: (e[1], e[0]))
    rp = np.zeros(n + 1, np.int64)
    for _, v in edges:
        rp[v + 1] += 1
    rp = np.cumsum(rp).astype(np.int32)
    col = np.array([u for u, _ in edges], np.int32)
    return {"row_ptr": rp, "col": col, "n_rows": n}


@pytest.mark.parametrize("seed", [1, 2])
def test_gradcheck_fp64(seed):
    """torch.autograd.gradcheck of w -> x*(colnorm(w)) in FP64 (converged
    forward and adjoint), on a tiny graph with a dangling vertex."""
    dev = require_gpu()
    g = _tiny_graph(12, seed)
    op = _diff_setup(g, torch.float64, dev, max_iter=260, check_every=20)
    w0 = 1.5 - np.random.default_rng(seed).random(len(g["col"]))
    w = torch.tensor(w0, dtype=torch.float64, device=dev, requires_grad=True)
    assert torch.autograd.gradcheck(lambda t: op(t), (w,), eps=1e-6, atol=1e-8, rtol=1e-5)
    op.close()


@pytest.mark.parametrize("stripes", [0, 4])
@pytest.mark.parametrize("seed", [3, 4])
def test_loss_gradient_vs_oracle_small(seed, stripes):
    """FP64 gradient of ||x* - t||^2 equals the oracle's adjoint gradient
    (also with the forward and adjoint iterations on column-stripe plans)."""
    dev = require_gpu()
    g = _tiny_graph(40, seed)
    rng = np.random.default_rng(seed)
    w0 = 1.5 - rng.random(len(g["col"]))
    tgt = rng.dirichlet(np.ones(40))
    op = _diff_setup(g, torch.float64, dev, max_iter=300, check_every=20, stripes=stripes)
    w = torch.tensor(w0, dtype=torch.float64, device=dev, requires_grad=True)
    x = op(w)
    loss = ((x - torch.from_numpy(tgt).to(dev)) ** 2).sum()
    loss.backward()
    L, grad, _, _ = oracle.pagerank_loss_grad(g["row_ptr"], g["col"], w0, tgt, ALPHA, 300)
    assert abs(loss.item() - L) <= 1e-13 * L
    assert np.abs(w.grad.cpu().numpy() - grad).max() <= 1e-10 * np.abs(grad).max()
    op.close()


def test_rmat20_fp32_gradient_vs_fp64_oracle_and_finite_differences():
    """Differentiable PageRank at R-MAT scale 20 (weights (0.5, 1.5], column
    normalised, loss ||pr(w) - t||^2): the FP32 GPU gradient against the FP64
    oracle gradient (normwise 1e-3), and the FP64 GPU gradient against central
    finite differences of the FP64 GPU forward on 100 seeded edges."""
    dev = require_gpu()
    w = workload("rmat20")
    n, m = w["n_rows"], w["nnz"]
    w0 = graphgen.uniform(5, 83, m, 0.5, 1.5, closed_high=True)
    t0 = graphgen.uniform(6, 84, n, 0.0, 1.0)
    tgt = t0 / t0.sum()
    _, grad_ref, _, _ = oracle.pagerank_loss_grad(w["row_ptr"], w["col"], w0, tgt, ALPHA, 120)
    tg = torch.from_numpy(tgt)
    grads = {}
    for dtype in DTYPES:
        op = _diff_setup(w, dtype, dev, tol=1e-7 if dtype == torch.float32 else 1e-15,
                         max_iter=400, check_every=10)
        wt = torch.from_numpy(w0).to(dtype).to(dev).requires_grad_(True)
        x = op(wt)
        loss = ((x.double() - tg.to(dev)) ** 2).sum()
        loss.backward()
        grads[dtype] = (op, wt.grad.double().cpu().numpy())
    g32 = grads[torch.float32][1]
    err = np.linalg.norm(g32 - grad_ref) / np.linalg.norm(grad_ref)
    assert err <= 1e-3, err
    # the same FP32 gradient with the forward and adjoint iterations on
    # column-stripe plans (8 stripes)
    ops = _diff_setup(w, torch.float32, dev, tol=1e-7, max_iter=400, check_every=10, stripes=8)
    wt = torch.from_numpy(w0).float().to(dev).requires_grad_(True)
    x = ops(wt)
    ((x.double() - tg.to(dev)) ** 2).sum().backward()
    gs = wt.grad.double().cpu().numpy()
    assert np.linalg.norm(gs - grad_ref) / np.linalg.norm(grad_ref) <= 1e-3
    ops.close()
    op64, g64 = grads[torch.float64]
    assert np.linalg.norm(g64 - grad_ref) / np.linalg.norm(grad_ref) <= 1e-6
    edges = np.random.default_rng(7).choice(m, 100, replace=False)
    base = torch.from_numpy(w0).to(dev)
    scale = np.abs(g64).max()
    with torch.no_grad():
        for e in edges:
            h = 1e-3 * w0[e]
            vals = []
            for sgn in (1, -1):
                wp = base.clone()
                wp[e] += sgn * h
                x = op64(wp)
                vals.append(float(((x - tg.to(dev)) ** 2).sum().item()))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - g64[e]) <= 1e-4 * scale + 1e-3 * abs(g64[e]), (e, fd, g64[e])
    for op, _ in grads.values():
        op.close()


@pytest.mark.parametrize("stripes", [0, 8])
def test_training_steps_replay_the_recorded_graphs(stripes):
    """Five gradient steps on the Chung-Lu graph: the forward power method and
    the adjoint fixed point record their iteration-chunk HIP graphs in the
    first step only and replay them afterwards, and every step's gradient
    matches a fresh DiffPageRank (no graphs kept) on the same weights."""
    dev = require_gpu()
    g = workload("chung_lu_10k")
    n, m = g["n_rows"], len(g["col"])
    op = _diff_setup(g, torch.float32, dev, max_iter=20, check_every=10, stripes=stripes)
    rng = np.random.default_rng(11)
    w = torch.tensor(0.5 + rng.random(m), dtype=torch.float32, device=dev, requires_grad=True)
    tgt = torch.from_numpy(rng.dirichlet(np.ones(n))).float().to(dev)
    # forward graphs live on the forward plan, adjoint graphs on the plan of P^T
    plans = [op.plan_fwd, op.plan_t]
    captures, replays = [], []
    for step in range(5):
        x = op(w)
        loss = ((x - tgt) ** 2).sum()
        loss.backward()
        grad = w.grad.detach().clone()
        ref_op = _diff_setup(g, torch.float32, dev, max_iter=20, check_every=10, stripes=stripes)
        w_ref = w.detach().clone().requires_grad_(True)
        ((ref_op(w_ref) - tgt) ** 2).sum().backward()
        ref_op.close()
        scale = w_ref.grad.abs().max().item()
        assert (grad - w_ref.grad).abs().max().item() <= 1e-4 * scale, f"step {step}"
        captures.append([p.info()["graph_captures"] for p in plans])
        replays.append([p.info()["graph_replays"] for p in plans])
        with torch.no_grad():
            w -= 2e3 * w.grad
            w.clamp_(min=0.1)
        w.grad = None
    assert all(c == captures[0] for c in captures[1:]), captures
    assert all(r1 > r0 for r0, r1 in zip(replays[0], replays[-1])), replays
    op.close()
