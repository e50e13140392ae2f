"""Pins for the oracle's PageRank power method (Sec. 5.5.1, damping 0.85,
dangling mass spread uniformly).

Checked against: a dense direct solve of the stationary equation (numpy's
LU solver), closed-form stationary vectors (cycle, complete digraph, alpha = 0,
no edges), probability-mass conservation, stationarity and the contraction
bound ||x_t - x*||_1 <= alpha^t ||x_0 - x*||_1.
"""
import numpy as np
import pytest

import graphgen
import oracle

ALPHA = 0.85


def _pr_matrix(n, edges):
    """CSR of the column-stochastic P (rows = destinations) from u->v edges."""
    edges = sorted(set(edges), key=lambda e: (e[1], e[0]))
    outdeg = np.zeros(n)
    for u, v in edges:
        outdeg[u] += 1
    rp = np.zeros(n + 1, np.int32)
    for u, v in edges:
        rp[v + 1] += 1
    rp = np.cumsum(rp).astype(np.int32)
    col = np.array([u for u, v in edges], np.int32)
    vals = np.array([1.0 / outdeg[u] for u, v in edges])
    return rp, col, vals


def _dense_stationary(n, rp, col, vals, alpha):
    P = np.zeros((n, n))
    for r in range(n):
        for k in range(rp[r], rp[r + 1]):
            P[r, col[k]] += vals[k]
    dangling = np.bincount(col, minlength=n) == 0
    M = np.eye(n) - alpha * P - (alpha / n) * np.outer(np.ones(n), dangling.astype(float))
    return np.linalg.solve(M, np.full(n, (1 - alpha) / n))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_dense_direct_solve(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 40))
    edges = [(int(rng.integers(n)), int(rng.integers(n))) for _ in range(3 * n)]
    rp, col, vals = _pr_matrix(n, edges)
    x_star = _dense_stationary(n, rp, col, vals, ALPHA)
    x, resid, _ = oracle.pagerank(rp, col, vals, ALPHA, 300, np.full(n, 1.0 / n))
    assert np.all(np.abs(x - x_star) <= 1e-13 * x_star)
    assert abs(x.sum() - 1.0) < 1e-14


def test_closed_forms():
    n = 17
    x0 = np.random.default_rng(0).dirichlet(np.ones(n))
    # directed cycle: P is a permutation, the stationary vector is uniform
    rp, col, vals = _pr_matrix(n, [(i, (i + 1) % n) for i in range(n)])
    x, _, _ = oracle.pagerank(rp, col, vals, ALPHA, 400, x0)
    assert np.allclose(x, 1.0 / n, rtol=1e-14, atol=0)
    # complete digraph with self-loops: uniform after one step from uniform
    rp, col, vals = _pr_matrix(n, [(u, v) for u in range(n) for v in range(n)])
    x, _, _ = oracle.pagerank(rp, col, vals, ALPHA, 1, np.full(n, 1.0 / n))
    assert np.allclose(x, 1.0 / n, rtol=1e-15, atol=0)
    # alpha = 0: pure teleport
    rp, col, vals = _pr_matrix(n, [(0, 1), (1, 2), (2, 0), (3, 0)])
    x, _, _ = oracle.pagerank(rp, col, vals, 0.0, 1, x0)
    assert np.allclose(x, 1.0 / n, rtol=1e-15, atol=0)
    # no edges at all: every vertex dangling, uniform after one step
    rp = np.zeros(n + 1, np.int32)
    x, _, _ = oracle.pagerank(rp, np.zeros(0, np.int32), np.zeros(0), ALPHA, 1, x0)
    assert np.allclose(x, 1.0 / n, rtol=1e-15, atol=0)


def test_mass_stationarity_contraction_on_chung_lu():
    w = graphgen.workload("chung_lu_10k")
    n = w["n_rows"]
    rp, col, vals = w["row_ptr"], w["col"], w["values"]
    assert (np.bincount(col, minlength=n) == 0).any()  # has dangling vertices
    x0 = np.full(n, 1.0 / n)
    x_star, _, _ = oracle.pagerank(rp, col, vals, ALPHA, 230, x0)
    x20, resid, hist = oracle.pagerank(rp, col, vals, ALPHA, 20, x0, history=True)
    for t in range(20):
        xt = hist[t]
        assert abs(xt.sum() - 1.0) < 1e-12
        assert np.abs(xt - x_star).sum() <= ALPHA ** (t + 1) * np.abs(x0 - x_star).sum() + 1e-15
        prev = x0 if t == 0 else hist[t - 1]
        assert abs(resid[t] - np.abs(xt - prev).sum()) <= 1e-15
    assert np.array_equal(x20, hist[19])
    # stationarity of the converged vector: one more step moves it < 1e-14
    x_next, r1, _ = oracle.pagerank(rp, col, vals, ALPHA, 1, x_star)
    assert r1[0] < 1e-14
    assert np.all(x_star > 0)
