"""Pins for the oracle's batched forms: multi-vector SpMV, PageRank with a
general teleport vector (personalised PageRank), and PageRank of many graphs
stored on the diagonal of one matrix.

Independent checks: dense brute force, a dense direct solve of the teleport
stationary equation, closed forms, mass conservation, and the block
structure of a block-diagonal matrix.
"""
import numpy as np
import pytest

import graphgen
import oracle

ALPHA = 0.85


def _dense(row_ptr, col, vals, n_cols):
    n = len(row_ptr) - 1
    A = np.zeros((n, n_cols))
    for r in range(n):
        for k in range(row_ptr[r], row_ptr[r + 1]):
            A[r, col[k]] += vals[k]
    return A


@pytest.mark.parametrize("k", [1, 3, 64])
@pytest.mark.parametrize("seed", [0, 1])
def test_spmm_dense_bruteforce(k, seed):
    rp, col, vals = graphgen.random_csr(37, 29, 0.2, seed, empty_frac=0.3, long_rows=(5,))
    X = np.random.default_rng(seed + 9).uniform(-1, 1, (29, k))
    Y = oracle.spmm(rp, col, vals, X)
    A = _dense(rp, col, vals, 29)
    assert Y.shape == (37, k)
    assert np.all(np.abs(Y - A @ X) <= 1e-14 * (np.abs(A) @ np.abs(X)) + 1e-300)
    assert np.all(Y[np.diff(rp) == 0] == 0.0)


def _pr_matrix(n, edges):
    edges = sorted(set(edges), key=lambda e: (e[1], e[0]))
    outdeg = np.zeros(n)
    for u, _ in edges:
        outdeg[u] += 1
    rp = np.zeros(n + 1, np.int64)
    for _, v in edges:
        rp[v + 1] += 1
    rp = np.cumsum(rp).astype(np.int32)
    col = np.array([u for u, _ in edges], np.int32)
    vals = np.array([1.0 / outdeg[u] for u, _ in edges])
    return rp, col, vals


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_teleport_dense_direct_solve(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(6, 30))
    rp, col, vals = _pr_matrix(n, [(int(rng.integers(n)), int(rng.integers(n)))
                                   for _ in range(2 * n)])
    P = _dense(rp, col, vals, n)
    dangling = (np.bincount(col, minlength=n) == 0).astype(float)
    v = rng.dirichlet(np.ones(n))
    M = np.eye(n) - ALPHA * P - ALPHA * np.outer(v, dangling)
    x_star = np.linalg.solve(M, (1 - ALPHA) * v)
    x, resid = oracle.pagerank_teleport(rp, col, vals, ALPHA, 300, v, v)
    assert np.all(np.abs(x - x_star) <= 1e-13 * np.maximum(x_star, 1e-300) + 1e-15)
    assert abs(x.sum() - 1.0) < 1e-14
    # personalised: every source column satisfies the same equation with v = e_s
    s = int(rng.integers(n))
    e = np.zeros(n)
    e[s] = 1.0
    xs = oracle.personalized_pagerank(rp, col, vals, ALPHA, 300, [s])[:, 0]
    xe = np.linalg.solve(np.eye(n) - ALPHA * P - ALPHA * np.outer(e, dangling), (1 - ALPHA) * e)
    assert np.allclose(xs, xe, rtol=1e-12, atol=1e-15)
    assert abs(xs.sum() - 1.0) < 1e-14


def test_teleport_closed_forms():
    n = 11
    # no edges: all mass is dangling and returns to the source in one step
    rp = np.zeros(n + 1, np.int32)
    X = oracle.personalized_pagerank(rp, np.zeros(0, np.int32), np.zeros(0), ALPHA, 1, [3, 7])
    assert X[3, 0] == 1.0 and X[7, 1] == 1.0 and X.sum() == 2.0
    # a uniform teleport vector is the plain PageRank of Sec. 5.5.1
    w = graphgen.workload("chung_lu_10k")
    m = w["n_rows"]
    v = np.full(m, 1.0 / m)
    a, _ = oracle.pagerank_teleport(w["row_ptr"], w["col"], w["values"], ALPHA, 15, v, v)
    b, _, _ = oracle.pagerank(w["row_ptr"], w["col"], w["values"], ALPHA, 15, v)
    assert np.allclose(a, b, rtol=1e-14, atol=0)


def test_multi_graph_block_structure():
    sizes = [50, 1, 200, 73]
    graphs = []
    rng = np.random.default_rng(4)
    for g, n in enumerate(sizes):
        edges = [(int(rng.integers(n)), int(rng.integers(n))) for _ in range(3 * n)]
        graphs.append(_pr_matrix(n, edges))
    graph_ptr = np.concatenate([[0], np.cumsum(sizes)])

    def assemble(gs):
        rps, cols, vals = [np.zeros(1, np.int64)], [], []
        nnz = 0
        for g, (rp, col, val) in enumerate(gs):
            rps.append(rp[1:].astype(np.int64) + nnz)
            cols.append(col.astype(np.int64) + graph_ptr[g])
            vals.append(val)
            nnz += rp[-1]
        return (np.concatenate(rps).astype(np.int32), np.concatenate(cols).astype(np.int32),
                np.concatenate(vals))

    rp, col, val = assemble(graphs)
    N = graph_ptr[-1]
    x0 = np.concatenate([np.full(n, 1.0 / n) for n in sizes])
    x = oracle.pagerank_multi(rp, col, val, graph_ptr, ALPHA, 40, x0)
    for g in range(len(sizes)):
        a, b = graph_ptr[g], graph_ptr[g + 1]
        assert abs(x[a:b].sum() - 1.0) < 1e-13
    # graph 2's ranks do not depend on graph 0's edges
    g0 = _pr_matrix(sizes[0], [(i, (i + 1) % sizes[0]) for i in range(sizes[0])])
    rp2, col2, val2 = assemble([g0] + graphs[1:])
    x2 = oracle.pagerank_multi(rp2, col2, val2, graph_ptr, ALPHA, 40, x0)
    assert np.array_equal(x2[graph_ptr[2]:graph_ptr[3]], x[graph_ptr[2]:graph_ptr[3]])
    assert np.allclose(x2[:sizes[0]], 1.0 / sizes[0], rtol=1e-13, atol=0)  # a cycle: uniform
    # a single graph is the plain PageRank
    one, _, _ = oracle.pagerank(graphs[2][0], graphs[2][1], graphs[2][2], ALPHA, 40,
                                np.full(sizes[2], 1.0 / sizes[2]))
    assert np.array_equal(one, x[graph_ptr[2]:graph_ptr[3]])
    assert N == sum(sizes)
