"""Pins for the oracle's adjoint pieces (the derivative of the PageRank fixed
point of Sec. 5.5.1 with respect to the matrix values): the CSR transpose, the
adjoint fixed point, the per-nonzero value gradient and the column
normalisation.

Independent checks: dense transposes, the adjoint identity, a dense linear
solve of the adjoint equation, and central finite differences of the oracle's
converged forward PageRank.
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


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_transpose_dense_and_stable(seed):
    rp, col, vals = graphgen.random_csr(31, 23, 0.2, seed, empty_frac=0.3, long_rows=(4,))
    rt, ct, perm = oracle.transpose(23, rp, col)
    assert len(rt) == 24 and rt[0] == 0 and rt[-1] == len(col)
    At = _dense(rt, ct, vals[perm], 31)
    assert np.array_equal(At, _dense(rp, col, vals, 23).T)
    rows = oracle.row_index(rp)
    for c in range(23):
        seg = perm[rt[c]:rt[c + 1]]
        assert np.all(col[seg] == c)
        assert np.all(np.diff(seg) > 0)  # stable: increasing position in A
        assert np.array_equal(ct[rt[c]:rt[c + 1]], rows[seg])
    # transposing twice gives A back, nonzero for nonzero
    r2, c2, p2 = oracle.transpose(31, rt, ct)
    assert np.array_equal(r2, rp) and np.array_equal(c2, col)
    assert np.array_equal(perm[p2], np.arange(len(col)))


def test_transpose_degenerate():
    rt, ct, perm = oracle.transpose(5, np.zeros(4, np.int32), np.zeros(0, np.int32))
    assert np.array_equal(rt, np.zeros(6)) and len(ct) == 0 and len(perm) == 0


@pytest.mark.parametrize("seed", [3, 4])
def test_adjoint_identity(seed):
    """<A x, g> = <x, A^T g> with A^T from the transpose."""
    rp, col, vals = graphgen.random_csr(200, 150, 0.03, seed, empty_frac=0.2)
    rng = np.random.default_rng(seed)
    x, g = rng.uniform(-1, 1, 150), rng.uniform(-1, 1, 200)
    rt, ct, perm = oracle.transpose(150, rp, col)
    lhs = oracle.spmv(rp, col, vals, x) @ g
    rhs = x @ oracle.spmv(rt, ct, vals[perm], g)
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(vals).sum() + 1)


def _pr_graph(n, seed, dangling=True):
    rng = np.random.default_rng(seed)
    edges = {(int(rng.integers(n)), int(rng.integers(n))) for _ in range(3 * n)}
    if dangling:  # vertex n-1 keeps no out-edge
        edges = {(u, v) for u, v in edges if u != n - 1}
    edges = sorted(edges, key=lambda e: (e[1], e[0]))
    rp = np.zeros(n + 1, np.int64)
    for _, v in edges:
        rp[v + 1] += 1
    rp = np.cumsum(rp).astype(np.int32)
    col = np.array([u for u, _ in edges], np.int32)
    return rp, col


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_adjoint_dense_solve(seed):
    """lambda solves (I - M^T) lambda = g, M = alpha P + (alpha/n) 1 d^T."""
    n = 17
    rp, col = _pr_graph(n, seed)
    vals = graphgen.column_stochastic_values(col, n)
    P = _dense(rp, col, vals, n)
    d = (np.bincount(col, minlength=n) == 0).astype(float)
    assert d.sum() >= 1
    M = ALPHA * P + ALPHA / n * np.outer(np.ones(n), d)
    g = np.random.default_rng(seed).uniform(-1, 1, n)
    lam_star = np.linalg.solve(np.eye(n) - M.T, g)
    lam = oracle.pagerank_adjoint(rp, col, vals, ALPHA, 300, g)
    assert np.abs(lam - lam_star).max() <= 1e-12 * np.abs(lam_star).max()
    # a symmetric stand-in would hide a P / P^T mix-up: P here is not symmetric
    assert np.abs(P - P.T).max() > 0.1


def _loss(rp, col, vals, target, iters=400):
    n = len(rp) - 1
    x, _, _ = oracle.pagerank(rp, col, vals, ALPHA, iters, np.full(n, 1.0 / n))
    return float(((x - target) ** 2).sum())


@pytest.mark.parametrize("seed", [8, 9])
def test_value_gradient_finite_differences(seed):
    """dL/dP[e] = alpha lambda[row] x*[col] against central differences of the
    converged forward PageRank, perturbing one stored value at a time."""
    n = 14
    rp, col = _pr_graph(n, seed)
    vals = graphgen.column_stochastic_values(col, n)
    target = np.random.default_rng(seed).dirichlet(np.ones(n))
    x, _, _ = oracle.pagerank(rp, col, vals, ALPHA, 400, np.full(n, 1.0 / n))
    lam = oracle.pagerank_adjoint(rp, col, vals, ALPHA, 400, 2 * (x - target))
    G = oracle.pagerank_value_grad(rp, col, lam, x, ALPHA)
    h = 1e-6
    for e in range(len(col)):
        vp, vm = vals.copy(), vals.copy()
        vp[e] += h
        vm[e] -= h
        fd = (_loss(rp, col, vp, target) - _loss(rp, col, vm, target)) / (2 * h)
        assert abs(fd - G[e]) <= 1e-6 * max(abs(G).max(), 1e-12), (e, fd, G[e])


@pytest.mark.parametrize("seed", [10, 11])
def test_weight_gradient_through_colnorm(seed):
    """dL/dw of ||x*(colnorm(w)) - t||^2 against central differences in w."""
    n = 12
    rp, col = _pr_graph(n, seed)
    rng = np.random.default_rng(seed)
    w = 1.5 - rng.random(len(col))  # (0.5, 1.5]
    target = rng.dirichlet(np.ones(n))
    loss, grad, x, _ = oracle.pagerank_loss_grad(rp, col, w, target, ALPHA, 400)
    h = 1e-6
    for e in range(len(col)):
        wp, wm = w.copy(), w.copy()
        wp[e] += h
        wm[e] -= h
        Lp = _loss(rp, col, oracle.colnorm(col, wp, n)[0], target)
        Lm = _loss(rp, col, oracle.colnorm(col, wm, n)[0], target)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - grad[e]) <= 1e-6 * max(abs(grad).max(), 1e-12), (e, fd, grad[e])
    assert abs(loss - _loss(rp, col, oracle.colnorm(col, w, n)[0], target)) < 1e-15


def test_colnorm_closed_forms():
    rp, col = _pr_graph(30, 12)
    w = np.random.default_rng(12).uniform(0.5, 1.5, len(col))
    P, s = oracle.colnorm(col, w, 30)
    sums = np.bincount(col, weights=P, minlength=30)
    has = np.bincount(col, minlength=30) > 0
    assert np.allclose(sums[has], 1.0, rtol=0, atol=1e-15) and np.all(sums[~has] == 0)
    # equal weights give 1/outdeg
    P1, _ = oracle.colnorm(col, np.full(len(col), 3.0), 30)
    assert np.allclose(P1, graphgen.column_stochastic_values(col, 30), rtol=1e-15, atol=0)
    # scaling a whole column leaves P unchanged, so the gradient is orthogonal
    # to w within each column
    G = np.random.default_rng(13).uniform(-1, 1, len(col))
    gw = oracle.colnorm_backward(col, w, G, 30)
    per_col = np.bincount(col, weights=gw * w, minlength=30)
    assert np.abs(per_col).max() <= 1e-14
