"""Pins for the oracle's BiCGSTAB (Sec. 5.5.2; van der Vorst 1992).

Independent checks: dense solves of well-conditioned systems, SciPy's own
BiCGSTAB iterate by iterate (same algorithm, different code), exact
termination on a multiple of the identity, and the true residual at exit.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import graphgen
import oracle


def _dominant(n, density, seed, sym=False):
    """Sparse, strictly diagonally dominant (non-symmetric unless sym)."""
    rng = np.random.default_rng(seed)
    A = sp.random(n, n, density=density, random_state=rng, format="csr")
    A.data = rng.uniform(-1, 1, A.nnz)
    if sym:
        A = (A + A.T).tocsr()
    A = A + sp.diags(np.asarray(abs(A).sum(axis=1)).ravel() + 1.0)
    A = A.tocsr()
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64), A


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dense_solve(seed):
    rp, col, vals, A = _dominant(60, 0.08, seed)
    rng = np.random.default_rng(seed + 10)
    b = rng.uniform(-1, 1, 60)
    x, it, status, hist = oracle.bicgstab(rp, col, vals, b, np.zeros(60), 1e-13, 500)
    assert status == "converged" and it == len(hist) and hist[-1] < 1e-13
    x_star = np.linalg.solve(A.toarray(), b)
    assert np.abs(x - x_star).max() <= 1e-11 * np.abs(x_star).max()
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-12


@pytest.mark.parametrize("seed", [3, 4])
def test_matches_scipy_iterate_by_iterate(seed):
    rp, col, vals, A = _dominant(80, 0.05, seed)
    b = np.random.default_rng(seed).uniform(-1, 1, 80)
    x0 = np.random.default_rng(seed + 1).uniform(-1, 1, 80)
    for k in range(1, 7):
        x, it, status, _ = oracle.bicgstab(rp, col, vals, b, x0, 1e-300, k)
        assert it == k and status == "iteration cap"
        xs, _ = spla.bicgstab(A, b, x0=x0.copy(), rtol=1e-300, atol=0.0, maxiter=k)
        assert np.abs(x - xs).max() <= 1e-12 * max(np.abs(xs).max(), 1.0), k


def test_identity_multiple_terminates_in_one_step():
    n = 25
    rp = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    vals = np.full(n, 4.0)
    b = np.random.default_rng(5).uniform(-1, 1, n)
    x, it, status, hist = oracle.bicgstab(rp, col, vals, b, np.zeros(n), 1e-10, 10)
    assert it == 1 and status == "converged" and hist[0] == 0.0
    assert np.array_equal(x, b / 4.0)
    # a zero right-hand side with x0 = 0 is solved before the first step
    x, it, status, _ = oracle.bicgstab(rp, col, vals, np.zeros(n), np.zeros(n), 1e-10, 10)
    assert it == 0 and status == "converged" and not x.any()


def test_symmetric_01_workload():
    """The paper's construction: A = 0/1 adjacency of an undirected graph
    (plus the identity here, so the small system is nonsingular), b = A x
    with x uniform in [-1, 1]; the solve recovers x."""
    rp0, col0, _ = graphgen.random_csr(300, 300, 0.02, 7)
    A = sp.csr_matrix((np.ones(len(col0)), col0, rp0), shape=(300, 300))
    A = ((A + A.T) > 0).astype(np.float64) + 8.0 * sp.eye(300)
    A = A.tocsr()
    A.sort_indices()
    xt = graphgen.uniform(7, 85, 300, -1.0, 1.0)
    b = A @ xt
    x, it, status, hist = oracle.bicgstab(A.indptr.astype(np.int32), A.indices.astype(np.int32),
                                          A.data, b, np.zeros(300), 1e-10, 2000)
    assert status == "converged" and hist[-1] < 1e-10
    assert np.abs(x - xt).max() <= 1e-8
