"""CPU checks of the column-stripe decomposition that striped plans use: the
stacked matrix A' (rows = non-empty (stripe, row) pairs, stripe-major) and
the per-row sum R, with A x = R (A' x) -- on a hand-worked example and on
random matrices against dense products.  The stacked row pointer is the
definition the GPU tests compare the library's plans with."""
import numpy as np

from helpers import stacked_row_ptr


def _dense(rp, col, vals, n_rows, n_cols):
    A = np.zeros((n_rows, n_cols))
    for r in range(n_rows):
        for k in range(rp[r], rp[r + 1]):
            A[r, col[k]] += vals[k]
    return A


def test_hand_example():
    # 3 rows, 8 columns, 2 stripes of width 4: row 0 = {1, 5, 6}, row 1 = {},
    # row 2 = {7, 0}
    rp = np.array([0, 3, 3, 5])
    col = np.array([1, 5, 6, 7, 0])
    vrp, order = stacked_row_ptr(rp, col, 8, 2)
    # stripe 0: (0, row 0) = {1}, (0, row 2) = {0}; stripe 1: (1, row 0) =
    # {5, 6}, (1, row 2) = {7}
    assert vrp.tolist() == [0, 1, 2, 4, 5]
    assert col[order].tolist() == [1, 0, 5, 6, 7]


def test_stacked_product_sums_to_the_matrix_product():
    rng = np.random.default_rng(3)
    for n_rows, n_cols, dens, S in [(50, 40, 0.2, 2), (120, 1000, 0.01, 8), (30, 7, 0.5, 32),
                                    (200, 64, 0.05, 4), (1, 5, 1.0, 8)]:
        mask = rng.random((n_rows, n_cols)) < dens
        rp = np.r_[0, np.cumsum(mask.sum(1))]
        col = np.nonzero(mask)[1]
        vals = rng.uniform(-1, 1, len(col))
        x = rng.uniform(-1, 1, n_cols)
        vrp, order = stacked_row_ptr(rp, col, n_cols, S)
        cs, vs = col[order], vals[order]
        yv = np.array([np.dot(vs[vrp[v]:vrp[v + 1]], x[cs[vrp[v]:vrp[v + 1]]])
                       for v in range(len(vrp) - 1)])
        # the row of each stacked row, and its stripe (both non-decreasing
        # within a stripe: stripe-major, rows in order)
        rows = np.repeat(np.arange(n_rows), np.diff(rp))[order]
        vrow = rows[vrp[:-1]]
        cbits = int(np.ceil(np.log2(n_cols))) if n_cols > 1 else 0
        shift = max(0, cbits - int(np.log2(S)))
        vstripe = (cs[vrp[:-1]] >> shift) if len(vrp) > 1 else np.zeros(0, int)
        assert np.all(np.diff(vstripe * (n_rows + 1) + vrow) > 0)  # distinct pairs, ordered
        assert vstripe.max(initial=0) < S
        y = np.zeros(n_rows)
        np.add.at(y, vrow, yv)
        np.testing.assert_allclose(y, _dense(rp, col, vals, n_rows, n_cols) @ x, atol=1e-12)
        # every nonzero of a stacked row lies in its pair's stripe and row
        for v in range(len(vrp) - 1):
            seg = slice(vrp[v], vrp[v + 1])
            assert np.all(cs[seg] >> shift == vstripe[v]) and np.all(rows[seg] == vrow[v])
