"""The hot-column selection of a plan (the columns whose x values the fused
kernel reads from LDS), checked against the rule it implements, computed
here from exact column counts (the matrices are small enough that the plan
counts every nonzero):

* a plain plan takes the columns whose count is above a cut count t, where
  t is the largest count at which the columns of count t or more exceed the
  cap (the columns at the cut are left out together; no cut when every
  counted column fits);
* a column-stripe plan takes, per tile range, the cap columns of largest
  count of that range's nonzeros, ties by increasing column, so every range
  with at least cap distinct columns takes exactly cap.

The plan reports how many columns it took and the share of the nonzeros
they hold; both must equal the rule's, and the SpMV on the plan must still
match the oracle."""
import numpy as np
import pytest
import torch

from helpers import check_spmv, host_values, require_gpu, seeded_x, to_device

pytestmark = pytest.mark.gpu

HIST_TOP = 65535  # counts at or above this share the histogram's last bin


def _skewed_matrix(n_rows, n_cols, mean_len, seed):
    """Rows of Poisson length, columns drawn as floor(n_cols * u^3): a few
    frequent columns and long runs of equal counts (ties at every cut)."""
    rng = np.random.default_rng(seed)
    lens = rng.poisson(mean_len, n_rows).astype(np.int64)
    row_ptr = np.zeros(n_rows + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum(lens)
    m = int(row_ptr[-1])
    col = np.minimum((n_cols * rng.random(m) ** 3).astype(np.int64), n_cols - 1).astype(np.int32)
    for r in range(n_rows):  # sorted, duplicates allowed (they count twice)
        col[row_ptr[r]:row_ptr[r + 1]].sort()
    vals = rng.uniform(-1.0, 1.0, m)
    return row_ptr, col, vals


def _plain_rule(col, n_cols, cap):
    """(columns taken, nonzeros they hold) of the plain plan's rule."""
    c = np.minimum(np.bincount(col, minlength=n_cols), HIST_TOP)
    counts, freq = np.unique(c[c > 0], return_counts=True)
    run, t = 0, 0
    for b, h in zip(counts[::-1], freq[::-1]):  # from the largest count down
        if run + h > cap:
            t = int(b)
            break
        run += int(h)
    taken = int((c > t).sum()) if t > 0 else int((c > 0).sum())
    return taken, int(c[c > t].sum())


@pytest.mark.parametrize("cap", [37, 256, 1000, 3072])
def test_plain_plan_hot_set_follows_the_cut_rule(cap):
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    n_rows, n_cols = 3000, 6000
    # nnz < 4 n_cols: the plan counts every nonzero (no sampling)
    rp, col, vals = _skewed_matrix(n_rows, n_cols, 3.5, seed=cap)
    assert len(col) < 4 * n_cols
    taken, covered = _plain_rule(col, n_cols, cap)
    assert 0 < taken <= cap
    dtype = torch.float32
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, n_cols, commit="wave", hot_columns=cap)
    info = plan.info()
    print(f"hot select plain cap={cap}: taken {info['hot_columns']} (rule {taken})", flush=True)
    assert info["hot_columns"] == taken
    assert info["hot_coverage"] == pytest.approx(covered / len(col), rel=1e-12, abs=0.0)
    x64 = seeded_x(n_cols, 31, dtype)
    y = plan.spmv(torch.from_numpy(x64).to(dtype).to(dev))
    torch.cuda.synchronize()
    check_spmv(y, rp, col, host_values(vals, dtype), x64, dtype, f"hot cap {cap}")
    plan.close()


def test_plain_plan_whole_tie_at_the_cut_is_left_out():
    """Every column has the same count: the cut falls on that count and the
    whole tie is left out, so the plan keeps no cache at all."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    n_rows, n_cols = 2000, 2048
    rng = np.random.default_rng(5)
    col = np.tile(np.arange(n_cols, dtype=np.int32), 3)  # every column 3 times
    rng.shuffle(col)
    lens = np.full(n_rows, len(col) // n_rows, dtype=np.int64)
    lens[: len(col) - int(lens.sum())] += 1
    rp = np.zeros(n_rows + 1, dtype=np.int32)
    rp[1:] = np.cumsum(lens)
    vals = rng.uniform(-1.0, 1.0, len(col))
    assert _plain_rule(col, n_cols, 1000) == (0, 0)
    r, c, v = to_device(rp, col, vals, torch.float32, dev)
    plan = pkg.Plan(r, c, v, n_cols, commit="wave", hot_columns=1000)
    assert plan.info()["hot_columns"] == 0
    plan.close()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_striped_plan_takes_cap_columns_per_range(dtype):
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    n_rows, n_cols = 40000, 60000
    rp, col, vals = _skewed_matrix(n_rows, n_cols, 6.0, seed=11)
    # a range of fewer than 64 * cap nonzeros is counted exactly (no sample)
    cap = 1024
    assert len(col) < 8 * 64 * cap // 2
    r, c, v = to_device(rp, col, vals, dtype, dev)
    plan = pkg.Plan(r, c, v, n_cols, commit="wave", stripes=8, hot_columns=cap)
    info = plan.info()
    print(f"hot select striped {dtype}: ranges {info['ranges']} taken {info['hot_columns']}",
          flush=True)
    # every range holds thousands of distinct columns: each takes exactly cap
    assert info["ranges"] == 8 and info["hot_columns"] == cap * info["ranges"]
    # each range's cap most frequent columns hold at least as many of its
    # nonzeros as the matrix's cap most frequent columns do: summed over the
    # ranges, at least those columns' share of the matrix
    top = np.sort(np.bincount(col, minlength=n_cols))[::-1]
    assert top[:cap].sum() / len(col) <= info["hot_coverage"] <= 1.0
    x64 = seeded_x(n_cols, 32, dtype)
    y = plan.spmv(torch.from_numpy(x64).to(dtype).to(dev))
    torch.cuda.synchronize()
    check_spmv(y, rp, col, host_values(vals, dtype), x64, dtype, "striped hot")
    plan.close()


def test_striped_plan_with_room_for_every_column_covers_all():
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    n_rows, n_cols = 4000, 3000
    rp, col, vals = _skewed_matrix(n_rows, n_cols, 4.0, seed=12)
    r, c, v = to_device(rp, col, vals, torch.float32, dev)
    plan = pkg.Plan(r, c, v, n_cols, commit="wave", stripes=8, hot_columns=4096)
    info = plan.info()
    assert info["hot_coverage"] == 1.0
    # a range takes each of its distinct columns once
    assert np.unique(col).size <= info["hot_columns"] <= info["ranges"] * np.unique(col).size
    plan.close()


@pytest.mark.parametrize("stripes", [0, 8], ids=["plain", "striped8"])
def test_wide_sparse_matrix_hot_set(stripes):
    """Far more columns than nonzeros (the selection's work space then
    outgrows what the build reserves from the nonzero count): the hot set is
    still the rule's and the SpMV matches the oracle."""
    import paper_2605_07391_amd as pkg
    dev = require_gpu()
    n_rows, n_cols = 600, 1_500_000
    rp, col, vals = _skewed_matrix(n_rows, n_cols, 5.0, seed=21)
    cap = 64
    r, c, v = to_device(rp, col, vals, torch.float32, dev)
    plan = pkg.Plan(r, c, v, n_cols, commit="wave", stripes=stripes, hot_columns=cap)
    info = plan.info()
    print(f"wide sparse stripes={stripes}: taken {info['hot_columns']}", flush=True)
    if stripes == 0:
        taken, covered = _plain_rule(col, n_cols, cap)
        assert info["hot_columns"] == taken
        assert info["hot_coverage"] == pytest.approx(covered / len(col), rel=1e-12, abs=0.0)
    else:
        assert 0 < info["hot_columns"] <= cap * info["ranges"]
    x64 = seeded_x(n_cols, 33, torch.float32)
    y = plan.spmv(torch.from_numpy(x64).to(torch.float32).to(dev))
    torch.cuda.synchronize()
    check_spmv(y, rp, col, host_values(vals, torch.float32), x64, torch.float32, "wide sparse")
    plan.close()
