"""Pins for the oracle's merge path and TILE plan (Sec. 3.3, Algorithm 1,
Sec. 4.1.1-4.1.2, Sec. 4.3).

Independent derivations used here:
* the merge path written as the concatenation, row by row, of one right step
  per nonzero followed by one down step (Sec. 3.3: right = accumulate,
  down = store);
* Algorithm 1 (binary search) against the sequential walk on every diagonal;
* the worked example printed in Sec. 3.3 / 4.1.1 (tests/golden);
* the closed forms of Sec. 4.1.1 / 4.3 and invariants of the encoding;
* replaying the decoded TILE reproduces the SpMV of Sec. 3.1 bit for bit.
"""
import numpy as np
import pytest

import graphgen
import oracle
from conftest import golden

OMEGA = 64


def step_string(row_ptr):
    """Sec. 3.3 merge path as a step list: per row, len(row) rights then a down."""
    steps = []
    for r in range(len(row_ptr) - 1):
        steps += [0] * int(row_ptr[r + 1] - row_ptr[r]) + [1]
    return np.array(steps, np.int64)


def coords_from_steps(steps):
    down = np.concatenate([[0], np.cumsum(steps)])
    right = np.arange(len(steps) + 1) - down
    return right, down


def plan_from_steps(row_ptr, omega, sigma):
    """Brute-force TILE from the step list (no walk, no search)."""
    steps = step_string(row_ptr)
    L = len(steps)
    xs, ys = coords_from_steps(steps)
    b = int(np.ceil(np.log2(omega * sigma)))
    T = -(-L // (omega * sigma))
    lanes = -(-L // sigma)
    tile_x = np.zeros(T + 1, np.int64)
    tile_y = np.zeros(T + 1, np.int64)
    for i in range(T):
        s = i * omega * sigma
        e = min(s + omega * sigma, L)
        tile_x[i] = xs[s]
        tile_y[i] = ys[s] | (0 if steps[s:e].any() else 1 << 31)
    tile_x[T] = row_ptr[-1]
    tile_y[T] = len(row_ptr) - 1
    desc = np.zeros(lanes, np.uint64)  # up to 64-bit descriptors
    for j in range(lanes):
        s = j * sigma
        t0 = (j // omega) * omega * sigma
        flags = sum(int(v) << k for k, v in enumerate(steps[s:s + sigma]))
        desc[j] = (flags << (2 * b)) | (int(ys[s] - ys[t0]) << b) | int(xs[s] - xs[t0])
    return tile_x, tile_y, desc


CASES = [
    ("one_row", np.array([0, 1], np.int32)),
    ("empty_rows_only", np.zeros(9, np.int32)),
    ("no_rows", np.zeros(1, np.int32)),
    ("single_long_row", np.array([0, 3000], np.int32)),
    ("long_then_empty", np.array([0, 2000, 2000, 2000, 2001, 4500], np.int32)),
]


def _random_cases():
    out = []
    for seed, (n, nc, dens, emp) in enumerate([(50, 40, 0.3, 0.2), (200, 300, 0.05, 0.5),
                                               (120, 800, 0.4, 0.1), (333, 64, 0.02, 0.0)]):
        rp, _, _ = graphgen.random_csr(n, nc, dens, seed, empty_frac=emp, long_rows=(n // 3,))
        out.append((f"random{seed}", rp))
    rp, _ = graphgen.chung_lu_pattern(2000, 20000, 2.1, 0.1, seed=9)
    out.append(("chung_lu_2k", rp))
    return out


ALL = CASES + _random_cases()


@pytest.mark.parametrize("name,row_ptr", ALL, ids=[c[0] for c in ALL])
def test_walk_and_search_match_step_string(name, row_ptr):
    xs_ref, ys_ref = coords_from_steps(step_string(row_ptr))
    xs, ys = oracle.path_coords(row_ptr)
    assert np.array_equal(xs, xs_ref) and np.array_equal(ys, ys_ref)
    L = len(xs) - 1
    diags = range(L + 1) if L <= 5000 else np.linspace(0, L, 3000).astype(int)
    for d in diags:
        assert oracle.merge_search(row_ptr, int(d)) == (xs_ref[d], ys_ref[d])


@pytest.mark.parametrize("sigma", [1, 4, 7, 12])
@pytest.mark.parametrize("name,row_ptr", ALL, ids=[c[0] for c in ALL])
def test_plan_matches_step_string(name, row_ptr, sigma):
    tx, ty, desc = oracle.plan(row_ptr, OMEGA, sigma)
    rx, ry, rd = plan_from_steps(row_ptr, OMEGA, sigma)
    assert np.array_equal(tx.astype(np.int64), rx)
    assert np.array_equal(ty.astype(np.int64), ry)
    assert np.array_equal(desc.astype(np.int64), rd)


def test_worked_example():
    g = golden("worked_example.txt")
    omega, sigma = int(g["omega"][0]), int(g["sigma"][0])
    rp = np.array([int(v) for v in g["row_ptr"]], np.int32)
    n, m = len(rp) - 1, int(rp[-1])
    assert [m, n] == [int(v) for v in g["path_end"]]
    tx, ty, desc = oracle.plan(rp, omega, sigma)
    assert len(tx) - 1 == int(g["tile_num"][0])
    assert (m + n) - (len(tx) - 2) * omega * sigma == int(g["last_tile_steps"][0])
    assert [int(v) & 0x7FFFFFFF for v in ty] == [int(v) for v in g["tile_y"]]
    xo, yo, fl = oracle.unpack_desc(desc, omega, sigma)
    starts = [int(v) for v in g["tile0_lane_starts"]]
    for j in range(4):
        assert (tx[0] + xo[j], (ty[0] & 0x7FFFFFFF) + yo[j]) == (starts[2 * j], starts[2 * j + 1])
    assert (tx[1], ty[1] & 0x7FFFFFFF) == tuple(int(v) for v in g["tile0_end"])
    assert list(xo[4:8]) == [int(v) for v in g["tile1_x_offset"]]
    assert list(yo[4:8]) == [int(v) for v in g["tile1_y_offset"]]
    bits = [(int(fl[4]) >> k) & 1 for k in range(sigma)]
    assert bits == [1 if v == "T" else 0 for v in g["tile1_lane0_bit_flag"]]
    # path coordinates agree with the same facts
    xs, ys = oracle.path_coords(rp)
    assert (xs[16], ys[16]) == (13, 3)


def test_closed_forms_and_field_widths():
    # Sec. 4.1.1: tile_num, lane_num
    assert oracle.plan_sizes(8, 34, 4, 4) == (3, 11)
    assert oracle.plan_sizes(0, 0, 64, 12) == (0, 0)
    # Fig. 4 layout at omega = 32, sigma = 14: offsets 9 bits each, flags at bit 18
    assert oracle.offset_bits(32, 14) == 9 and 2 * 9 + 14 == 32
    # wavefront-64 layouts: sigma 12 -> 10 | 10 | 12, sigma 7 -> 9 | 9 | 7
    assert oracle.offset_bits(64, 12) == 10
    assert oracle.offset_bits(64, 7) == 9
    assert oracle.offset_bits(64, 8) == 9
    # 2b + sigma <= 32 (Sec. 4.1.1); sigma = 13 at omega = 64 does not fit
    with pytest.raises(ValueError):
        oracle.plan(np.array([0, 5], np.int32), 64, 13)
    tx, ty, desc = oracle.plan(np.array([0, 5], np.int32), 64, 12)
    assert len(desc) == 1


def test_desc_roundtrip_and_packing():
    rp, _, _ = graphgen.random_csr(150, 100, 0.2, 21, empty_frac=0.3)
    for sigma in (7, 12):
        tx, ty, desc = oracle.plan(rp, OMEGA, sigma)
        b = oracle.offset_bits(OMEGA, sigma)
        xo, yo, fl = oracle.unpack_desc(desc, OMEGA, sigma)
        repacked = (fl << (2 * b)) | (yo << b) | xo
        assert np.array_equal(repacked.astype(np.uint32), desc)
        assert xo.max() < (1 << b) and yo.max() < (1 << b) and fl.max() < (1 << sigma)


@pytest.mark.parametrize("sigma", [7, 12])
@pytest.mark.parametrize("name,row_ptr", ALL, ids=[c[0] for c in ALL])
def test_plan_invariants(name, row_ptr, sigma):
    n = len(row_ptr) - 1
    m = int(row_ptr[-1])
    L = m + n
    tx, ty, desc = oracle.plan(row_ptr, OMEGA, sigma)
    T, lanes = oracle.plan_sizes(n, m, OMEGA, sigma)
    assert len(tx) == T + 1 and len(desc) == lanes
    row = (ty & 0x7FFFFFFF).astype(np.int64)
    # the tile start lies on diagonal i * omega * sigma; the last entry is (m, n)
    for i in range(T + 1):
        assert tx[i] + row[i] == min(i * OMEGA * sigma, L)
    assert tx[T] == m and ty[T] == n
    # MSB <=> the tile finishes no row
    for i in range(T):
        assert bool(ty[i] >> 31) == (row[i + 1] == row[i])
    # per lane: downs = rows finished, rights = nonzeros consumed; tail bits 0
    xo, yo, fl = oracle.unpack_desc(desc, OMEGA, sigma)
    xs, ys = oracle.path_coords(row_ptr)
    for j in range(lanes):
        i = j // OMEGA
        s = j * sigma
        e = min(s + sigma, L)
        assert tx[i] + xo[j] == xs[s] and row[i] + yo[j] == ys[s]
        pc = bin(int(fl[j])).count("1")
        assert pc == ys[e] - ys[s]
        assert (e - s) - pc == xs[e] - xs[s]
        assert int(fl[j]) >> (e - s) == 0


@pytest.mark.parametrize("name,row_ptr", ALL, ids=[c[0] for c in ALL])
def test_plan_replay_reproduces_spmv(name, row_ptr):
    n = len(row_ptr) - 1
    m = int(row_ptr[-1])
    rng = np.random.default_rng(5)
    nc = 900
    col = rng.integers(0, nc, m).astype(np.int32)
    vals = rng.uniform(-1, 1, m)
    x = rng.uniform(-1, 1, nc)
    ref = oracle.spmv(row_ptr, col, vals, x)
    for sigma in (1, 7, 12):
        tile = oracle.plan(row_ptr, OMEGA, sigma)
        y, nnz_row = oracle.plan_replay(row_ptr, col, vals, x, tile, OMEGA, sigma)
        assert np.array_equal(y, ref)  # same order -> identical bits
        assert np.array_equal(nnz_row, np.repeat(np.arange(n), np.diff(row_ptr)))


def test_replay_detects_corrupt_plan():
    # A plan with a flipped flag bit no longer reproduces the SpMV (or fails
    # its bounds checks): the replay pin can tell a wrong TILE apart.
    rp, col, vals = graphgen.random_csr(60, 50, 0.3, 8, empty_frac=0.2)
    x = np.random.default_rng(1).uniform(-1, 1, 50)
    tx, ty, desc = oracle.plan(rp, OMEGA, 7)
    ref = oracle.spmv(rp, col, vals, x)
    bad = desc.copy()
    bad[3] ^= np.uint32(1 << (2 * oracle.offset_bits(OMEGA, 7) + 2))
    try:
        y, _ = oracle.plan_replay(rp, col, vals, x, (tx, ty, bad), OMEGA, 7)
        assert not np.array_equal(y, ref)
    except ValueError:
        pass


def test_tile_memory_formula():
    # Sec. 4.3: mem_sigma counts 8 (T + 1) bytes of tile starts plus 4 bytes per
    # descriptor of the non-fast tiles (r_f = fraction of fast tiles)
    rp, _ = graphgen.chung_lu_pattern(3000, 60000, 2.1, 0.1, seed=4)
    n, m = len(rp) - 1, int(rp[-1])
    for sigma in (7, 12):
        tx, ty, desc = oracle.plan(rp, OMEGA, sigma)
        T = len(tx) - 1
        fast = (ty[:T] >> 31).astype(bool)
        r_f = fast.mean()
        lanes_per_tile = np.minimum(OMEGA, len(desc) - np.arange(T) * OMEGA)
        actual = 8 * (T + 1) + 4 * int(lanes_per_tile[~fast].sum())
        formula = oracle.tile_mem_bytes(n, m, OMEGA, sigma, r_f)
        assert abs(formula - actual) <= 4 * OMEGA
    assert oracle.smem_bytes(256, 12, 4) == 257 * 12 * 4


# ------------------------------------------------- 64-bit lane descriptors --

@pytest.mark.parametrize("sigma", [1, 7, 12, 13, 16, 24, 33, 40])
@pytest.mark.parametrize("name,row_ptr", CASES + _random_cases())
def test_plan64_matches_step_string(name, row_ptr, sigma):
    tx, ty, d = oracle.plan64(row_ptr, OMEGA, sigma)
    bx, by, bd = plan_from_steps(row_ptr, OMEGA, sigma)
    assert np.array_equal(tx, bx) and np.array_equal(ty.astype(np.int64), by)
    assert np.array_equal(d.astype(np.uint64), bd.astype(np.uint64))
    if sigma <= 12:  # the 32-bit plan holds the same values
        t32 = oracle.plan(row_ptr, OMEGA, sigma)
        assert np.array_equal(t32[2].astype(np.uint64), d)
    b = oracle.offset_bits(OMEGA, sigma)
    assert 2 * b + sigma <= 64 and np.all((d >> np.uint64(2 * b)) < (np.uint64(1) << np.uint64(sigma)))


def test_plan64_fit_condition_and_replay():
    # sigma 40 is the largest that fits: b = 12, 24 + 40 = 64; sigma 41 does not
    assert oracle.offset_bits(64, 40) == 12 and oracle.offset_bits(64, 41) == 12
    with pytest.raises(ValueError):
        oracle.plan64(np.array([0, 1], np.int32), OMEGA, 41)
    with pytest.raises(ValueError):
        oracle.plan(np.array([0, 1], np.int32), OMEGA, 13)
    rp, col, vals = graphgen.random_csr(700, 500, 0.03, 11, empty_frac=0.4, long_rows=(9, 300))
    x = np.random.default_rng(11).uniform(-1, 1, 500)
    ref = oracle.spmv(rp, col, vals, x)
    for sigma in (16, 24, 40):
        y = oracle.plan_replay64(rp, col, vals, x, oracle.plan64(rp, OMEGA, sigma), OMEGA, sigma)
        assert np.array_equal(y, ref)
    # a corrupted descriptor (one flag bit flipped) is rejected or changes y
    t = oracle.plan64(rp, OMEGA, 24)
    bad = (t[0], t[1], t[2].copy())
    bad[2][3] ^= np.uint64(1) << np.uint64(2 * oracle.offset_bits(OMEGA, 24))
    try:
        y = oracle.plan_replay64(rp, col, vals, x, bad, OMEGA, 24)
        assert not np.array_equal(y, ref)
    except ValueError:
        pass
