"""Host logic of bench.py (no GPU): the one-GPU refusal, kernel-instance
names, and the choice of the committed HBM-traffic record."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def _info(sigma=32, dtype=0, desc_bits=64, commit=2, stripes=8, lanes=512, hot=1):
    return {"sigma": sigma, "dtype": dtype, "desc_bits": desc_bits, "commit": commit,
            "stripes": stripes, "block_lanes": lanes, "hot_columns": hot}


def test_kernel_instance_names():
    assert bench.kernel_instance(_info()) == \
        "merbit::spmv_wave_kernel<float, 32, 8, true, unsigned long>"
    assert bench.kernel_instance(_info(sigma=7, dtype=1, desc_bits=32, hot=0)) == \
        "merbit::spmv_wave_kernel<double, 7, 8, false, unsigned int>"
    assert bench.kernel_instance(_info(sigma=12, commit=1, desc_bits=32, lanes=256)) == \
        "merbit::spmv_kernel<float, 12, 4, true>"


def test_traffic_record_must_match_instance_stripes_and_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    info = _info()
    good = {"kernel": bench.kernel_instance(info), "stripes": 8,
            "spmv_source_sha256_16": bench.spmv_source_hash(2, 8), "hbm_bytes_per_launch": 123}
    near = dict(good, kernel=bench.kernel_instance(_info(sigma=28)), hbm_bytes_per_launch=456)
    stale = dict(good, spmv_source_sha256_16="0" * 16, hbm_bytes_per_launch=789)
    (prof / "spmv_traffic_w_f32.json").write_text(json.dumps(good))
    (prof / "spmv_traffic_w_f32_sigma28.json").write_text(json.dumps(near))
    (prof / "spmv_traffic_v_f32.json").write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.load_traffic("w", "f32", info) == 123
    assert bench.load_traffic("w", "f32", _info(sigma=28)) == 456
    assert bench.load_traffic("w", "f32", _info(sigma=24)) is None   # no record
    assert bench.load_traffic("w", "f32", _info(stripes=4)) is None  # other stripe count
    assert bench.load_traffic("v", "f32", info) is None              # taken on other sources
    assert bench.load_traffic("w", "f64", info) is None


@pytest.mark.parametrize("vs", [4, 8])
def test_algorithmic_bytes_cover_the_csr_arrays_and_vectors(vs):
    info = {"nnz": 1000, "n_rows": 300, "n_cols": 200, "tile_num": 10, "lane_num": 640,
            "fast_tiles": 2, "sigma": 2, "desc_bits": 32, "stripes": 1, "plan_rows": 300}
    floor = (4 + vs) * 1000 + vs * (300 + 200)
    assert bench.algorithmic_bytes(info, vs) >= floor


def test_descriptor_bytes_follow_the_descriptor_width():
    info = {"nnz": 1000, "n_rows": 300, "n_cols": 200, "tile_num": 10, "lane_num": 640,
            "fast_tiles": 2, "desc_bits": 32}
    b32 = bench.algorithmic_bytes(info, 4)
    b64 = bench.algorithmic_bytes(dict(info, desc_bits=64), 4)
    assert b64 - b32 == pytest.approx(4 * 640 * (1 - 2 / 10))


def _pagerank_chunk_keys(buf, stacked, steps, check_every=10):
    """The HIP-graph keys one merbit_pagerank call looks up, as its host loop
    forms them: full chunks of check_every iterations are keyed by (parity of
    the chunk's first iteration, output buffer holding zeros at the boundary
    rows, first chunk of the call or not, stacked-buffer parity); a shorter
    last chunk runs without a graph.  Both buffer states flip once per
    iteration.  Returns (keys, buf, stacked) after the call."""
    keys, t = [], 0
    while t < steps:
        ln = min(check_every - t % check_every, steps - t)
        if ln == check_every:
            keys.append((t & 1, buf, int(t == 0), stacked))
        t += ln
        buf ^= ln & 1
        stacked ^= ln & 1
    return keys, buf, stacked


@pytest.mark.parametrize("warmup", [0, 5, 20, 33])
@pytest.mark.parametrize("steps", [10, 20, 25, 100, 7])
def test_timed_pagerank_call_replays_recorded_graphs(warmup, steps):
    recorded = set()
    buf, stacked = 0, 0
    if warmup:
        keys, buf, stacked = _pagerank_chunk_keys(buf, stacked, warmup)
        recorded.update(keys)
    for _ in range(bench.timed_prep_calls(steps)):
        keys, buf, stacked = _pagerank_chunk_keys(buf, stacked, steps)
        recorded.update(keys)
    timed, _, _ = _pagerank_chunk_keys(buf, stacked, steps)
    assert set(timed) <= recorded
    assert len(recorded) <= 8  # the plan keeps eight graphs


def _counter_csv(path, rows):
    path.mkdir()
    with open(path / "run_counter_collection.csv", "w") as f:
        f.write('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
        for disp, name, ctr, val in rows:
            f.write(f'{disp},"{name}","{ctr}",{val}\n')


def test_traffic_record_from_counter_runs(tmp_path):
    """FETCH / WRITE per SpMV = fused + stripe-sum launches, averaged over the
    dispatches (summing the per-instance rows of one dispatch), scaled by the
    1 GiB copy's counters."""
    info = _info()
    fused = "void " + bench.kernel_instance(info) + "(merbit::SpmvArgs)"
    comb = "void merbit::stripe_combine_kernel<float, 8>(float const*, long)"
    _counter_csv(tmp_path / "f", [(1, fused, "FETCH_SIZE", 100.0), (1, fused, "FETCH_SIZE", 50.0),
                                  (2, fused, "FETCH_SIZE", 170.0), (3, comb, "FETCH_SIZE", 10.0),
                                  (4, "other", "FETCH_SIZE", 1e6)])
    _counter_csv(tmp_path / "w", [(1, fused, "WRITE_SIZE", 20.0), (2, comb, "WRITE_SIZE", 4.0)])
    _counter_csv(tmp_path / "cf", [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0)])
    _counter_csv(tmp_path / "cw", [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576.0)])
    rec = bench.traffic_record("rmat22", "f32", info, 1.5e8, str(tmp_path / "f"),
                               str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"))
    assert rec["fetch_size_kib_per_spmv_raw"] == 170.0   # (150 + 170) / 2 + 10
    assert rec["write_size_kib_per_spmv_raw"] == 24.0
    assert rec["copy_calibration"]["fetch_factor"] == 2.0
    assert rec["hbm_fetch_bytes_per_launch"] == 170 * 1024 * 2
    assert rec["hbm_write_bytes_per_launch"] == 24 * 1024
    assert rec["spmv_source_sha256_16"] == bench.spmv_source_hash(2, 8)
    assert rec["kernel"] == bench.kernel_instance(info) and rec["stripes"] == 8
