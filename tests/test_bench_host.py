"""Host-side logic of bench.py: the roofline entry of the dominant kernel,
the counter-traffic gate on the kernel sources, and the one-GPU contract."""
import json
import os
import subprocess
import sys

import pytest

import bench


def _timing():
    # name -> (launches, total ms, algorithmic bytes, algorithmic flops), as prnu.timing_report()
    return {
        "dwt_fwd_wiener<16>": (10, 5.0, 10 * 2.0e8, 10 * 2.0e9),
        "pce_direct_mfma": (1, 2.0, 5.0e9, 1.0e11),
        "rfft_rows": (4, 1.0, 4 * 1.0e9, 0.0),
    }


def test_roofline_of_the_dominant_kernel():
    roof, kernels = bench.roofline_block(_timing(), steps=2, use_traffic=False)
    assert roof["kernel"] == "dwt_fwd_wiener<16>"  # the largest total time
    assert roof["bound"] == "alu" and roof["unit"] == "TFLOP/s" and roof["peak"] == bench.VALU_PEAK_TFLOPS
    dur = 5.0e-3 / 10
    assert roof["avg_launch_us"] == pytest.approx(dur * 1e6)
    assert roof["achieved"] == pytest.approx(2.0e9 / dur / 1e12, rel=1e-3)
    assert roof["frac"] == pytest.approx(roof["achieved"] / bench.VALU_PEAK_TFLOPS, rel=1e-3)
    assert roof["hbm_gbs"] == pytest.approx(2.0e8 / dur / 1e9, rel=1e-3)
    assert roof["traffic"] is None
    assert list(kernels) == ["dwt_fwd_wiener<16>", "pce_direct_mfma", "rfft_rows"]
    assert kernels["dwt_fwd_wiener<16>"]["ms_per_step"] == pytest.approx(2.5)
    assert kernels["rfft_rows"]["tflops"] is None


def test_bound_classes():
    t = {"pce_direct_mfma": (2, 10.0, 1.0e9, 4.0e11)}
    roof, _ = bench.roofline_block(t, steps=1, use_traffic=False)
    assert roof["bound"] == "mfma" and roof["peak"] == bench.MFMA_F32_PEAK_TFLOPS
    assert roof["achieved"] == pytest.approx(4.0e11 / 2 / 5.0e-3 / 1e12, rel=1e-3)
    t = {"sda_u8_quads<3>": (4, 2.0, 4 * 1.0e9, 0.0)}
    roof, _ = bench.roofline_block(t, steps=1, use_traffic=False)
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == bench.HBM_PEAK_GBS
    assert roof["achieved"] == pytest.approx(1.0e9 / 0.5e-3 / 1e9, rel=1e-3)


def test_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    rec = {"source_hash": bench.kernel_source_hash(), "bytes_per_launch": 123456789}
    f.write_text(json.dumps({"dwt_fwd_wiener<16>": rec}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    roof, _ = bench.roofline_block(_timing(), steps=1, use_traffic=True)
    assert roof["traffic"] == 123456789
    rec["source_hash"] = "0" * 16  # counters taken on other kernel sources
    f.write_text(json.dumps({"dwt_fwd_wiener<16>": rec}))
    roof, _ = bench.roofline_block(_timing(), steps=1, use_traffic=True)
    assert roof["traffic"] is None


def test_committed_traffic_record_is_consistent():
    """The committed record names the dominant kernel, carries both counter
    readings and the copy calibration, and its bytes are the calibrated sum."""
    with open(bench.TRAFFIC_FILE) as fh:
        tr = json.load(fh)
    rec = tr["dwt_fwd_wiener<16>"]
    got = rec["fetch_kib_per_launch"] * 1024 * rec["fetch_factor"] + rec["write_kib_per_launch"] * 1024 * rec[
        "write_factor"]
    assert rec["bytes_per_launch"] == pytest.approx(got, rel=1e-3)
    assert rec["bytes_per_launch"] >= 0.9 * rec["algorithmic_bytes_per_launch"]
    assert len(rec["source_hash"]) == 16


def test_more_than_one_gpu_is_refused(repo_root):
    env = dict(os.environ, WORLD_SIZE="1")
    r = subprocess.run([sys.executable, os.path.join(repo_root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, env=env, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_oracle_pool_leaves_no_process():
    """The oracle's multi-core leg runs plain child processes and joins them:
    no worker, tracker or helper process outlives the call."""
    import numpy as np
    import psutil

    rng = np.random.default_rng(3)
    jobs = [(rng.uniform(0, 255, (48, 64)), "sda" if i % 2 else "query") for i in range(5)]
    before = {p.pid for p in psutil.Process().children(recursive=True)}
    assert bench.oracle_pool_seconds(jobs, 3) > 0
    after = {p.pid for p in psutil.Process().children(recursive=True)}
    assert after <= before
