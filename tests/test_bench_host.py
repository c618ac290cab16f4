"""Host-side checks of bench.py (no GPU): the one-GPU contract, the byte
model and the counter-record lookup that fills roofline.traffic."""
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
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_of_the_headline_workload():
    # 48^3 elements, N = 7: n_L = 110592 * 512, n_u = 337^3
    assert bench.bytes_ax_gs(110592 * 512, 337 ** 3) == 3_556_765_456


def test_kernel_names_follow_the_tile():
    t = {"elements_per_block": 2, "grid_cap": 0, "xcd_remap": 0, "pipeline": 0}
    assert bench.kernel_name(t, 7) == "k_ax<8,double,ATOMIC,double,8>"
    assert bench.kernel_name({**t, "pipeline": 1}, 7) == "k_ax<8,double,ATOMIC,double,2>"


def test_traffic_record_matches_only_current_source_and_tile(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    tile = {"elements_per_block": 2, "grid_cap": 0, "xcd_remap": 0, "pipeline": 0}
    rec = {"workload": "box48_N7", "kernel": "k_ax<8,double,ATOMIC,double,8>", "tile": tile,
           "source_sha256": bench.source_digest(), "hbm_bytes_per_launch": 123}
    (prof / "x.md").write_text("# summary\n\ntraffic-record: %s\n" % json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the digest is taken from the library source under ROOT: mirror it
    src = tmp_path / "paper_2207_07098_amd" / "csrc"
    src.mkdir(parents=True)
    with open(os.path.join(ROOT, "paper_2207_07098_amd", "csrc", "sem_kernels.hip"), "rb") as f:
        (src / "sem_kernels.hip").write_bytes(f.read())
    assert bench.recorded_traffic("box48_N7", rec["kernel"], tile)[0] == 123
    assert bench.recorded_traffic("box48_N7", rec["kernel"], {**tile, "pipeline": 1})[0] is None
    assert bench.recorded_traffic("ogrid_N7", rec["kernel"], tile)[0] is None
    (src / "sem_kernels.hip").write_bytes(b"changed")
    assert bench.recorded_traffic("box48_N7", rec["kernel"], tile)[0] is None
