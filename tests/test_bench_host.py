"""Host-side logic of bench.py (no GPU): the algorithmic byte count behind the
roofline, the counter summary that writes the traffic record, the guard that
drops a traffic record taken from other kernel sources, and the one-GPU
refusal of ``--gpus N``."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_of_one_launch():
    # pixels read and written once, r int32 + r float32 words per 8x8 tile,
    # one 8-byte error energy per image
    b, h, w, r = 3, 16, 40, 10
    tiles = b * (h // 8) * (w // 8)
    assert bench.algorithmic_bytes(b, h, w, r) == b * h * w * 2 + tiles * r * 8 + b * 8
    # the C1 launch at r = 64 moves 42.95 GB
    assert round(bench.algorithmic_bytes(1024, 2048, 2048, 64) / 1e9, 2) == 42.95


def write_pmc(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        wr = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        wr.writeheader()
        for name, value in rows:
            wr.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_pmc_summary_scales_by_the_copy_and_guards_the_digest(tmp_path, monkeypatch):
    traffic = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(traffic))
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctor_add<float>>"
    fused = "void adct::compress8<1, 0, 10, false>(adct::PassParams)"
    kib = bench.COPY_BYTES / 1024.0
    # the copy kernel's counters read 2x (fetch) and 1x (write) its bytes
    write_pmc(tmp_path / "f", "FETCH_SIZE", [(copy, 2 * kib), (fused, 1000.0), (fused, 1002.0)])
    write_pmc(tmp_path / "w", "WRITE_SIZE", [(copy, kib), (fused, 3000.0)])
    bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"))
    rec = json.loads(traffic.read_text())
    assert rec["fetch_scale"] == pytest.approx(0.5) and rec["write_scale"] == pytest.approx(1.0)
    k = rec["kernels"][fused]
    assert k["fetch_bytes"] == pytest.approx(1001.0 * 1024 * 0.5)
    assert k["write_bytes"] == pytest.approx(3000.0 * 1024)
    assert rec["source_digest"] == bench.kernel_source_digest()
    assert bench.measured_traffic() == pytest.approx(k["fetch_bytes"] + k["write_bytes"])
    # a record of other kernel sources is not used
    rec["source_digest"] = "0" * 16
    traffic.write_text(json.dumps(rec))
    assert bench.measured_traffic() is None


def test_committed_traffic_record_is_close_to_the_algorithmic_bytes():
    """The committed counter summary of the fused 8x8 launches: copy scales
    near 2 (fetch) and 1 (write), and per-launch traffic within a few percent
    of the algorithmic bytes of the r sweep it was taken on."""
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    assert 1.9 < rec["fetch_scale"] < 2.1 and 0.95 < rec["write_scale"] < 1.05
    for name, k in rec["kernels"].items():
        r = int(name.split("compress8<")[1].split(",")[2])
        alg = bench.algorithmic_bytes(1024, 2048, 2048, r)
        assert 0.98 < (k["fetch_bytes"] + k["write_bytes"]) / alg < 1.05, name


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stdout
