"""Host-side logic of bench.py: the single-GPU contract and the counter calibration."""

import json
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _csv(path, counter, rows):
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for disp, name, value in rows:
            f.write(f'{disp},"{name}",{counter},{value}\n')


def test_traffic_calibration(tmp_path, monkeypatch):
    """FETCH_SIZE and WRITE_SIZE readings are summed over a dispatch's instances and scaled by
    what the same counters read for the 1 GiB copy; the record is tied to the kernel digest."""
    kib_gib = float(1 << 20)
    fetch = tmp_path / "fetch.csv"
    write = tmp_path / "write.csv"
    step = "void csc::k_step_batch<csc::Bf16S, unsigned short, 8>(csc::StepBatch)"
    # two instances per dispatch; the copy reads half a GiB of FETCH units and a full GiB of writes
    _csv(fetch, "FETCH_SIZE", [(1, step, 100.0), (1, step, 300.0), (2, step, 500.0), (2, step, 300.0),
                               (3, "__amd_rocclr_copyBuffer", kib_gib / 4), (3, "__amd_rocclr_copyBuffer", kib_gib / 4),
                               (4, "__amd_rocclr_copyBuffer", 10.0)])
    _csv(write, "WRITE_SIZE", [(1, step, 50.0), (2, step, 150.0),
                               (3, "__amd_rocclr_copyBuffer", kib_gib), (4, "__amd_rocclr_copyBuffer", 5.0)])
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "traffic_path", lambda workload: str(out))
    args = types.SimpleNamespace(traffic=[str(fetch), str(write)], probe="bf16sb", headline="bf16sb",
                                 workload="c3")
    bench.traffic_summary(args)
    rec = json.loads(out.read_text())
    # fetch: mean over dispatches 600 KiB raw x 2 (copy calibration); write: 100 KiB x 1
    assert rec["detail"]["bf16sb"]["scale_fetch"] == pytest.approx(2.0)
    assert rec["detail"]["bf16sb"]["scale_write"] == pytest.approx(1.0)
    assert rec["bytes_per_launch"]["bf16sb"] == pytest.approx((600.0 * 2 + 100.0) * 1024)
    assert rec["kernel_sha256_16"] == bench.kernel_digest()
    assert bench.load_traffic(bench.kernel_digest(), "bf16sb") == pytest.approx((600.0 * 2 + 100.0) * 1024)
    assert bench.load_traffic("0" * 16, "bf16sb") is None
