"""Host logic of bench.py that needs no GPU: the one-GPU guard and the
HBM-traffic digest of rocprofv3 counter files (scaling by a plain copy)."""
import csv
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


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


@pytest.mark.parametrize("kind,kernel", [("fused", "void xy::k_or2_f32<0, 3, true>(xy::SweepArgs)"),
                                         ("half", "void xy::k_tile_f32<1, false, 3, 1, false>(xy::SweepArgs)"),
                                         ("metro", "void xy::k_tile_f32<0, false, 5, 1, true>(xy::SweepArgs)")])
def test_traffic_digest_scales_by_the_copy(tmp_path, monkeypatch, kind, kernel):
    out = tmp_path / f"traffic_{kind}.json"
    monkeypatch.setattr(bench, "traffic_path", lambda k: str(out))
    fetch, write = tmp_path / "fetch.csv", tmp_path / "write.csv"
    # the copy reads COPY_BYTES: 524288 units of 2048 bytes; the kernel 3 and 5 units
    _counter_csv(fetch, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 524288.0), (kernel, 3.0), (kernel, 5.0),
                                       ("xy::k_tick(xy::Ctl*)", 1.0)])
    _counter_csv(write, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 1048576.0), (kernel, 10.0), (kernel, 10.0)])
    bench.digest_traffic(str(fetch), str(write))
    d = json.load(open(out))
    assert d["kernel"] == kind
    assert d["fetch_scale_bytes_per_unit"] == pytest.approx(2048.0)
    assert d["write_scale_bytes_per_unit"] == pytest.approx(1024.0)
    assert d["fetch_bytes_per_launch"] == pytest.approx(4.0 * 2048)
    assert d["write_bytes_per_launch"] == pytest.approx(10.0 * 1024)
    assert d["hbm_bytes_per_launch"] == pytest.approx(4.0 * 2048 + 10.0 * 1024)
    assert d["kernel_source_hash"] == bench.kernel_source_hash()
    per_update = bench.BYTES_PER_UPDATE_F32 * bench.R * bench.L ** 3
    assert d["algorithmic_bytes_per_launch"] == pytest.approx(per_update if kind == "fused" else per_update / 2)
    # the bench reports the digest only for the kernel source it was taken on
    assert bench.load_traffic(bench.kernel_source_hash(), kind) == pytest.approx(d["hbm_bytes_per_launch"])
    assert bench.load_traffic("0" * 16, kind) is None


def test_traffic_digest_rejects_files_without_the_copy(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "traffic_path", lambda k: str(tmp_path / "t.json"))
    fetch, write = tmp_path / "fetch.csv", tmp_path / "write.csv"
    kernel = "void xy::k_or2_f32<0, 3>(xy::SweepArgs)"
    _counter_csv(fetch, "FETCH_SIZE", [(kernel, 3.0)])
    _counter_csv(write, "WRITE_SIZE", [(kernel, 3.0)])
    with pytest.raises(SystemExit):
        bench.digest_traffic(str(fetch), str(write))


def test_cpu_model_and_oracle_run_timing():
    """The host description and the single-core timing helper of the CPU
    baseline (a tiny oracle run)."""
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()
    updates, secs = bench._oracle_run((4, [0.3, 0.4], 3, 2, 1, 1, 1))
    assert updates == 2 * 4 ** 3 * 2 * 2 and secs > 0
