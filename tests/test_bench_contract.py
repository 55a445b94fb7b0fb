"""bench.py's host-side contract on the CPU: one GPU only, algorithmic bytes
per cell-stage, and HBM traffic figures used only for the kernel source,
stencil variant (or batched tile policy) they were measured on."""
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


def test_counter_summary_needs_the_variant():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--counters-summary", "a", "b"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "--variant" in r.stderr
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "patches_2000",
                        "--counters-summary", "a", "b"], capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "--policy" in r.stderr


def test_algorithmic_bytes():
    # stage j >= 2: Y_{j-1}, Y_{j-2}, Y0 (8 B each), tau M(Y0) and 3 b components
    # (8 B each in FP64, 4 B in mixed precision), one 8 B write
    assert bench.bytes_per_cell_stage("fp64", 1) == 8 * 3 + 8 + 24 + 8 == 64
    assert bench.bytes_per_cell_stage("mixed", 1) == 8 * 3 + 4 + 12 + 8 == 48
    assert bench.bytes_per_cell_stage("mixed", 2) == (8 * 3 + 4 + 12 + 2 * 8) / 2 == 28


def test_traffic_is_keyed_by_source_and_variant(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    for fuse in (1, 2, "batch"):
        for f in bench.KERNEL_SOURCES[fuse]:
            os.makedirs(tmp_path / os.path.dirname(f), exist_ok=True)
            (tmp_path / f).write_text("source of %s\n" % f)
    path = bench.traffic_path("spitzer_256", "fp64", 1, 6)
    assert os.path.basename(path) == "stage_kernel_spitzer_256_fp64_v6_traffic.json"
    assert os.path.basename(bench.traffic_path("patches_2000_fp64", "fp64", "batch", 0)) == \
        "batch_stage_kernel_patches_2000_fp64_p0_traffic.json"
    good = {"kernel_hash": bench.kernel_hash(1), "variant": 6, "bytes_per_launch": 1.5e9}
    with open(path, "w") as f:
        json.dump(good, f)
    assert bench.traffic_for("spitzer_256", "fp64", 1, 6) == 1.5e9
    assert bench.traffic_for("spitzer_256", "fp64", 1, 4) is None          # another variant: no file
    with open(path, "w") as f:
        json.dump(dict(good, variant=4), f)
    assert bench.traffic_for("spitzer_256", "fp64", 1, 6) is None          # file of another variant
    with open(path, "w") as f:
        json.dump(dict(good, kernel_hash="0" * 16), f)
    assert bench.traffic_for("spitzer_256", "fp64", 1, 6) is None          # stale source
    with open(path, "w") as f:
        f.write("{not json")
    assert bench.traffic_for("spitzer_256", "fp64", 1, 6) is None


@pytest.mark.parametrize("name", sorted(f for f in os.listdir(os.path.join(ROOT, "profiles"))
                                        if f.endswith("_traffic.json")))
def test_committed_traffic_files_are_well_formed(name):
    d = json.load(open(os.path.join(ROOT, "profiles", name)))
    kind = "p" if d["kernel"] == "batch_stage_kernel" else "v"
    assert name.endswith("_%s%d_traffic.json" % (kind, d["variant"]))
    assert d["bytes_per_launch"] == pytest.approx(d["read_bytes_per_launch"] + d["write_bytes_per_launch"])
    # request counters of a 1 GiB streaming copy count 1 GiB each way
    assert 0.99 < d["calibration_copy_read_over_1GiB"] < 1.01
    assert 0.99 < d["calibration_copy_write_over_1GiB"] < 1.01
    # taken on the current kernel sources (else bench.py reports no traffic)
    fuse = {"stage_kernel": 1, "fused_kernel": 2, "batch_stage_kernel": "batch"}[d["kernel"]]
    assert d["kernel_hash"] == bench.kernel_hash(fuse)
