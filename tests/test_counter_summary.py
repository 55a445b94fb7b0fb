"""bench.py's reduction of two rocprofv3 counter files (FETCH_SIZE, then
WRITE_SIZE, KiB per dispatch) to HBM bytes per launch, on synthetic counter
files whose answer is known: each counter is scaled so that the plain 1 GiB
copy that opens the run reads 1 GiB, rows of one dispatch are summed, the
one-stage kernel's stage-1 launches (the first after each finalize launch)
are left out, a two-stage run counts only its two-stage launches, and a
batched run averages the stage launches j >= 2 of its last super-step."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

GIB_KIB = float(1 << 20)
FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def write_counters(path, counter, dispatches):
    """dispatches: (kernel name, KiB) in launch order; a KiB given as a tuple
    is split over several rows of the same dispatch"""
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for d, (name, kib) in enumerate(dispatches, start=1):
            for part in (kib if isinstance(kib, tuple) else (kib,)):
                w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": part})


@pytest.fixture
def tmp_root(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    for fuse in (1, 2, "batch"):
        for f in bench.KERNEL_SOURCES[fuse]:
            os.makedirs(tmp_path / os.path.dirname(f), exist_ok=True)
            (tmp_path / f).write_text("source of %s\n" % f)
    return tmp_path


def one_stage_run(copy_kib, stage_kib):
    """a calibration copy, then two super-steps of three stages each"""
    fill = ("void at::native::vectorized_elementwise_kernel<4, FillFunctor<double>>", 3.0)
    step = [("void rkl::reduce_minmax_kernel<double>(rkl::ReduceLaunch)", 100.0),
            ("void rkl::finalize_kernel(rkl::FinalizeLaunch)", 0.5),
            ("void rkl::stage_kernel<double, true, 1, 1, 16, 16, true>(rkl::StageLaunch)", 7777.0),   # stage 1
            ("void rkl::stage_kernel<double, true, 1, 1, 16, 16, true>(rkl::StageLaunch)", stage_kib[0]),
            ("void rkl::stage_kernel<double, true, 1, 1, 16, 16, true>(rkl::StageLaunch)", stage_kib[1])]
    return [fill, ("__amd_rocclr_copyBuffer", copy_kib)] + step + step


def test_one_stage_launches(tmp_root):
    f, w = tmp_root / "fetch.csv", tmp_root / "write.csv"
    # FETCH reads half the copy's bytes (factor 2), WRITE all of them (factor 1)
    write_counters(f, "FETCH_SIZE", one_stage_run((GIB_KIB / 4, GIB_KIB / 4), (1000.0, 3000.0)))
    write_counters(w, "WRITE_SIZE", one_stage_run(GIB_KIB, (10.0, 30.0)))
    d = bench.summarize_counters(str(f), str(w), "spitzer_256", "fp64", 1, 4)
    assert d["fetch_factor"] == 2.0 and d["write_factor"] == 1.0
    assert d["dispatches"] == [4, 4]                       # stage-1 launches left out
    assert d["read_bytes_per_launch"] == 2.0 * 2000.0 * 1024
    assert d["write_bytes_per_launch"] == 20.0 * 1024
    assert d["bytes_per_launch"] == d["read_bytes_per_launch"] + d["write_bytes_per_launch"]
    assert d["variant"] == 4 and d["kernel_hash"] == bench.kernel_hash(1)
    saved = json.load(open(bench.traffic_path("spitzer_256", "fp64", 1, 4)))
    assert saved == json.loads(json.dumps(d))
    assert bench.traffic_for("spitzer_256", "fp64", 1, 4) == d["bytes_per_launch"]


def test_two_stage_launches(tmp_root):
    seq = [("__amd_rocclr_copyBuffer", GIB_KIB / 2),
           ("void rkl::finalize_kernel(rkl::FinalizeLaunch)", 1.0),
           ("void rkl::stage_kernel<float, true, 1, 1, 64, 4, true>(rkl::StageLaunch)", 5000.0),    # stage 1
           ("void rkl::fused2_kernel<true, 16, 16, 32>(rkl::FusedLaunch)", 600.0),
           ("void rkl::fused2_kernel<true, 16, 16, 32>(rkl::FusedLaunch)", 800.0),
           ("void rkl::stage_kernel<float, true, 1, 1, 64, 4, true>(rkl::StageLaunch)", 5000.0)]   # last stage
    f, w = tmp_root / "fetch.csv", tmp_root / "write.csv"
    write_counters(f, "FETCH_SIZE", seq)
    write_counters(w, "WRITE_SIZE", seq)
    d = bench.summarize_counters(str(f), str(w), "fused_768", "mixed", 2, 8)
    assert d["dispatches"] == [2, 2]
    assert d["read_bytes_per_launch"] == 2.0 * 700.0 * 1024
    assert d["write_bytes_per_launch"] == 2.0 * 700.0 * 1024


def test_batched_launches(tmp_root):
    st = "void rkl::batch_stage_kernel<float, 1, 1>(rkl::BatchLaunch)"
    red = "void rkl::batch_reduce_kernel<float>(rkl::BatchReduceLaunch)"
    seq = [("__amd_rocclr_copyBuffer", GIB_KIB),
           (red, 1.0), (st, 9000.0), (st, 9000.0), (st, 9000.0),      # graph replays: not counted
           (red, 1.0), (st, 4000.0), (st, 100.0), (st, 300.0), (st, 200.0)]
    f, w = tmp_root / "fetch.csv", tmp_root / "write.csv"
    write_counters(f, "FETCH_SIZE", seq)
    write_counters(w, "WRITE_SIZE", seq)
    d = bench.summarize_counters(str(f), str(w), "patches_2000", "mixed", "batch", 1)
    assert d["fetch_factor"] == 1.0 and d["dispatches"] == [3, 3]
    assert d["read_bytes_per_launch"] == 200.0 * 1024
    assert os.path.basename(bench.traffic_path("patches_2000", "mixed", "batch", 1)) == \
        "batch_stage_kernel_patches_2000_mixed_p1_traffic.json"


def test_missing_calibration_copy(tmp_root):
    seq = [("void rkl::finalize_kernel(rkl::FinalizeLaunch)", 1.0),
           ("void rkl::stage_kernel<double, true, 1, 1, 16, 16, true>(rkl::StageLaunch)", 10.0),
           ("void rkl::stage_kernel<double, true, 1, 1, 16, 16, true>(rkl::StageLaunch)", 10.0)]
    f = tmp_root / "fetch.csv"
    write_counters(f, "FETCH_SIZE", seq)
    with pytest.raises(SystemExit, match="copy-calibration"):
        bench.summarize_counters(str(f), str(f), "spitzer_256", "fp64", 1, 4)
