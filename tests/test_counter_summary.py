"""bench.py's reduction of two rocprofv3 counter files to HBM bytes per
launch, on synthetic counter files whose answer is known: read bytes are
the read requests by size (32, 64, 128 B), write bytes the 64-byte write
requests times 64 plus the others times 32; rows of one dispatch are
summed; the library's 1 GiB streaming copy that opens the run is recorded
as a check (its counted bytes over 1 GiB); the one-stage kernel's stage-1
launches (the first after each finalize launch) are left out, a two-stage
run counts only its two-stage launches, and a batched run averages the
stage launches j >= 2 of its last super-step."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

GIB = float(1 << 30)
FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
COPY = "void (anonymous namespace)::copy_kernel<double>(double const*, double*, long)"


def write_reads(path, dispatches):
    """dispatches: (kernel name, bytes); each dispatch's bytes are written as
    128-byte, 64-byte and 32-byte request counts (a half, a quarter and a
    quarter of the bytes), the 128-byte count split over two rows"""
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for d, (name, nbytes) in enumerate(dispatches, start=1):
            for c, v in (("TCC_EA0_RDREQ_128B_sum", nbytes / 4 / 128), ("TCC_EA0_RDREQ_128B_sum", nbytes / 4 / 128),
                         ("TCC_EA0_RDREQ_64B_sum", nbytes / 4 / 64), ("TCC_EA0_RDREQ_32B_sum", nbytes / 4 / 32),
                         ("SQ_WAVES", 12345.0)):
                w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": c, "Counter_Value": v})


def write_writes(path, dispatches):
    """(kernel name, bytes): three quarters in 64-byte requests, a quarter in
    32-byte ones (TCC_EA0_WRREQ counts both)"""
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for d, (name, nbytes) in enumerate(dispatches, start=1):
            n64, n32 = 0.75 * nbytes / 64, 0.25 * nbytes / 32
            for c, v in (("TCC_EA0_WRREQ_sum", n64 + n32), ("TCC_EA0_WRREQ_64B_sum", n64)):
                w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": c, "Counter_Value": v})


@pytest.fixture
def tmp_root(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    for fuse in (1, 2, "batch"):
        for f in bench.KERNEL_SOURCES[fuse]:
            os.makedirs(tmp_path / os.path.dirname(f), exist_ok=True)
            (tmp_path / f).write_text("source of %s\n" % f)
    return tmp_path


def one_stage_run(copy_bytes, stage_bytes):
    """a calibration copy, then two super-steps of three stages each"""
    fill = ("void at::native::vectorized_elementwise_kernel<4, FillFunctor<double>>", 4096.0)
    step = [("void rkl::reduce_minmax_kernel(double const*, long, double*)", 8192.0),
            ("void rkl::finalize_kernel(double const*, int, rkl::GridConst, ...)", 1024.0),
            ("void rkl::stage_kernel<double, true, 1, 1, 16, 16, true>(rkl::StageLaunch)", 777.0 * 1024),   # stage 1
            ("void rkl::stage_kernel<double, true, 1, 1, 16, 16, true>(rkl::StageLaunch)", stage_bytes[0]),
            ("void rkl::stage_kernel<double, true, 1, 1, 16, 16, true>(rkl::StageLaunch)", stage_bytes[1])]
    return [fill, (COPY, copy_bytes)] + step + step


def test_one_stage_launches(tmp_root):
    r, w = tmp_root / "read.csv", tmp_root / "write.csv"
    write_reads(r, one_stage_run(GIB, (1024.0 * 1000, 1024.0 * 3000)))
    write_writes(w, one_stage_run(1.5 * GIB, (1024.0 * 10, 1024.0 * 30)))
    d = bench.summarize_counters(str(r), str(w), "spitzer_256", "fp64", 1, 4)
    assert d["calibration_copy_read_over_1GiB"] == 1.0 and d["calibration_copy_write_over_1GiB"] == 1.5
    assert d["dispatches"] == [4, 4]                       # stage-1 launches left out
    assert d["read_bytes_per_launch"] == 2000.0 * 1024
    assert d["write_bytes_per_launch"] == 20.0 * 1024
    assert d["bytes_per_launch"] == d["read_bytes_per_launch"] + d["write_bytes_per_launch"]
    assert d["variant"] == 4 and d["kernel_hash"] == bench.kernel_hash(1)
    saved = json.load(open(bench.traffic_path("spitzer_256", "fp64", 1, 4)))
    assert saved == json.loads(json.dumps(d))
    assert bench.traffic_for("spitzer_256", "fp64", 1, 4) == d["bytes_per_launch"]


def test_two_stage_launches(tmp_root):
    seq = [(COPY, GIB),
           ("void rkl::finalize_kernel(double const*, int, rkl::GridConst, ...)", 1024.0),
           ("void rkl::stage_kernel<float, true, 1, 1, 64, 4, true>(rkl::StageLaunch)", 5000.0 * 1024),   # stage 1
           ("void rkl::fused_kernel<true, 1, 1, 16, 16, 2>(rkl::FusedLaunch)", 600.0 * 1024),
           ("void rkl::fused_kernel<true, 1, 1, 16, 16, 2>(rkl::FusedLaunch)", 800.0 * 1024),
           ("void rkl::stage_kernel<float, true, 1, 1, 64, 4, true>(rkl::StageLaunch)", 5000.0 * 1024)]  # last stage
    r, w = tmp_root / "read.csv", tmp_root / "write.csv"
    write_reads(r, seq)
    write_writes(w, seq)
    d = bench.summarize_counters(str(r), str(w), "fused_768", "mixed", 2, 8)
    assert d["dispatches"] == [2, 2]
    assert d["read_bytes_per_launch"] == 700.0 * 1024
    assert d["write_bytes_per_launch"] == 700.0 * 1024


def test_batched_launches(tmp_root):
    st = "void rkl::batch_stage_kernel<float, true, 0, 1>(rkl::BatchBufs, int2 const*, int)"
    red = "void rkl::batch_reduce_kernel(rkl::BatchGrid const*, ...)"
    seq = [(COPY, GIB),
           (red, 1024.0), (st, 9000.0 * 1024), (st, 9000.0 * 1024), (st, 9000.0 * 1024),   # graph replays: not counted
           (red, 1024.0), (st, 4000.0 * 1024), (st, 100.0 * 1024), (st, 300.0 * 1024), (st, 200.0 * 1024)]
    r, w = tmp_root / "read.csv", tmp_root / "write.csv"
    write_reads(r, seq)
    write_writes(w, seq)
    d = bench.summarize_counters(str(r), str(w), "patches_2000", "mixed", "batch", 1)
    assert d["dispatches"] == [3, 3]
    assert d["read_bytes_per_launch"] == 200.0 * 1024
    assert os.path.basename(bench.traffic_path("patches_2000", "mixed", "batch", 1)) == \
        "batch_stage_kernel_patches_2000_mixed_p1_traffic.json"


def test_missing_calibration_copy(tmp_root):
    seq = [("void rkl::finalize_kernel(double const*, int, rkl::GridConst, ...)", 1024.0),
           ("void rkl::stage_kernel<double, true, 1, 1, 16, 16, true>(rkl::StageLaunch)", 10.0 * 1024),
           ("void rkl::stage_kernel<double, true, 1, 1, 16, 16, true>(rkl::StageLaunch)", 10.0 * 1024)]
    r = tmp_root / "read.csv"
    write_reads(r, seq)
    with pytest.raises(SystemExit, match="calibration copy"):
        bench.summarize_counters(str(r), str(r), "spitzer_256", "fp64", 1, 4)
