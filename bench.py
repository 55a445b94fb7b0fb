#!/usr/bin/env python3
"""Benchmark of the RKL2 anisotropic-conduction super-step on one MI355X.

One step = one full RKL2 super-step (temperature reduction, dt_par and stage
count on the device, then s stencil/stage launches) over the whole grid.
Default workload: 256^3 periodic grid, FP64, tangled k^-11/3 field, kappa_par
= T^2.5, kappa_perp = 1e-3 kappa_par, MC-limited transverse gradients,
dt_hyp chosen for s = 16.  Prints one JSON line.

The stencil kernel variant (tile shape, z-chunk, stages per launch) is picked
by the library's autotuner on the workload's own fields before the timed
region, unless --variant is given.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--variant V] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
WORKLOADS = {
    # name: (builder, flux precision)
    "spitzer_256": ("spitzer_256", "fp64"),
    "spitzer_256_mixed": ("spitzer_256", "mixed"),
    "saturated_512": ("saturated_512", "mixed"),
    "saturated_512_fp64": ("saturated_512", "fp64"),
    "fused_768": ("fused_768", "mixed"),
}
KERNEL_SOURCES = {
    1: ["paper_1702_05487_amd/csrc/rkl_tile.h", "paper_1702_05487_amd/csrc/rkl_kernels.hip"],
    2: ["paper_1702_05487_amd/csrc/rkl_tile.h", "paper_1702_05487_amd/csrc/rkl_fused.h",
        "paper_1702_05487_amd/csrc/rkl_fused.hip"],
}
KERNEL_NAMES = {1: "stage_kernel", 2: "fused2_kernel"}


def bytes_per_cell_stage(precision, fuse):
    """Algorithmic HBM bytes per cell and stage of the dominant kernel.
    One stage j >= 2 reads Y_{j-1}, Y_{j-2}, Y0 (FP64), tau M(Y0) and the
    three components of b (FP64, or FP32 in mixed precision) and writes Y_j:
    64 B (FP64) or 48 B (mixed).  A two-stage launch reads the same inputs
    once and writes Y_j and Y_{j+1}: 56 B per cell for two stages."""
    if fuse == 2:
        return 28.0
    return 64.0 if precision == "fp64" else 48.0


def kernel_hash(fuse):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[fuse]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(name, precision, fuse):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3
    counter runs, if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "%s_%s_%s_traffic.json" % (KERNEL_NAMES[fuse], name, precision))
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_hash(fuse):
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(w, T0, b, s, dt):
    """The oracle, untuned, on a bounded sample of the same workload: one
    super-step (s stages) of a 256 x 256 x 16 periodic slab cut from the same
    fields, on one host core."""
    import numpy as np
    import oracle
    nz = 16
    m = 256
    T = np.ascontiguousarray(T0[:nz, :m, :m].cpu().numpy())
    b = np.ascontiguousarray(b[:, :nz, :m, :m].double().cpu().numpy())
    g = oracle.Grid(n=(m, m, nz), h=w.h, ndim=3, **w.params)
    t0 = time.perf_counter()
    oracle.rkl2_fixed(g, T, b, s, dt)
    sec = time.perf_counter() - t0
    cells = m * m * nz
    return {"value": cells * s / sec, "unit": "cell-stage/s", "cores": 1, "kind": "oracle",
            "sample": "one %d-stage super-step of a %dx%dx%d periodic slab cut from the same fields "
                      "(%.1f s serial)" % (s, m, m, nz, sec)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="spitzer_256", choices=sorted(WORKLOADS))
    ap.add_argument("--variant", type=int, default=-1, help="kernel variant; -1 = autotune")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 1 GiB device-to-device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import oracle
    from paper_1702_05487_amd import inputs, rkl

    builder, precision = WORKLOADS[args.workload]
    rkl.load(build_if_missing=True)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    dev = torch.device("cuda:0")
    w = getattr(inputs, builder)(device=dev)       # fields generated on the GPU
    plan = rkl.Plan([rkl.grid_desc(w.n, w.h, ndim=3, **w.params)], precision=precision)
    T0 = w.T
    bdev = w.b.to(dtype=torch.float32 if precision == "mixed" else torch.float64)
    w.b = None
    T = T0.clone()
    dt = w.ratio * plan.dt_par(T)     # the library's own dt_par of the initial field
    cells = w.cells
    tuned_ms = None
    if args.variant >= 0:
        plan.set_variant(args.variant)
        variant = args.variant
    else:
        variant, tuned_ms = rkl.rkl_autotune(plan.handle, 0, *plan._tb(0, T, bdev), dt, 2,
                                             rkl.ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    tile = rkl.rkl_variant_info(variant)
    fuse = tile[3]
    bytes_per_cs = bytes_per_cell_stage(precision, fuse)

    for _ in range(args.warmup):
        plan.superstep(T, bdev, dt)
    T.copy_(T0)
    torch.cuda.synchronize()
    rkl.rkl_profile(plan.handle, 1)
    stages = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stages += plan.superstep(T, bdev, dt)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    ms, launches, cell_stages = rkl.rkl_profile_read(plan.handle, fuse)
    rkl.rkl_profile(plan.handle, 0)
    s_last = plan.query()[0]

    avg_launch_s = ms / 1e3 / launches
    bytes_per_launch = bytes_per_cs * cells * fuse
    achieved = bytes_per_launch / avg_launch_s / 1e9
    traffic = traffic_for(args.workload, precision, fuse)
    out = {
        "metric": "cell-stage updates/s",
        "value": cells * stages / sec,
        "unit": "cell-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32 flux + f64 recurrence",
        "data": "synthetic",
        "config": {
            "workload": w.name, "grid": list(w.n), "stages": s_last, "precision": precision,
            "kappa_par": "T^2.5", "kperp_ratio": w.params["kperp_ratio"],
            "limiter": "MC" if w.params["limiter"] else "mean", "saturation": bool(w.params["saturation"]),
            "variant": variant, "tile": list(tile[:3]), "stages_per_launch": fuse,
            "autotuned_ms_per_step": tuned_ms,
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
            "kernel": "%s (stages j>=2)" % KERNEL_NAMES[fuse], "bytes_per_cell_stage": bytes_per_cs,
            "avg_launch_ms": avg_launch_s * 1e3, "launches": launches,
            "kernel_cell_stage_per_s": cell_stages / (ms / 1e3),
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, T0, bdev, s_last, dt)
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
