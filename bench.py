#!/usr/bin/env python3
"""Benchmark of the RKL2 anisotropic-conduction super-step on one MI355X.

One step = one full RKL2 super-step (temperature reduction, dt_par and stage
count on the device, then s stencil/stage launches) over the whole grid.
Default workload: 256^3 periodic grid, FP64, tangled k^-11/3 field, kappa_par
= T^2.5, kappa_perp = 1e-3 kappa_par, MC-limited transverse gradients,
dt_hyp chosen for s = 16.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
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
    # name: (builder, flux precision, algorithmic bytes per cell-stage of the stage kernel)
    "spitzer_256": ("spitzer_256", "fp64", 64),
    "spitzer_256_mixed": ("spitzer_256", "mixed", 48),
    "saturated_512": ("saturated_512", "mixed", 48),
    "saturated_512_fp64": ("saturated_512", "fp64", 64),
}
KERNEL_SOURCES = ["paper_1702_05487_amd/csrc/rkl_tile.h", "paper_1702_05487_amd/csrc/rkl_kernels.hip"]


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(name, precision):
    """HBM bytes per stage-kernel launch from committed rocprofv3 counter runs,
    if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "stage_kernel_%s_%s_traffic.json" % (name, precision))
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(w, s, dt):
    """The oracle, untuned, on a bounded sample of the same workload: one
    super-step (s stages) of a 256 x 256 x 16 periodic slab cut from the same
    fields, on one host core."""
    import numpy as np
    import oracle
    nz = 16
    T = np.ascontiguousarray(w.T[:nz])
    b = np.ascontiguousarray(w.b[:, :nz])
    g = oracle.Grid(n=(w.n[0], w.n[1], nz), h=w.h, ndim=3, **w.params)
    t0 = time.perf_counter()
    oracle.rkl2_fixed(g, T, b, s, dt)
    sec = time.perf_counter() - t0
    cells = w.n[0] * w.n[1] * nz
    return {"value": cells * s / sec, "unit": "cell-stage/s", "cores": 1, "kind": "oracle",
            "sample": "one %d-stage super-step of a %dx%dx%d periodic slab of the same fields "
                      "(%.1f s serial)" % (s, w.n[0], w.n[1], nz, sec)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="spitzer_256", choices=sorted(WORKLOADS))
    ap.add_argument("--variant", type=int, default=-1)
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

    builder, precision, bytes_per_cs = WORKLOADS[args.workload]
    rkl.load(build_if_missing=True)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = getattr(inputs, builder)()
    dev = torch.device("cuda:0")
    plan = rkl.Plan([rkl.grid_desc(w.n, w.h, ndim=3, **w.params)], precision=precision, variant=args.variant)
    T0 = torch.from_numpy(w.T).to(dev)
    bdev = torch.from_numpy(w.b).to(dev, dtype=torch.float32 if precision == "mixed" else torch.float64)
    T = T0.clone()
    dt = w.ratio * plan.dt_par(T)     # the library's own dt_par of the initial field
    cells = w.cells

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
    ms, launches, cell_stages = rkl.rkl_profile_read(plan.handle)
    rkl.rkl_profile(plan.handle, 0)
    s_last = plan.query()[0]

    avg_launch_s = ms / 1e3 / launches
    bytes_per_launch = bytes_per_cs * cells
    achieved = bytes_per_launch / avg_launch_s / 1e9
    traffic = traffic_for(args.workload, precision)
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
            "variant": args.variant,
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
            "kernel": "stage_kernel (stage j>=2)", "bytes_per_cell_stage": bytes_per_cs,
            "avg_launch_ms": avg_launch_s * 1e3, "launches": launches,
            "kernel_cell_stage_per_s": cell_stages / (ms / 1e3),
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, s_last, dt)
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
