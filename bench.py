#!/usr/bin/env python3
"""Benchmark of the RKL2 anisotropic-conduction super-step on one MI355X.

One step = one full RKL2 super-step (temperature reduction, dt_par and stage
count on the device, then s stencil/stage launches) over the whole grid.
Default workload: 256^3 periodic grid, FP64, tangled k^-11/3 field, kappa_par
= T^2.5, kappa_perp = 1e-3 kappa_par, MC-limited transverse gradients,
dt_hyp chosen for s = 16.  Prints one JSON line.

The stencil kernel variant (tile shape, z-chunk, stages per launch) is picked
by the library's autotuner on the workload's own fields before the timed
region, unless --variant is given; for the batched patch workloads the tile
policy likewise, unless --policy is given.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--variant V] [--policy P]
                  [--no-cpu-baseline]
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
    "saturated_512_upwind": ("saturated_512_upwind", "mixed"),
    "fused_768": ("fused_768", "mixed"),
    "fused_768_fp64": ("fused_768", "fp64"),   # the 768^3 workload in FP64 (one-stage kernels only)
    "patches_2000": ("patch_set", "mixed"),   # batched, graph-captured
    "patches_2000_fp64": ("patch_set", "fp64"),   # the same, FP64 throughout
    "patches_2000_fp64_loop": ("patch_set", "fp64"),   # plain FP64: one rkl_superstep per patch
    "spitzer_256_subcycle": ("spitzer_256", "fp64"),   # explicit sub-cycling over the same dt_hyp
}
KERNEL_SOURCES = {
    1: ["paper_1702_05487_amd/csrc/rkl_tile.h", "paper_1702_05487_amd/csrc/rkl_kernels.hip"],
    2: ["paper_1702_05487_amd/csrc/rkl_tile.h", "paper_1702_05487_amd/csrc/rkl_fused.h",
        "paper_1702_05487_amd/csrc/rkl_fused.hip"],
    "batch": ["paper_1702_05487_amd/csrc/rkl_tile.h", "paper_1702_05487_amd/csrc/rkl_batch.hip"],
}
KERNEL_NAMES = {1: "stage_kernel", 2: "fused2_kernel", "batch": "batch_stage_kernel"}


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


def traffic_path(name, precision, fuse, variant):
    """profiles/<kernel>_<workload>[_<precision>]_<v|p><n>_traffic.json: the
    counters of one stencil variant (v) or batched tile policy (p); the
    precision is left out where the workload's name already ends with it"""
    tag = name if name.endswith("_" + precision) else "%s_%s" % (name, precision)
    kind = "p" if fuse == "batch" else "v"
    return os.path.join(ROOT, "profiles", "%s_%s_%s%d_traffic.json" % (KERNEL_NAMES[fuse], tag, kind, variant))


def traffic_for(name, precision, fuse, variant):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3
    counter runs, if they were taken on the current kernel source with the
    same variant (or batched tile policy)."""
    path = traffic_path(name, precision, fuse, variant)
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_hash(fuse) or d.get("variant") != variant:
        return None
    return d.get("bytes_per_launch")


def summarize_counters(fetch_csv, write_csv, workload, precision, fuse, variant):
    """HBM bytes per launch of the dominant kernel from two rocprofv3 --pmc
    runs of this script with --copy-calibration (FETCH_SIZE, then
    WRITE_SIZE; KiB per dispatch).  Each counter is scaled by the factor that
    makes it read 1 GiB for the plain 1 GiB device copy that starts the
    calibration run.  Stage-1 launches (the first stencil launch after each finalize
    launch) are left out: the measured kernel is stages j >= 2.  For the
    batched workload (fuse "batch") the launches are the stage launches j >= 2
    of the last, eagerly launched super-step, and the figure is their average
    per launch, like the roofline's.  `variant` is the stencil variant (or
    batched tile policy) the counter runs used.  Writes the JSON that
    traffic_for reads and returns it."""
    import csv

    def per_dispatch(path, counter):
        out = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            d = int(r["Dispatch_Id"])
            name, v = out.get(d, (r["Kernel_Name"], 0.0))
            out[d] = (name, v + float(r["Counter_Value"]))
        return out

    def measured(disp):
        # the calibration copy is the run's first device copy
        copies = [disp[d][1] for d in sorted(disp) if "copyBuffer" in disp[d][0]]
        if not copies:
            raise SystemExit("no copy-calibration dispatch in the counter file")
        vals, after_finalize = [], False
        if fuse == "batch":
            # the last (eager) batched super-step: its stage launches after the
            # last reduce launch, stage 1 left out
            last = max(d for d in disp if "batch_reduce" in disp[d][0])
            vals = [disp[d][1] for d in sorted(disp) if d > last and KERNEL_NAMES[fuse] in disp[d][0]][1:]
        for d in sorted(disp) if fuse != "batch" else []:
            name, v = disp[d]
            if "finalize_kernel" in name:
                after_finalize = True
                continue
            if KERNEL_NAMES[fuse] in name:
                if not (fuse == 1 and after_finalize):
                    vals.append(v)
                after_finalize = False
        if not vals:
            raise SystemExit("no %s dispatch in the counter file" % KERNEL_NAMES[fuse])
        return sum(vals) / len(vals), copies[0], len(vals)

    f_k, f_copy, nf = measured(per_dispatch(fetch_csv, "FETCH_SIZE"))
    w_k, w_copy, nw = measured(per_dispatch(write_csv, "WRITE_SIZE"))
    gib_kib = float(1 << 20)
    ff, wf = gib_kib / f_copy, gib_kib / w_copy
    rd, wr = f_k * ff * 1024.0, w_k * wf * 1024.0
    d = {"kernel": KERNEL_NAMES[fuse], "workload": workload, "precision": precision,
         "kernel_hash": kernel_hash(fuse), "variant": variant, "fetch_factor": ff, "write_factor": wf,
         "read_bytes_per_launch": rd, "write_bytes_per_launch": wr, "bytes_per_launch": rd + wr,
         "dispatches": [nf, nw]}
    with open(traffic_path(workload, precision, fuse, variant), "w") as fh:
        json.dump(d, fh, indent=1)
        fh.write("\n")
    return d


def copy_ceiling(torch):
    """Bandwidth of a plain 1 GiB device-to-device copy (read + write bytes
    per second), measured on the same GPU for reference."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 5 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    return gbs


def bench_batched(args, torch, inputs, rkl, precision="mixed", loop=False):
    """2000 independent periodic patches (edges log-uniform in [16, 64], own
    fields, dt_hyp for s_p uniform in [4, 40]), one super-step of all of them
    per step.  Batched form: the captured HIP graph of rkl_superstep_batched
    replayed, with the batched tile policy picked by the autotuner first; its
    roofline comes from the same launches run eagerly right after the timed
    replays, each stage launch of j >= 2 timed with HIP events.  Loop form
    (plain, FP64): the host calls rkl_superstep once per patch, with the
    one-grid stencil variant the autotuner picks on the largest patch; its
    roofline comes from one more super-step of every patch from the initial
    fields, after the timed ones, with its stage launches j >= 2 timed."""
    import numpy as np
    ps = inputs.patch_set(2000, device="cuda:0")
    descs = [rkl.grid_desc(n, (1 / 64,) * 3, ndim=3, **ps.params) for n in ps.n]
    bdtype = torch.float32 if precision == "mixed" else torch.float64
    bpc = 48.0 if precision == "mixed" else 64.0      # algorithmic bytes per cell-stage, stages j >= 2
    T0 = torch.cat([t.reshape(-1) for t in ps.T]).contiguous()
    b = torch.cat([x.reshape(-1) for x in ps.b]).to(bdtype).contiguous()
    ps.T = ps.b = None
    plan = rkl.Plan(descs, precision=precision, smax=48)
    off = plan.offsets()
    cells = np.array(ps.cells, dtype=np.int64)
    dts = [ps.ratio[p] * plan.dt_par(T0[off[p]:off[p + 1]], grid=p) for p in range(len(descs))]
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda:0")
    s_out = torch.zeros(len(descs), dtype=torch.int32, device="cuda:0")
    T = T0.clone()
    stream = rkl.ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if loop:
        big = int(cells.argmax())
        if args.variant >= 0:
            plan.set_variant(args.variant)
            policy, tuned_ms = args.variant, None
        else:
            policy, tuned_ms = rkl.rkl_autotune(plan.handle, big, *plan._tb(big, T0[off[big]:off[big + 1]],
                                                                            b[3 * off[big]:3 * off[big + 1]]),
                                                dts[big], 2, stream)
        ptrs = [(rkl.ctypes.c_void_p(T[off[p]:].data_ptr()), rkl.ctypes.c_void_p(b[3 * off[p]:].data_ptr()))
                for p in range(len(descs))]

        def step(s_host):
            for p in range(len(descs)):
                s_host[p] = rkl.rkl_superstep(plan.handle, p, ptrs[p][0], ptrs[p][1], dts[p], stream)
    else:
        if args.policy >= 0:
            plan.set_batch_policy(args.policy)
            policy, tuned_ms = args.policy, None
        else:
            policy, tuned_ms = plan.autotune_batched(T0, b, dt, reps=2)   # tile policy by timed search
        plan.graph_capture(T, b, dt, s_out)

        def step(s_host):
            plan.graph_launch()
            s_acc.add_(s_out)
    s_acc = torch.zeros(len(descs), dtype=torch.int64, device="cuda:0")
    s_host = np.zeros(len(descs), dtype=np.int64)
    s_loop = np.zeros(len(descs), dtype=np.int64)
    for _ in range(args.warmup):
        step(s_host)
    T.copy_(T0)
    s_acc.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(s_host)
        s_loop += s_host
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    s_tot = s_loop if loop else s_acc.cpu().numpy()
    cell_stages = float((cells * s_tot).sum())
    if loop:
        # roofline: the first super-step of every patch from the initial
        # fields, run again with its stage launches j >= 2 timed (one event
        # pair per launch; the host submits each launch while the GPU waits,
        # so an interval also holds the submission latency)
        T.copy_(T0)
        torch.cuda.synchronize()
        rkl.rkl_profile(plan.handle, 1)
        step(s_host)
        ms, launches, profiled_cs = rkl.rkl_profile_read(plan.handle, 1)
        rkl.rkl_profile(plan.handle, 0)
        s1 = s_host.copy()
        achieved = bpc * profiled_cs / (ms / 1e3) / 1e9
        kernel = "stage_kernel (stages j>=2 of the per-patch super-steps)"
        traffic = None
    else:
        # roofline: eager launches of the same super-step from the initial fields
        T.copy_(T0)
        torch.cuda.synchronize()
        rkl.rkl_profile(plan.handle, 1)
        plan.superstep_batched(T, b, dt, s_out)
        ms, launches, _ = rkl.rkl_profile_read(plan.handle, 1)
        rkl.rkl_profile(plan.handle, 0)
        s1 = s_out.cpu().numpy().astype(np.int64)
        achieved = bpc * float((cells * (s1 - 1)).sum()) / (ms / 1e3) / 1e9
        kernel = "batch_stage_kernel (stages j>=2, eager launches)"
        traffic = traffic_for(args.workload, precision, "batch", policy)   # average bytes per stage j >= 2 launch
    flags = max(plan.query(g)[2] for g in range(0, len(descs), 97))
    sample = None
    if not args.no_cpu_baseline:
        # host copies of the first patches (about 2.5e7 cell-stages) and the
        # library's result of the same super-step
        npick, work = 0, 0
        while npick < len(descs) and work < 2.5e7:
            work += int(cells[npick] * s1[npick])
            npick += 1
        sample = [(ps.n[p], dts[p], int(s1[p]), T0[off[p]:off[p + 1]].cpu().numpy(),
                   b[3 * off[p]:3 * off[p + 1]].double().cpu().numpy(), T[off[p]:off[p + 1]].cpu().numpy())
                  for p in range(npick)]
    plan.close()
    del T, T0, b
    torch.cuda.empty_cache()
    ceil = copy_ceiling(torch)
    if loop:
        launch = "host loop, one rkl_superstep per patch"
        tile = {"variant": policy, "tile": list(rkl.rkl_variant_info(policy)[:3])}
    else:
        launch = "hipGraph replay, one launch per stage"
        tile = {"tile_policy": policy, "policy_half_rows_tile_z": list(rkl.rkl_batch_policy_info(policy))}
    out = {
        "metric": "cell-stage updates/s",
        "value": cell_stages / sec,
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
        "config": dict({
            "workload": args.workload, "patches": len(descs), "cells": int(cells.sum()),
            "stages_min": int(s1.min()), "stages_max": int(s1.max()), "precision": precision,
            "kappa_par": "T^2.5", "kperp_ratio": ps.params["kperp_ratio"], "limiter": "MC",
            "saturation": "off", "launch": launch, "flags": int(flags),
        }, autotuned_ms_per_step=tuned_ms, **tile),
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
            "kernel": kernel, "bytes_per_cell_stage": bpc,
            "avg_launch_ms": ms / launches, "launches": launches,
            "copy_GBs": ceil, "frac_of_copy": achieved / ceil,
        },
    }
    if sample is not None:
        out["cpu_baseline"], out["accuracy"] = cpu_baseline_patches(sample, ps.params, precision, launch)
    return out


def cpu_baseline_patches(sample, params, precision, launch):
    """The oracle, untuned, on the first patches of the patch workload (one
    super-step each, one host core), and the error of the library's result
    for those patches against it."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    err = ref_sum = chg_sum = linf = 0.0
    cs = 0
    same_s = True
    for n, dt, s_lib, T, bb, got in sample:
        g = oracle.Grid(n=tuple(n), h=(1 / 64,) * 3, ndim=3, **params)
        shape = (n[2], n[1], n[0])
        T = T.reshape(shape)
        ref, s, _ = oracle.superstep(g, T, bb.reshape((3,) + shape), dt)
        got = got.reshape(shape)
        err += float(np.abs(got - ref).sum())
        ref_sum += float(np.abs(ref).sum())
        chg_sum += float(np.abs(ref - T).sum())
        linf = max(linf, float(np.abs(got - ref).max()))
        same_s = same_s and s == s_lib
        cs += int(np.prod(n)) * s
    sec = time.perf_counter() - t0
    base = {"value": cs / sec, "unit": "cell-stage/s", "cores": 1, "kind": "oracle",
            "sample": "one super-step of the first %d patches (%d cell-stages, %.1f s serial)"
                      % (len(sample), cs, sec), "host": host_cpu()}
    acc = {"rel_l1": err / ref_sum, "linf": linf, "rel_l1_change": err / chg_sum, "same_stage_counts": same_s,
           "sample": "the same patches and super-step, library (%s, %s) vs oracle (FP64)" % (precision, launch)}
    return base, acc


def _timed_reps(torch, T, T0, fn, args):
    """args.warmup untimed calls, then args.steps timed ones, each from T0;
    returns (seconds, summed return values of the timed calls)"""
    for _ in range(max(args.warmup, 1)):
        T.copy_(T0)
        fn()
    total, count = 0.0, 0
    for _ in range(args.steps):
        T.copy_(T0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        count += fn()
        torch.cuda.synchronize()
        total += time.perf_counter() - t0
    return total, count


def bench_subcycle(args, torch, inputs, rkl):
    """Explicit sub-cycling (N_sub = ceil(dt_hyp/dt_par) forward-Euler
    sub-steps) of the 256^3 FP64 workload over the dt_hyp that gives its
    RKL2 super-step s = 16, against that super-step (and the RKL1 and AAG
    ones) on the same fields: the measured speed-up of super-time-stepping
    over sub-cycling on this GPU.  One step = one dt_hyp interval; value =
    cell-sub-steps per second.  Also the speed-up against dt_hyp/dt_par for
    s = 8, 16, 32, 64 (three timed repetitions each), which the paper's
    scaling table expects to grow as (dt_hyp/dt_par)^(1/2)."""
    dev = torch.device("cuda:0")
    w = inputs.spitzer_256(device=dev)
    plan = rkl.Plan([rkl.grid_desc(w.n, w.h, ndim=3, **w.params)], precision="fp64")
    T0, w.T = w.T, None
    b, w.b = w.b, None
    T = T0.clone()
    dt = w.ratio * plan.dt_par(T)
    if args.variant >= 0:
        plan.set_variant(args.variant)
    else:
        rkl.rkl_autotune(plan.handle, 0, *plan._tb(0, T, b), dt, 2,
                         rkl.ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))

    def timed(fn):
        return _timed_reps(torch, T, T0, fn, args)

    sec_sts, stages = timed(lambda: plan.superstep(T, b, dt))
    plan1 = rkl.Plan([rkl.grid_desc(w.n, w.h, ndim=3, **w.params)], precision="fp64", scheme="rkl1")
    sec_rkl1, stages1 = timed(lambda: plan1.superstep(T, b, dt))
    plan1.close()
    sec_aag, stages_aag = timed(lambda: plan.aag(T, b, dt, 0.01))
    rkl.rkl_profile(plan.handle, 1)
    sec_sub, nsub = timed(lambda: plan.subcycle(T, b, dt))
    ms, launches, _ = rkl.rkl_profile_read(plan.handle, 3)
    rkl.rkl_profile(plan.handle, 0)
    dtp = plan.dt_par(T0)
    sweep = []
    for s_target in (8, 16, 32, 64):
        dt_k = inputs.midpoint_ratio(s_target) * dtp
        reps = argparse.Namespace(steps=3, warmup=1)
        t_rkl2 = _timed_reps(torch, T, T0, lambda: plan.superstep(T, b, dt_k), reps)
        t_sub = _timed_reps(torch, T, T0, lambda: plan.subcycle(T, b, dt_k), reps)
        sweep.append({"ratio": dt_k / dtp, "stages": t_rkl2[1] // 3, "substeps": t_sub[1] // 3,
                      "rkl2_ms": t_rkl2[0] * 1e3 / 3, "subcycle_ms": t_sub[0] * 1e3 / 3,
                      "speedup": t_sub[0] / t_rkl2[0]})
    plan.close()
    cells = w.cells
    bpc = 40.0                                   # read Y 8 + b 24, write 8
    achieved = bpc * cells / (ms / 1e3 / launches) / 1e9
    del T, T0, b
    torch.cuda.empty_cache()
    ceil = copy_ceiling(torch)
    return {
        "metric": "cell-stage updates/s",
        "value": cells * nsub / sec_sub,
        "unit": "cell-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_sub * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "tangled3d_256_fp64 explicit sub-cycling", "grid": list(w.n),
            "substeps_per_step": nsub // args.steps, "precision": "fp64", "kappa_par": "T^2.5",
            "kperp_ratio": w.params["kperp_ratio"], "limiter": "MC", "saturation": "off",
            "rkl2_stages_same_dt": stages // args.steps,
            "rkl2_ms_per_step": sec_sts * 1e3 / args.steps,
            "sts_speedup": sec_sub / sec_sts,
            "rkl1_stages_same_dt": stages1 // args.steps,
            "rkl1_ms_per_step": sec_rkl1 * 1e3 / args.steps,
            "aag_nu": 0.01, "aag_stages_same_dt": stages_aag // args.steps,
            "aag_ms_per_step": sec_aag * 1e3 / args.steps,
            "speedup_vs_ratio": sweep,
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": None,
            "kernel": "stage_kernel (explicit sub-steps)", "bytes_per_cell_stage": bpc,
            "avg_launch_ms": ms / launches, "launches": launches,
            "copy_GBs": ceil, "frac_of_copy": achieved / ceil,
        },
    }


def host_cpu():
    """CPU model and the number of hardware threads visible to this process"""
    model = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return "%s, %d threads visible" % (model, len(os.sched_getaffinity(0)))


def cpu_baseline(w, T0, b, dt, precision, torch, rkl):
    """The oracle, untuned, on a bounded sample of the same workload: one
    super-step of length dt of a 256 x 256 x 16 periodic slab cut from the
    same fields (host arrays T0 [16][256][256], b [3][16][256][256]), on one
    host core.  The library then runs the same slab (as its own periodic
    grid, in the plan's precision) and its error against the oracle is
    returned with the baseline."""
    import numpy as np
    import oracle
    nz, m = 16, 256
    T = np.ascontiguousarray(T0)
    b = np.ascontiguousarray(b)
    g = oracle.Grid(n=(m, m, nz), h=w.h, ndim=3, **w.params)
    t0 = time.perf_counter()
    ref, s, _ = oracle.superstep(g, T, b, dt)
    sec = time.perf_counter() - t0
    cells = m * m * nz
    base = {"value": cells * s / sec, "unit": "cell-stage/s", "cores": 1, "kind": "oracle",
            "sample": "one %d-stage super-step of a %dx%dx%d periodic slab cut from the same fields "
                      "(%.1f s serial)" % (s, m, m, nz, sec), "host": host_cpu()}
    plan = rkl.Plan([rkl.grid_desc((m, m, nz), w.h, ndim=3, **w.params)], precision=precision)
    Td = torch.from_numpy(T).to("cuda:0")
    bd = torch.from_numpy(b).to("cuda:0", dtype=torch.float32 if precision == "mixed" else torch.float64)
    s_gpu = plan.superstep(Td, bd, dt)
    got = Td.cpu().numpy()
    plan.close()
    acc = {"rel_l1": float(np.abs(got - ref).sum() / np.abs(ref).sum()),
           "linf": float(np.abs(got - ref).max()),
           "rel_l1_change": float(np.abs(got - ref).sum() / np.abs(ref - T).sum()),
           "stages": [int(s_gpu), int(s)],
           "sample": "the same slab and super-step, library (%s) vs oracle (FP64)" % precision}
    return base, acc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="spitzer_256", choices=sorted(WORKLOADS))
    ap.add_argument("--variant", type=int, default=-1, help="kernel variant; -1 = autotune")
    ap.add_argument("--policy", type=int, default=-1,
                    help="batched tile policy (patches_2000, patches_2000_fp64); -1 = autotune")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 1 GiB device-to-device copy (reference for HBM counters)")
    ap.add_argument("--counters-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic JSON of --workload/--variant from two rocprofv3 counter files")
    ap.add_argument("--fuse", type=int, default=1, help="stages per launch of the kernel summarized")
    args = ap.parse_args()
    if args.counters_summary:
        batch = args.workload in ("patches_2000", "patches_2000_fp64")
        fuse = "batch" if batch else args.fuse
        v = args.policy if batch else args.variant
        if v < 0:
            raise SystemExit("--counters-summary needs the --%s the counter runs used" % ("policy" if batch else "variant"))
        print(json.dumps(summarize_counters(*args.counters_summary, args.workload,
                                            WORKLOADS[args.workload][1], fuse, v)))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus %d" % args.gpus,
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
    if builder == "patch_set":
        print(json.dumps(bench_batched(args, torch, inputs, rkl, precision, args.workload.endswith("_loop"))),
              flush=True)
        return
    if args.workload == "spitzer_256_subcycle":
        print(json.dumps(bench_subcycle(args, torch, inputs, rkl)), flush=True)
        return
    dev = torch.device("cuda:0")
    w = getattr(inputs, builder)(device=dev)       # fields generated on the GPU
    plan = rkl.Plan([rkl.grid_desc(w.n, w.h, ndim=3, **w.params)], precision=precision)
    T0, w.T = w.T, None
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
    per_step = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        per_step.append(plan.superstep(T, bdev, dt))
    torch.cuda.synchronize()
    stages = sum(per_step)
    sec = time.perf_counter() - t0
    ms, launches, cell_stages = rkl.rkl_profile_read(plan.handle, fuse)
    rkl.rkl_profile(plan.handle, 0)
    s_last = plan.query()[0]
    # host copies of a 256 x 256 x 16 slab for the CPU baseline
    T0_host = T0[:16, :256, :256].cpu().numpy()
    b_host = bdev[:, :16, :256, :256].double().cpu().numpy()

    avg_launch_s = ms / 1e3 / launches
    bytes_per_launch = bytes_per_cs * cells * fuse
    achieved = bytes_per_launch / avg_launch_s / 1e9
    traffic = traffic_for(args.workload, precision, fuse, variant)
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
            "workload": w.name.replace("_" + w.precision, "_" + precision), "grid": list(w.n), "stages": s_last, "stages_per_step": per_step, "precision": precision,
            "kappa_par": "T^2.5", "kperp_ratio": w.params["kperp_ratio"],
            "limiter": "MC" if w.params["limiter"] else "mean",
            "saturation": ["off", "central", "upwind"][w.params["saturation"]],
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
    plan.close()
    del T, T0, bdev
    torch.cuda.empty_cache()
    ceil = copy_ceiling(torch)
    out["roofline"]["copy_GBs"] = ceil
    out["roofline"]["frac_of_copy"] = achieved / ceil
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["accuracy"] = cpu_baseline(w, T0_host, b_host, dt, precision, torch, rkl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
