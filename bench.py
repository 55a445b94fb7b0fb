#!/usr/bin/env python3
"""Benchmark of the RKL2 anisotropic-conduction super-step on one MI355X.

One step = one full RKL2 super-step (temperature reduction, dt_par and stage
count on the device, then s stencil/stage launches) over the whole grid.
Default workload (the largest single-GPU configuration): a 768^3 periodic
grid in mixed precision (FP32 flux arithmetic, FP64 stage recurrence),
tangled k^-11/3 field, kappa_par = T^2.5, kappa_perp = 1e-3 kappa_par,
MC-limited transverse gradients, central saturated flux (phi = 0.3),
dt_hyp chosen for s = 32, 20 super-steps.  The same JSON line carries the
comparison legs on the same fields and patches (the plain FP64 form of the
768^3 grid; the 2000 uneven patches as the mixed batched graph and as a
plain FP64 loop of one super-step per patch), the error against the oracle
over the workload's whole horizon on the same fields sampled at 64^3, and
the oracle's own rate (serial and on all host cores).  Prints one JSON line.

The stencil kernel variant (tile shape, z-chunk, stages per launch) is picked
by the library's autotuner on the workload's own fields before the timed
region, unless --variant is given; for the batched patch workloads the tile
policy likewise, unless --policy is given.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--variant V] [--policy P]
                  [--no-cpu-baseline] [--no-legs]
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
_FUSED_SOURCES = ["paper_1702_05487_amd/csrc/rkl_tile.h", "paper_1702_05487_amd/csrc/rkl_fused.h",
                  "paper_1702_05487_amd/csrc/rkl_fused.hip"]
KERNEL_SOURCES = {
    1: ["paper_1702_05487_amd/csrc/rkl_tile.h", "paper_1702_05487_amd/csrc/rkl_stage.h",
        "paper_1702_05487_amd/csrc/rkl_kernels.hip"]
       + ["paper_1702_05487_amd/csrc/rkl_stage_%s.hip" % u
          for u in ("f32_32x8", "f32_64x4", "f32_16x16", "f64_32x8", "f64_64x4", "f64_16x16")],
    2: _FUSED_SOURCES, 3: _FUSED_SOURCES, 4: _FUSED_SOURCES,
    "batch": ["paper_1702_05487_amd/csrc/rkl_tile.h", "paper_1702_05487_amd/csrc/rkl_batch.hip"],
}
KERNEL_NAMES = {1: "stage_kernel", 2: "fused_kernel", 3: "fused_kernel", 4: "fused_kernel",
                "batch": "batch_stage_kernel"}


def bytes_per_cell_stage(precision, fuse):
    """Algorithmic HBM bytes per cell and stage of the dominant kernel.
    One stage j >= 2 reads Y_{j-1}, Y_{j-2}, Y0 (FP64), tau M(Y0) and the
    three components of b (FP64, or FP32 in mixed precision) and writes Y_j:
    64 B (FP64) or 48 B (mixed).  A launch of F fused stages (mixed) reads
    the same inputs once and writes the last two stage values: 56 B per cell
    for F stages."""
    if fuse >= 2:
        return 56.0 / fuse
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


def summarize_counters(read_csv, write_csv, workload, precision, fuse, variant):
    """HBM bytes per launch of the dominant kernel from two rocprofv3 --pmc
    runs of this script with --copy-calibration: the read run collects
    TCC_EA0_RDREQ_32B_sum, TCC_EA0_RDREQ_64B_sum and TCC_EA0_RDREQ_128B_sum
    (read requests to HBM by size), the write run TCC_EA0_WRREQ_sum and
    TCC_EA0_WRREQ_64B_sum (write requests, 64 B or else 32 B); bytes are the
    request counts times their sizes.  The calibration run starts with the
    library's streaming copy of 1 GiB (rkl_stream, 8-byte lanes), whose
    counted bytes must come out at 1 GiB each way; the factors that would make
    them so are recorded as a check, not applied.  Stage-1 launches (the
    first stencil launch after each finalize launch) are left out: the
    measured kernel is stages j >= 2.  For the batched workload (fuse
    "batch") the launches are the stage launches j >= 2 of the last, eagerly
    launched super-step, and the figure is their average per launch, like
    the roofline's.  `variant` is the stencil variant (or batched tile
    policy) the counter runs used.  Writes the JSON that traffic_for reads
    and returns it."""
    import csv

    def per_dispatch(path, weights):
        out = {}
        for r in csv.DictReader(open(path)):
            w = weights.get(r["Counter_Name"])
            if w is None:
                continue
            d = int(r["Dispatch_Id"])
            name, v = out.get(d, (r["Kernel_Name"], 0.0))
            out[d] = (name, v + w * float(r["Counter_Value"]))
        return out

    def measured(disp):
        copies = [disp[d][1] for d in sorted(disp) if "copy_kernel" in disp[d][0]]
        if not copies:
            raise SystemExit("no calibration copy (rkl_stream) dispatch in the counter file")
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

    # read requests by size; write requests: 64 B ones, the rest 32 B
    rd, r_copy, nf = measured(per_dispatch(read_csv, {"TCC_EA0_RDREQ_32B_sum": 32.0, "TCC_EA0_RDREQ_64B_sum": 64.0,
                                                      "TCC_EA0_RDREQ_128B_sum": 128.0}))
    wr, w_copy, nw = measured(per_dispatch(write_csv, {"TCC_EA0_WRREQ_sum": 32.0, "TCC_EA0_WRREQ_64B_sum": 32.0}))
    gib = float(1 << 30)
    d = {"kernel": KERNEL_NAMES[fuse], "workload": workload, "precision": precision,
         "kernel_hash": kernel_hash(fuse), "variant": variant,
         "calibration_copy_read_over_1GiB": r_copy / gib, "calibration_copy_write_over_1GiB": w_copy / gib,
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


def stream_ceiling(torch, rkl):
    """Bandwidth of the library's streaming copy kernel (rkl_stream, 8-byte
    lanes, 2 GiB source and destination; read + write bytes per second): the
    highest copy rate measured on this GPU, for reference."""
    src = torch.ones(1 << 28, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    rkl.stream_probe(src, dst, 0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        rkl.stream_probe(src, dst, 0)
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
        npol = rkl.rkl_batch_policy_count()
        if args.policy >= 0:
            # --policy: tile policy + launch mode x the policy count
            plan.set_batch_policy(args.policy % npol)
            plan.set_batch_mode(args.policy // npol)
            policy, tuned_ms = args.policy, None
        else:
            # tile policy and launch mode by timed search
            policy, tuned_ms = plan.autotune_batched(T0, b, dt, reps=2)
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
        persistent = policy // rkl.rkl_batch_policy_count() == 1
        ms, launches, _ = rkl.rkl_profile_read(plan.handle, 6 if persistent else 1)
        rkl.rkl_profile(plan.handle, 0)
        s1 = s_out.cpu().numpy().astype(np.int64)
        if persistent:
            # one launch holds every stage: stage 1 reads T and b and writes
            # Y1 and tau M(Y0) (mixed 32 B, FP64 40 B per cell), stages j >= 2 as above
            b1 = 32.0 if precision == "mixed" else 40.0
            achieved = float((cells * (b1 + bpc * (s1 - 1))).sum()) / (ms / 1e3) / 1e9
            kernel = "batch_persistent_kernel (all stages, eager launch)"
        else:
            achieved = bpc * float((cells * (s1 - 1)).sum()) / (ms / 1e3) / 1e9
            kernel = "batch_stage_kernel (stages j>=2, eager launches)"
        traffic = None if persistent else traffic_for(args.workload, precision, "batch", policy)
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
        npol = rkl.rkl_batch_policy_count()
        launch = ("hipGraph replay: reduce, schedule and one persistent launch" if policy // npol == 1
                  else "hipGraph replay, one launch per stage")
        tile = {"tile_policy": policy % npol, "launch_mode": policy // npol,
                "policy_half_rows_tile_z": list(rkl.rkl_batch_policy_info(policy % npol))}
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
    ms, launches, _ = rkl.rkl_profile_read(plan.handle, 5)
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


HORIZON_N = (64, 64, 64)


def horizon_check(w, precision, torch, rkl, threads):
    """The oracle's rate and the library's error over the workload's whole
    horizon, on the workload's own continuous fields sampled at 64^3 (same
    parameters, dt_hyp ratio and number of super-steps).

    cpu_baseline: the oracle (untuned) timed serially on one host core for
    the first super-step, and on `threads` cores (its OpenMP loop over the
    cells; the same result bits, checked) for the whole horizon.
    accuracy: the library in the workload's precision against that oracle
    run at every super-step; mixed precision also against the oracle fed the
    FP64 unit vectors (the FP64 problem), which adds the rounding of b to
    FP32.  The library's FP64 form runs beside it as a check."""
    import numpy as np
    import oracle
    from paper_1702_05487_amd import inputs
    n = HORIZON_N
    T0 = inputs.noisy_temperature(n, 2)
    b = inputs.tangled_b(n, 1)
    h = tuple(1.0 / v for v in n)
    g = oracle.Grid(n=n, h=h, ndim=3, **w.params)
    bq = b.astype(np.float32).astype(np.float64) if precision == "mixed" else b

    def lib(prec):
        plan = rkl.Plan([rkl.grid_desc(n, h, ndim=3, **w.params)], precision=prec)
        T = torch.from_numpy(T0.copy()).to("cuda:0")
        bd = torch.from_numpy(b).to("cuda:0", dtype=torch.float32 if prec == "mixed" else torch.float64)
        dt = w.ratio * plan.dt_par(T)
        outs, ss = [], []
        for _ in range(w.steps):
            ss.append(plan.superstep(T, bd, dt))
            outs.append(T.cpu().numpy())
        plan.close()
        return outs, ss, dt

    got, s_lib, dt = lib(precision)
    got64, s_lib64, dt64 = lib("fp64") if precision == "mixed" else (got, s_lib, dt)
    assert dt64 == dt == w.ratio * oracle.dt_par(g, T0)

    def orc(bb, nthreads):
        oracle.set_threads(nthreads)
        t0 = time.perf_counter()
        T, outs, ss = T0, [], []
        for _ in range(w.steps):
            T, s, _ = oracle.superstep(g, T, bb, dt)
            outs.append(T)
            ss.append(s)
        return outs, ss, time.perf_counter() - t0

    oracle.set_threads(1)
    t0 = time.perf_counter()
    first, s1, _ = oracle.superstep(g, T0, bq, dt)
    sec1 = time.perf_counter() - t0
    ref, s_ref, sec_all = orc(bq, threads)
    used = oracle.threads()
    ref64, s_ref64, _ = orc(b, threads) if precision == "mixed" else (ref, s_ref, 0.0)
    oracle.set_threads(1)
    assert np.array_equal(first, ref[0]), "threaded oracle differs from serial"
    cells = int(np.prod(n))

    def rel(a, r):
        return float(np.abs(a - r).sum() / np.abs(r).sum())

    base = {"value": cells * sum(s_ref) / sec_all, "unit": "cell-stage/s", "cores": used, "kind": "oracle",
            "sample": "%d super-steps (%d stages) of the workload's fields sampled at %dx%dx%d, all cells "
                      "(%.1f s on %d threads)" % (w.steps, sum(s_ref), n[0], n[1], n[2], sec_all, used),
            "serial": {"value": cells * s1 / sec1, "cores": 1,
                       "sample": "the first of those super-steps on one core (%.1f s)" % sec1},
            "host": host_cpu()}
    e64 = [rel(a, r) for a, r in zip(got64, ref64)]
    within = 0
    while within < len(e64) and e64[within] <= 1e-12:
        within += 1
    acc = {"kind": "whole horizon against the oracle, every cell (%dx%dx%d, %d super-steps)"
                   % (n[0], n[1], n[2], w.steps),
           "stages": {"library": s_lib, "oracle": s_ref},
           "first_step": {"rel_l1": rel(got[0], ref[0]), "linf": float(np.abs(got[0] - ref[0]).max()),
                          "rel_l1_change": float(np.abs(got[0] - ref[0]).sum() / np.abs(ref[0] - T0).sum())},
           "rel_l1_per_step": [rel(a, r) for a, r in zip(got, ref)],
           "rel_l1": rel(got[-1], ref[-1]),
           "linf": float(np.abs(got[-1] - ref[-1]).max()),
           # how far the FP64 library (operations in another order, same
           # arithmetic) drifts from the oracle over the same horizon: the
           # problem's own amplification of rounding differences
           "fp64_library": {"stages": s_lib64, "rel_l1_per_step": e64,
                            "steps_within_1e-12": within}}
    if precision == "mixed":
        acc["reference"] = "oracle fed the same FP32-rounded unit vectors (arithmetic only)"
        acc["against_fp64_problem"] = {
            "reference": "oracle fed the FP64 unit vectors", "stages_oracle": s_ref64,
            "rel_l1_per_step": [rel(a, r) for a, r in zip(got, ref64)],
            "rel_l1": rel(got[-1], ref64[-1]), "linf": float(np.abs(got[-1] - ref64[-1]).max())}
    return base, acc


def horizon_errors_from_tests():
    """Per-configuration horizon errors measured by the GPU tests (committed
    summary), if any."""
    path = os.path.join(ROOT, "profiles", "horizon_errors.json")
    try:
        return json.load(open(path))
    except (OSError, ValueError):
        return None


def run_grid(torch, rkl, w, T0, b, precision, steps, warmup, variant=-1, one_stage_only=False, chain=False):
    """One timed single-grid run: plan, variant (autotuned unless given),
    `warmup` untimed and `steps` timed super-steps from T0, the dominant
    kernel's launches timed with HIP events.  Returns a dict.  chain: also
    time the same super-steps as one rkl_supersteps_async call (each
    super-step after the first takes its extrema from the previous one's
    last stage) and check that it gives the same bits."""
    plan = rkl.Plan([rkl.grid_desc(w.n, w.h, ndim=3, **w.params)], precision=precision)
    T = T0.clone()
    dt = w.ratio * plan.dt_par(T)     # the library's own dt_par of the initial field
    stream = rkl.ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    tuned_ms = None
    if variant < 0:
        variant, tuned_ms = rkl.rkl_autotune(plan.handle, 0, *plan._tb(0, T, b), dt, 2, stream)
        if one_stage_only and rkl.rkl_variant_info(variant)[3] != 1:
            raise RuntimeError("autotuner picked a fused variant for a one-stage-only run")
    else:
        plan.set_variant(variant)
    tile = rkl.rkl_variant_info(variant)
    fuse = tile[3]
    for _ in range(warmup):
        plan.superstep(T, b, dt)
    T.copy_(T0)
    torch.cuda.synchronize()
    rkl.rkl_profile(plan.handle, 1)
    per_step = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        per_step.append(plan.superstep(T, b, dt))
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    ms, launches, cell_stages = rkl.rkl_profile_read(plan.handle, fuse)
    rkl.rkl_profile(plan.handle, 0)
    chained = None
    if chain and fuse == 1:
        s_cap = max(per_step) + 1
        s_out = torch.zeros(steps, dtype=torch.int32, device=T.device)
        T2 = T0.clone()
        plan.supersteps_async(T2, b, dt, steps, s_cap, s_out=s_out)   # untimed
        T2.copy_(T0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.supersteps_async(T2, b, dt, steps, s_cap, s_out=s_out)
        torch.cuda.synchronize()
        sec2 = time.perf_counter() - t0
        ss = [int(v) for v in s_out.cpu().tolist()]
        chained = {"value": w.cells * sum(ss) / sec2, "ms_per_step": sec2 * 1e3 / steps, "s_cap": s_cap,
                   "stages_per_step": ss, "same_bits_as_rkl_superstep": bool(torch.equal(T, T2)),
                   "entry": "rkl_supersteps_async (one call, the extrema of each super-step's start from "
                            "the previous super-step's last stage)"}
        del T2
    plan.close()
    del T
    bpc = bytes_per_cell_stage(precision, fuse)
    avg = ms / 1e3 / launches
    achieved = bpc * w.cells * fuse / avg / 1e9
    return {"value": w.cells * sum(per_step) / sec, "ms_per_step": sec * 1e3 / steps, "stages_per_step": per_step,
            "dt_hyp": dt, "variant": variant, "tile": list(tile[:3]), "stages_per_launch": fuse,
            "autotuned_ms_per_step": tuned_ms, "kernel": "%s (stages j>=2)" % KERNEL_NAMES[fuse],
            "bytes_per_cell_stage": bpc, "avg_launch_ms": avg * 1e3, "launches": launches,
            "achieved": achieved, "kernel_cell_stage_per_s": cell_stages / (ms / 1e3), "chained": chained}


def batched_leg(torch, inputs, rkl, workload, steps, warmup):
    """One of the 2000-patch forms, timed, without its CPU baseline."""
    a = argparse.Namespace(workload=workload, steps=steps, warmup=warmup, variant=-1, policy=-1,
                           no_cpu_baseline=True)
    _, precision = WORKLOADS[workload]
    d = bench_batched(a, torch, inputs, rkl, precision, workload.endswith("_loop"))
    r = d["roofline"]
    return {"value": d["value"], "ms_per_step": d["ms_per_step"], "steps": steps,
            "stages_min": d["config"]["stages_min"], "stages_max": d["config"]["stages_max"],
            "launch": d["config"]["launch"], "kernel": r["kernel"], "achieved_GBs": r["achieved"],
            "frac": r["frac"], "traffic": r["traffic"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="fused_768", choices=sorted(WORKLOADS))
    ap.add_argument("--variant", type=int, default=-1, help="kernel variant; -1 = autotune")
    ap.add_argument("--policy", type=int, default=-1,
                    help="batched tile policy (patches_2000, patches_2000_fp64); -1 = autotune")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="leave out the comparison legs of the default workload (FP64 form, patches)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run the library's 1 GiB streaming copy (reference for HBM counters)")
    ap.add_argument("--counters-summary", nargs=2, metavar=("READ_CSV", "WRITE_CSV"),
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

    import torch

    from paper_1702_05487_amd import inputs, rkl

    builder, precision = WORKLOADS[args.workload]
    rkl.load(build_if_missing=True)
    if args.copy_calibration:
        # the reference dispatch of the HBM counters: the library's streaming
        # copy of 1 GiB with 8-byte lanes (rkl_stream)
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        rkl.stream_probe(src, dst, 0)
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
    T0, w.T = w.T, None
    b64, w.b = w.b, None
    bdev = b64.to(dtype=torch.float32 if precision == "mixed" else torch.float64)
    if precision == "mixed" and (args.no_legs or args.workload != "fused_768"):
        del b64
        b64 = None
    r = run_grid(torch, rkl, w, T0, bdev, precision, args.steps, args.warmup, args.variant,
                 chain=args.workload == "fused_768" and not args.no_legs)
    del bdev
    torch.cuda.empty_cache()
    traffic = traffic_for(args.workload, precision, r["stages_per_launch"], r["variant"])
    out = {
        "metric": "cell-stage updates/s",
        "value": r["value"],
        "unit": "cell-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32 flux + f64 recurrence",
        "data": "synthetic",
        "config": {
            "workload": w.name.replace("_" + w.precision, "_" + precision), "grid": list(w.n),
            "stages": r["stages_per_step"][-1], "stages_per_step": r["stages_per_step"], "precision": precision,
            "kappa_par": "T^2.5", "kperp_ratio": w.params["kperp_ratio"],
            "limiter": "MC" if w.params["limiter"] else "mean",
            "saturation": ["off", "central", "upwind"][w.params["saturation"]],
            "variant": r["variant"], "tile": r["tile"], "stages_per_launch": r["stages_per_launch"],
            "autotuned_ms_per_step": r["autotuned_ms_per_step"],
        },
        "roofline": {
            "bound": "hbm", "achieved": r["achieved"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": r["achieved"] / PEAK_HBM_GBS, "traffic": traffic,
            "kernel": r["kernel"], "bytes_per_cell_stage": r["bytes_per_cell_stage"],
            "avg_launch_ms": r["avg_launch_ms"], "launches": r["launches"],
            "kernel_cell_stage_per_s": r["kernel_cell_stage_per_s"],
        },
    }
    if args.workload == "fused_768" and not args.no_legs:
        # the plain FP64 form on the same fields (one-stage kernels), then the patches
        legs = {}
        bf = b64.to(torch.float64)
        del b64
        f = run_grid(torch, rkl, w, T0, bf, "fp64", min(args.steps, 5), 1, one_stage_only=True)
        del bf
        torch.cuda.empty_cache()
        legs["fp64_plain_768"] = {k: f[k] for k in ("value", "ms_per_step", "stages_per_step", "variant", "tile",
                                                     "kernel", "achieved", "avg_launch_ms")}
        legs["fp64_plain_768"]["frac"] = f["achieved"] / PEAK_HBM_GBS
        legs["fp64_plain_768"]["dt_hyp_same"] = f["dt_hyp"] == r["dt_hyp"]
        legs["mixed_over_fp64_768"] = r["value"] / f["value"]
        if r["chained"]:
            legs["supersteps_async_768"] = r["chained"]
        del T0
        torch.cuda.empty_cache()
        legs["patches_2000_mixed_batched"] = batched_leg(torch, inputs, rkl, "patches_2000", 10, 2)
        legs["patches_2000_fp64_loop"] = batched_leg(torch, inputs, rkl, "patches_2000_fp64_loop", 2, 1)
        legs["patches_mixed_batched_over_fp64_loop"] = (legs["patches_2000_mixed_batched"]["value"]
                                                        / legs["patches_2000_fp64_loop"]["value"])
        legs["patches_mixed_batched_over_fp64_plain_768"] = (legs["patches_2000_mixed_batched"]["value"]
                                                             / legs["fp64_plain_768"]["value"])
        out["legs"] = legs
    else:
        del T0
    torch.cuda.empty_cache()
    ceil = copy_ceiling(torch)
    out["roofline"]["copy_GBs"] = ceil
    out["roofline"]["frac_of_copy"] = r["achieved"] / ceil
    sc = stream_ceiling(torch, rkl)
    out["roofline"]["stream_copy_GBs"] = sc
    out["roofline"]["frac_of_stream_copy"] = r["achieved"] / sc
    if traffic:
        # counted HBM bytes of the dominant kernel per second of its launches
        out["roofline"]["traffic_GBs"] = traffic / (r["avg_launch_ms"] / 1e3) / 1e9
        out["roofline"]["traffic_frac_of_stream_copy"] = out["roofline"]["traffic_GBs"] / sc
    if not args.no_cpu_baseline:
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        out["cpu_baseline"], out["accuracy"] = horizon_check(w, precision, torch, rkl, threads)
        out["accuracy"]["per_config_from_tests"] = horizon_errors_from_tests()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
