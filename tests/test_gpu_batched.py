"""Batched super-step (many uneven patches, per-patch s, one graph-capturable
launch sequence) vs the FP64 oracle run patch by patch."""
import numpy as np
import pytest

import oracle
from helpers import lib_desc, oracle_grid, rel_l1
from paper_1702_05487_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1702_05487_amd import rkl
    rkl.load(build_if_missing=False)
    return torch


def small_patch_set(npatch, seed, lo=8, hi=40, smin=2, smax=12):
    return inputs.patch_set(npatch, seed=seed, lo=lo, hi=hi, smin=smin, smax=smax)


def pack(torch, ps, precision):
    bdt = np.float32 if precision == "mixed" else np.float64
    T = np.concatenate([t.ravel() for t in ps.T])
    b = np.concatenate([bb.astype(bdt).ravel() for bb in ps.b])
    tdt = torch.float32 if precision == "mixed" else torch.float64
    return (torch.from_numpy(T).to("cuda:0"), torch.from_numpy(b).to("cuda:0", dtype=tdt))


def oracle_patches(ps, precision):
    outs, svals, dts = [], [], []
    for p, n in enumerate(ps.n):
        h = tuple(1.0 / 64 for _ in range(3))
        g = oracle_grid(n, h, 3, ps.params)
        b = ps.b[p].astype(np.float32).astype(np.float64) if precision == "mixed" else ps.b[p]
        dt = ps.ratio[p] * oracle.dt_par(g, ps.T[p])
        To, s, _ = oracle.superstep(g, ps.T[p], b, dt)
        outs.append(To)
        svals.append(s)
        dts.append(dt)
    return outs, svals, dts


def make_plan(ps, precision, smax=16):
    from paper_1702_05487_amd import rkl
    descs = [lib_desc(n, (1 / 64,) * 3, 3, ps.params) for n in ps.n]
    return rkl.Plan(descs, precision=precision, smax=smax)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_batched_matches_oracle(torch_cuda, precision, tol):
    torch = torch_cuda
    ps = small_patch_set(20, seed=3)
    print("batched", precision, [n for n in ps.n][:5], flush=True)
    ref, sref, dts = oracle_patches(ps, precision)
    plan = make_plan(ps, precision)
    T, b = pack(torch, ps, precision)
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda:0")
    s_out = torch.zeros(len(ps.n), dtype=torch.int32, device="cuda:0")
    plan.superstep_batched(T, b, dt, s_out)
    got = T.cpu().numpy()
    off = plan.offsets()
    assert list(s_out.cpu().numpy()) == sref
    for p in range(len(ps.n)):
        gp = got[off[p]:off[p + 1]].reshape(ref[p].shape)
        assert rel_l1(gp, ref[p]) <= tol, p
        assert plan.query(p)[0] == sref[p]


def test_batched_equals_single_grid_calls(torch_cuda):
    # the batched launch and per-grid rkl_superstep give bit-identical results
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    ps = small_patch_set(12, seed=4)
    _, _, dts = oracle_patches(ps, "fp64")
    plan = make_plan(ps, "fp64")
    T, b = pack(torch, ps, "fp64")
    T1 = T.clone()
    plan.superstep_batched(T, b, torch.tensor(dts, dtype=torch.float64, device="cuda:0"))
    off = plan.offsets()
    for p, n in enumerate(ps.n):
        single = rkl.Plan([lib_desc(n, (1 / 64,) * 3, 3, ps.params)], precision="fp64")
        Tp = T1[off[p]:off[p + 1]].clone()
        single.superstep(Tp, b[3 * off[p]:3 * off[p + 1]].clone(), dts[p])
        assert torch.equal(Tp, T[off[p]:off[p + 1]]), p


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_persistent_equals_per_stage_launches(torch_cuda, precision, tol):
    """The persistent launch (rkl_set_batch_mode 1: reduce, schedule and one
    persistent launch whose workgroups take (stage, grid, tile) items from a
    ticket counter) gives the same bits as one launch per stage, and matches
    the oracle; eager and graph-captured, three super-steps; no wait gave up."""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    ps = small_patch_set(24, seed=13, lo=8, hi=40, smin=2, smax=14)
    print("persistent", precision, ps.n[:4], flush=True)
    ref, sref, dts = oracle_patches(ps, precision)
    per = make_plan(ps, precision)
    pers = make_plan(ps, precision)
    pers.set_batch_mode(1)
    Ta, b = pack(torch, ps, precision)
    Tb, Tc = Ta.clone(), Ta.clone()
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda:0")
    sa = torch.zeros(len(ps.n), dtype=torch.int32, device="cuda:0")
    sb = torch.zeros_like(sa)
    per.superstep_batched(Ta, b, dt, sa)
    pers.superstep_batched(Tb, b, dt, sb)
    torch.cuda.synchronize()
    assert all(pers.query(p)[2] & rkl.RKL_FLAG_ABORTED == 0 for p in range(len(ps.n)))
    assert torch.equal(sa, sb) and list(sb.cpu().numpy()) == sref
    assert torch.equal(Ta, Tb)
    got = Tb.cpu().numpy()
    off = per.offsets()
    for p in range(len(ps.n)):
        assert rel_l1(got[off[p]:off[p + 1]].reshape(ref[p].shape), ref[p]) <= tol, p
    # two more super-steps, eager per-stage launches against the persistent graph
    pers.graph_capture(Tc, b, dt, sb)
    pers.graph_launch()                      # Tc: first super-step
    assert torch.equal(Tc, Ta)
    for _ in range(2):
        per.superstep_batched(Ta, b, dt, sa)
        pers.graph_launch()
        torch.cuda.synchronize()
        assert torch.equal(Tc, Ta) and torch.equal(sa, sb)
    assert all(pers.query(p)[2] & rkl.RKL_FLAG_ABORTED == 0 for p in range(len(ps.n)))
    per.close()
    pers.close()


def test_persistent_patch_workload(torch_cuda):
    """The 2000 patches: two super-steps of the persistent launch equal the
    per-stage launches bit for bit (mixed precision); timings printed."""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    ps = inputs.patch_set(2000, device="cuda:0")
    T0 = torch.cat([t.reshape(-1) for t in ps.T]).contiguous()
    b = torch.cat([x.reshape(-1) for x in ps.b]).float().contiguous()
    ps.T = ps.b = None
    descs = [lib_desc(n, (1 / 64,) * 3, 3, ps.params) for n in ps.n]
    out = {}
    for mode in (0, 1):
        plan = rkl.Plan(descs, precision="mixed", smax=48)
        plan.set_batch_mode(mode)
        off = plan.offsets()
        dt = torch.tensor([ps.ratio[k] * plan.dt_par(T0[off[k]:off[k + 1]], grid=k) for k in range(len(descs))],
                          dtype=torch.float64, device="cuda:0")
        T = T0.clone()
        s_out = torch.zeros(len(descs), dtype=torch.int32, device="cuda:0")
        plan.graph_capture(T, b, dt, s_out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(2):
            plan.graph_launch()
        e1.record()
        torch.cuda.synchronize()
        flags = max(plan.query(k)[2] for k in range(0, len(descs), 50))
        print("mode %d: %.2f ms per super-step, flags %d" % (mode, e0.elapsed_time(e1) / 2, flags), flush=True)
        assert flags & rkl.RKL_FLAG_ABORTED == 0
        out[mode] = (T.clone(), s_out.clone())
        plan.close()
    assert torch.equal(out[0][1], out[1][1])
    assert torch.equal(out[0][0], out[1][0])


def test_many_supersteps_match_oracle(torch_cuda):
    # three consecutive batched super-steps (s re-computed on the device each time)
    torch = torch_cuda
    ps = small_patch_set(12, seed=9, lo=8, hi=32, smax=10)
    plan = make_plan(ps, "fp64")
    T, b = pack(torch, ps, "fp64")
    off = plan.offsets()
    Tref = [t.copy() for t in ps.T]
    for _ in range(3):
        dts = []
        for p, n in enumerate(ps.n):
            g = oracle_grid(n, (1 / 64,) * 3, 3, ps.params)
            dt = ps.ratio[p] * oracle.dt_par(g, Tref[p])
            Tref[p], _, _ = oracle.superstep(g, Tref[p], ps.b[p], dt)
            dts.append(dt)
        plan.superstep_batched(T, b, torch.tensor(dts, dtype=torch.float64, device="cuda:0"))
    got = T.cpu().numpy()
    for p in range(len(ps.n)):
        assert rel_l1(got[off[p]:off[p + 1]].reshape(Tref[p].shape), Tref[p]) <= 1e-12


def test_graph_replays_match_eager(torch_cuda):
    """Capture one batched super-step in a HIP graph, replay it several
    times with eager work and synchronisations between, and check every
    replay against the eager launch sequence on a copy."""
    torch = torch_cuda
    ps = small_patch_set(16, seed=5)
    _, _, dts = oracle_patches(ps, "mixed")
    plan = make_plan(ps, "mixed")
    eager_plan = make_plan(ps, "mixed")
    T, b = pack(torch, ps, "mixed")
    Te = T.clone()
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda:0")
    s_g = torch.zeros(len(ps.n), dtype=torch.int32, device="cuda:0")
    s_e = torch.zeros_like(s_g)
    plan.graph_capture(T, b, dt, s_g)
    for r in range(4):
        plan.graph_launch()
        torch.cuda.synchronize()
        eager_plan.superstep_batched(Te, b, dt, s_e)
        torch.cuda.synchronize()
        _ = (Te * 2).sum().item()      # unrelated eager work between replays
        assert torch.equal(T, Te), r
        assert torch.equal(s_g, s_e), r


def test_batched_stage_limit_is_flagged(torch_cuda):
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    ps = small_patch_set(6, seed=6, smax=6)
    _, sref, dts = oracle_patches(ps, "fp64")
    assert max(sref) <= 8
    plan = make_plan(ps, "fp64", smax=8)
    T, b = pack(torch, ps, "fp64")
    T0 = T.clone()
    dts[2] = dts[2] * 100.0      # this patch would need more than 8 stages
    plan.superstep_batched(T, b, torch.tensor(dts, dtype=torch.float64, device="cuda:0"))
    off = plan.offsets()
    assert plan.query(2)[2] & rkl.RKL_FLAG_STAGES
    assert torch.equal(T[off[2]:off[3]], T0[off[2]:off[3]])
    assert not torch.equal(T[off[1]:off[2]], T0[off[1]:off[2]])


@pytest.mark.parametrize("precision,tol", [("mixed", 1e-5), ("fp64", 1e-12)])
def test_patches_2000_full_size_sampled(torch_cuda, precision, tol):
    """The 2000-patch workload at full size in the launch configuration that
    bench.py times (smax 48, captured graph replayed) with every tile policy
    (the autotuner picks among them; all give the same bits over the whole
    packed field): whole patches sampled and compared with the oracle -- the
    six smallest, two drawn at random and the small patch with the most
    stages."""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    ps = inputs.patch_set(2000, device="cuda:0")
    descs = [lib_desc(n, (1 / 64,) * 3, 3, ps.params) for n in ps.n]
    T0 = torch.cat([t.reshape(-1) for t in ps.T]).contiguous()
    b = torch.cat([x.reshape(-1) for x in ps.b]).to(torch.float32 if precision == "mixed" else torch.float64)
    b = b.contiguous()
    ps.T = ps.b = None
    plan = rkl.Plan(descs, precision=precision, smax=48)
    off = plan.offsets()
    dts = [ps.ratio[p] * plan.dt_par(T0[off[p]:off[p + 1]], grid=p) for p in range(len(descs))]
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda:0")
    s_out = torch.zeros(len(descs), dtype=torch.int32, device="cuda:0")
    T = None
    for pol in range(rkl.rkl_batch_policy_count()):
        plan.set_batch_policy(pol)
        Tp = T0.clone()
        plan.graph_capture(Tp, b, dt, s_out)
        plan.graph_launch()
        torch.cuda.synchronize()
        if T is None:
            T, s = Tp, s_out.cpu().numpy()
        else:
            assert torch.equal(Tp, T), pol
            assert np.array_equal(s_out.cpu().numpy(), s), pol
            del Tp
    assert s.min() >= 4 and s.max() <= 40
    cells = np.array(ps.cells)
    order = np.argsort(cells)
    rng = np.random.default_rng(17)
    small = order[cells[order] < 20000]
    picks = list(order[:6]) + list(rng.choice(small, 2, replace=False)) + [small[np.argmax(s[small])]]
    print("patches", [(int(p), ps.n[p], int(s[p])) for p in picks], flush=True)
    got = T.cpu().numpy()
    for p in picks:
        n = ps.n[p]
        shape = (n[2], n[1], n[0])
        Tp = T0[off[p]:off[p + 1]].cpu().numpy().reshape(shape)
        bp = b[3 * off[p]:3 * off[p + 1]].double().cpu().numpy().reshape((3,) + shape)
        g = oracle_grid(n, (1 / 64,) * 3, 3, ps.params)
        To, s_ref, _ = oracle.superstep(g, Tp, bp, dts[p])
        assert s_ref == s[p], p
        err = rel_l1(got[off[p]:off[p + 1]].reshape(shape), To)
        assert err <= tol, (p, err)
    plan.close()


def test_every_batch_policy_gives_the_same_bits(torch_cuda):
    """Tiling changes which workgroup computes a face, never the operations,
    so every batched tile policy gives the same bits."""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    ps = small_patch_set(16, seed=9, lo=8, hi=60)
    _, _, dts = oracle_patches(ps, "mixed")
    plan = make_plan(ps, "mixed")
    T, b = pack(torch, ps, "mixed")
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda:0")
    ref = None
    for pol in range(rkl.rkl_batch_policy_count()):
        plan.set_batch_policy(pol)
        Tp = T.clone()
        plan.superstep_batched(Tp, b, dt)
        if ref is None:
            ref = Tp
        else:
            assert torch.equal(Tp, ref), pol
    plan.close()


def test_policy_change_drops_the_graph(torch_cuda):
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    ps = small_patch_set(6, seed=10)
    _, _, dts = oracle_patches(ps, "fp64")
    plan = make_plan(ps, "fp64")
    T, b = pack(torch, ps, "fp64")
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda:0")
    plan.graph_capture(T, b, dt)
    plan.graph_launch()
    plan.set_batch_policy(1)
    with pytest.raises(rkl.RklError) as e:
        plan.graph_launch()
    assert e.value.status == rkl.RKL_ESTATE
    plan.graph_capture(T, b, dt)
    plan.graph_launch()
    torch.cuda.synchronize()
    plan.close()


def test_batched_autotune(torch_cuda):
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    ps = small_patch_set(12, seed=11, lo=8, hi=48)
    ref, sref, dts = oracle_patches(ps, "mixed")
    plan = make_plan(ps, "mixed")
    T, b = pack(torch, ps, "mixed")
    dt = torch.tensor(dts, dtype=torch.float64, device="cuda:0")
    T_before = T.clone()
    pol, ms = plan.autotune_batched(T, b, dt, reps=1)
    assert torch.equal(T, T_before)              # the caller's T is not touched
    # index = tile policy + launch mode x policy count (both modes are timed)
    assert 0 <= pol < 2 * rkl.rkl_batch_policy_count() and ms > 0
    plan.superstep_batched(T, b, dt)
    got = T.cpu().numpy()
    off = plan.offsets()
    for p in range(len(ps.n)):
        assert rel_l1(got[off[p]:off[p + 1]].reshape(ref[p].shape), ref[p]) <= 1e-5, p
    with pytest.raises(rkl.RklError):
        plan.autotune_batched(T, b, dt, reps=0)
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_one_grid_graph_equals_superstep(torch_cuda, precision):
    """A plan of one grid: rkl_superstep (host read-back of s), the batched
    entry point and a captured graph of it replayed give the same bits, for
    three consecutive super-steps."""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n = (48, 40, 36)
    h = tuple(1.0 / v for v in n)
    p = dict(inputs.SPITZER_MC_SAT, phi=0.003)
    T0 = inputs.noisy_temperature(n, 2, kmax=8)
    b = inputs.tangled_b(n, 1, kmax=8)
    bdt = torch.float32 if precision == "mixed" else torch.float64
    bd = torch.from_numpy(b).to("cuda:0", dtype=bdt)
    one = rkl.Plan([lib_desc(n, h, 3, p)], precision=precision)
    bat = rkl.Plan([lib_desc(n, h, 3, p)], precision=precision, smax=24)
    Ta = torch.from_numpy(T0).to("cuda:0")
    Tb = Ta.clone()
    Tg = Ta.clone()
    dt = inputs.midpoint_ratio(14) * one.dt_par(Ta)
    dtd = torch.tensor([dt], dtype=torch.float64, device="cuda:0")
    s_out = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    graph = rkl.Plan([lib_desc(n, h, 3, p)], precision=precision, smax=24)
    graph.graph_capture(Tg, bd, dtd, s_out)
    for _ in range(3):
        s = one.superstep(Ta, bd, dt)
        bat.superstep_batched(Tb, bd, dtd, s_out)
        assert int(s_out.item()) == s
        graph.graph_launch()
        torch.cuda.synchronize()
        assert int(s_out.item()) == s
        assert torch.equal(Ta, Tb)
        assert torch.equal(Ta, Tg)
    for pl in (one, bat, graph):
        pl.close()
