"""rkl_supersteps_async: several RKL2 super-steps in one enqueue.  Each
super-step after the first takes the extrema of its starting temperature
(for dt_par and the FP32 reference temperature, Sec. 3.1 Eq. dt_exp) from
its predecessor's last stage instead of a reduction pass over T, on 3-D
grids without fixed axes; other grids take the pass each time.  The
extrema are the same numbers either way, so the result must have the same
bits as the same number of rkl_superstep_async calls; FP64 runs are also
held to the oracle (rel-L1 <= 1e-12)."""
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


def fields(n, seed):
    rng = np.random.default_rng(seed)
    shape = (n[2], n[1], n[0])
    T = 1.0 + 0.2 * rng.random(shape)
    b = inputs.unit_vectors(rng.standard_normal((3,) + shape))
    return T, b


CASES = [
    # n, ndim, boundary, precision, variant
    ((40, 33, 23), 3, (0, 0, 0), "mixed", 0),
    ((40, 33, 23), 3, (0, 0, 0), "mixed", 3),
    ((40, 33, 23), 3, (0, 0, 0), "fp64", 1),
    ((24, 20, 36), 3, (1, 0, 1), "mixed", 2),
    ((24, 20, 36), 3, (0, 1, 0), "fp64", 4),
    ((48, 40, 1), 2, (0, 1, 0), "mixed", 0),    # 2-D: the reduction before every super-step
    ((17, 9, 70), 3, (0, 0, 0), "mixed", 8),    # a two-stage variant selected: routed stages use variant 0
]


def run_pair(torch, rkl, n, ndim, bnd, precision, variant, nsteps, ratio, s_cap=None, seed=3):
    T0, b = fields(n, seed)
    p = dict(inputs.SPITZER_MC_SAT, boundary=bnd, kperp_ratio=0.01)
    h = tuple(1.0 / v for v in n)
    plan = rkl.Plan([lib_desc(n, h, ndim, p)], precision=precision, variant=variant)
    bt = torch.float32 if precision == "mixed" else torch.float64
    bg = torch.from_numpy(b.astype(np.float32) if precision == "mixed" else b).to("cuda:0").to(bt)
    Tg = torch.from_numpy(T0).to("cuda:0")
    dt = ratio * plan.dt_par(Tg)
    cap = s_cap or 64
    Ta = Tg.clone()
    sa = torch.zeros(nsteps, dtype=torch.int32, device="cuda:0")
    for i in range(nsteps):
        plan.superstep_async(Ta, bg, dt, cap, s_out=sa[i:i + 1])
    Tb = Tg.clone()
    sb = torch.full((nsteps,), -1, dtype=torch.int32, device="cuda:0")
    plan.supersteps_async(Tb, bg, dt, nsteps, cap, s_out=sb)
    torch.cuda.synchronize()
    out = (Ta, sa, Tb, sb, T0, b, p, h, dt, plan)
    return out


@pytest.mark.parametrize("case", range(len(CASES)))
def test_same_bits_as_single_calls(torch_cuda, case):
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n, ndim, bnd, precision, variant = CASES[case]
    print("case", case, n, ndim, bnd, precision, "variant", variant, flush=True)
    Ta, sa, Tb, sb, T0, b, p, h, dt, plan = run_pair(torch, rkl, n, ndim, bnd, precision, variant, 5, 30.0)
    ss = sa.cpu().numpy()
    assert ss.min() >= 3, ss                      # real super-steps
    assert torch.equal(sa, sb), (ss, sb.cpu().numpy())
    assert torch.equal(Ta, Tb)
    assert not torch.equal(Tb, torch.from_numpy(T0).to("cuda:0"))
    plan.close()


def test_fp64_against_the_oracle(torch_cuda):
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n, ndim, bnd = (40, 33, 23), 3, (0, 0, 0)
    Ta, sa, Tb, sb, T0, b, p, h, dt, plan = run_pair(torch, rkl, n, ndim, bnd, "fp64", 3, 3, 20.0)
    g = oracle_grid(n, h, ndim, p)
    T = T0
    for i in range(3):
        T, s, _ = oracle.superstep(g, T, b, dt)
        assert s == int(sb[i].item())
    err = rel_l1(Tb.cpu().numpy(), T)
    print("rel-L1 after 3 super-steps: %.3e" % err, flush=True)
    assert err <= 1e-12
    plan.close()


def test_two_calls_and_interleaved_single_calls(torch_cuda):
    """the kept extrema belong to one call: a second call, and single calls in
    between, give the same bits as single calls throughout"""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n = (32, 24, 40)
    T0, b = fields(n, 11)
    p = dict(inputs.SPITZER_MC_SAT, kperp_ratio=0.01)
    h = tuple(1.0 / v for v in n)
    plan = rkl.Plan([lib_desc(n, h, 3, p)], precision="mixed", variant=1)
    bg = torch.from_numpy(b.astype(np.float32)).to("cuda:0")
    Tg = torch.from_numpy(T0).to("cuda:0")
    dt = 25.0 * plan.dt_par(Tg)
    Ta = Tg.clone()
    for _ in range(3 + 1 + 2):
        plan.superstep_async(Ta, bg, dt, 64)
    Tb = Tg.clone()
    plan.supersteps_async(Tb, bg, dt, 3, 64)
    plan.superstep_async(Tb, bg, dt, 64)
    plan.supersteps_async(Tb, bg, dt, 2, 64)
    torch.cuda.synchronize()
    assert torch.equal(Ta, Tb)
    plan.close()


def test_stage_cap_exceeded(torch_cuda):
    """s above s_cap: every super-step leaves T as it is and reports its s;
    the flag is set, and the reduction runs again each time"""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n = (24, 24, 24)
    T0, b = fields(n, 5)
    p = dict(inputs.SPITZER_MC_SAT, kperp_ratio=0.01)
    h = tuple(1.0 / v for v in n)
    plan = rkl.Plan([lib_desc(n, h, 3, p)], precision="mixed")
    bg = torch.from_numpy(b.astype(np.float32)).to("cuda:0")
    Tg = torch.from_numpy(T0).to("cuda:0")
    dt = 200.0 * plan.dt_par(Tg)
    s_out = torch.zeros(3, dtype=torch.int32, device="cuda:0")
    plan.supersteps_async(Tg, bg, dt, 3, 8, s_out=s_out)
    torch.cuda.synchronize()
    ss = s_out.cpu().numpy()
    assert (ss > 8).all() and (ss == ss[0]).all(), ss
    assert np.array_equal(Tg.cpu().numpy(), T0)
    _, _, flags = plan.query()
    assert flags & rkl.RKL_FLAG_STAGES
    plan.close()


@pytest.mark.parametrize("precision,variant", [("mixed", 3), ("fp64", 1)])
def test_non_finite_extrema_from_the_last_stage(torch_cuda, precision, variant):
    """A NaN in the starting T: the first super-step's reduction pass flags
    it on both routes, and the stage recurrence keeps that cell NaN, so every
    later super-step's extrema carry the flag too: from the last stage within
    one rkl_supersteps_async call, from the reduction pass between single
    calls.  Stage counts, dt_par, flags and every bit of T (NaN included)
    must agree between the two routes."""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n = (40, 33, 23)
    T0, b = fields(n, 9)
    T0[11, 20, 17] = np.nan
    p = dict(inputs.SPITZER_MC_SAT, kperp_ratio=0.01)
    h = tuple(1.0 / v for v in n)
    bg = torch.from_numpy(b).to("cuda:0", torch.float32 if precision == "mixed" else torch.float64)
    plans = [rkl.Plan([lib_desc(n, h, 3, p)], precision=precision, variant=variant) for _ in range(2)]
    Ts = [torch.from_numpy(T0).to("cuda:0") for _ in range(2)]
    dt = inputs.midpoint_ratio(6) * plans[0].dt_par(Ts[0])
    s_one = torch.zeros(3, dtype=torch.int32, device="cuda:0")
    flags_one = []
    for i in range(3):
        plans[0].superstep_async(Ts[0], bg, dt, 12, s_out=s_one[i:i + 1])
        flags_one.append(plans[0].query()[2])
    s_many = torch.zeros(3, dtype=torch.int32, device="cuda:0")
    plans[1].supersteps_async(Ts[1], bg, dt, 3, 12, s_out=s_many)
    torch.cuda.synchronize()
    q = [pl.query() for pl in plans]
    for pl in plans:
        pl.close()
    print(precision, "stages", s_one.tolist(), "flags per super-step", flags_one, "query", q, flush=True)
    assert s_one.tolist() == s_many.tolist() and s_one.tolist()[0] == 6
    assert all(f & rkl.RKL_FLAG_NONFINITE for f in flags_one)
    assert q[0] == q[1]
    a, c = (t.cpu().numpy() for t in Ts)
    assert np.isnan(a[11, 20, 17]) and not np.isinf(a).any()
    assert np.array_equal(a.view(np.int64), c.view(np.int64))


def test_refusals(torch_cuda):
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n = (16, 16, 16)
    T0, b = fields(n, 1)
    plan = rkl.Plan([lib_desc(n, (1 / 16,) * 3, 3, dict(inputs.SPITZER_MC))], precision="fp64")
    Tg = torch.from_numpy(T0).to("cuda:0")
    bg = torch.from_numpy(b).to("cuda:0")
    for nsteps, cap in ((0, 16), (2, 1), (2, 100000)):
        with pytest.raises(rkl.RklError):
            plan.supersteps_async(Tg, bg, 1e-3, nsteps, cap)
    plan.close()


def test_in_a_captured_graph(torch_cuda):
    """captured once (three super-steps), replayed four times with eager
    library work between the replays; each replay equals three eager
    super-steps, so the kept extrema work across replays too"""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n = (48, 40, 24)
    h = tuple(1.0 / v for v in n)
    T0, b = fields(n, 9)
    p = dict(inputs.SPITZER_MC_SAT, kperp_ratio=0.01)
    plan = rkl.Plan([lib_desc(n, h, 3, p)], precision="mixed", smax=64)
    ref_plan = rkl.Plan([lib_desc(n, h, 3, p)], precision="mixed", smax=64)
    T = torch.from_numpy(T0.copy()).to("cuda:0")
    bg = torch.from_numpy(b.astype(np.float32)).to("cuda:0")
    dt = inputs.midpoint_ratio(10) * plan.dt_par(T)
    s_dev = torch.zeros(3, dtype=torch.int32, device="cuda:0")
    Tref = T.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.supersteps_async(T, bg, dt, 3, 14, s_out=s_dev)   # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(side)
    for _ in range(3):
        ref_plan.superstep(Tref, bg, dt)
    torch.cuda.synchronize()
    assert torch.equal(T, Tref)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.supersteps_async(T, bg, dt, 3, 14, s_out=s_dev)
    for rep in range(4):
        graph.replay()
        ss = []
        for _ in range(3):
            ss.append(ref_plan.superstep(Tref, bg, dt))      # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(T, Tref), rep
        assert s_dev.cpu().tolist() == ss, (rep, s_dev.cpu().tolist(), ss)
    plan.close()
    ref_plan.close()
