"""rkl_superstep_async: the super-step with its stage count kept on the device
(no host synchronisation, graph-capturable) against rkl_superstep and the
oracle.

Bars: the same bits as rkl_superstep for the same stencil variant (both run
the same kernels in the same order; only the choice of stage buffers moves
to the device); against the oracle rel-L1 <= 1e-12 (FP64) and <= 1e-5
(mixed, oracle fed the FP32-rounded unit vectors); identical stage counts.
"""
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
    T = inputs.noisy_temperature(n, seed, kmax=6)
    b = inputs.tangled_b(n, seed + 1, kmax=6)
    return T, b


CASES = [
    ("fp64", (40, 36, 21), inputs.SPITZER_MC, 3, 9),
    ("mixed", (40, 36, 21), inputs.SPITZER_MC_SAT, 3, 12),
    ("fp64", (45, 29, 1), dict(inputs.SPITZER_MC_SAT, kperp_ratio=0.05), 2, 7),
    ("mixed", (33, 17, 70), dict(inputs.SPITZER_MC, boundary=(1, 0, 1)), 3, 5),
]


@pytest.mark.parametrize("precision,n,params,ndim,s", CASES)
def test_async_equals_superstep_and_oracle(torch_cuda, precision, n, params, ndim, s):
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    h = tuple(1.0 / v for v in n)
    T0, b = fields(n, 5)
    bdev = b.astype(np.float32) if precision == "mixed" else b
    plan = rkl.Plan([lib_desc(n, h, ndim, params)], precision=precision, smax=64)
    Ta = torch.from_numpy(T0.copy()).to("cuda:0")
    Tb = Ta.clone()
    bg = torch.from_numpy(np.ascontiguousarray(bdev)).to("cuda:0")
    dt = inputs.midpoint_ratio(s) * plan.dt_par(Ta)
    s_dev = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    for step in range(2):
        plan.superstep_async(Ta, bg, dt, s_cap=s + 3, s_out=s_dev)
        s_sync = plan.superstep(Tb, bg, dt)
        assert int(s_dev.item()) == s_sync
        assert torch.equal(Ta, Tb), step
    g = oracle_grid(n, h, ndim, params)
    ref = T0
    for _ in range(2):
        ref, s_ref, _ = oracle.superstep(g, ref, bdev.astype(np.float64), dt)
    err = rel_l1(Ta.cpu().numpy(), ref)
    print("%s %s: s %d/%d, rel-L1 vs oracle %.3e" % (precision, n, int(s_dev.item()), s_ref, err))
    assert int(s_dev.item()) == s_ref
    assert err <= (1e-12 if precision == "fp64" else 1e-5)
    plan.close()


def test_async_stage_cap_leaves_T_unchanged(torch_cuda):
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n = (24, 20, 16)
    h = tuple(1.0 / v for v in n)
    T0, b = fields(n, 7)
    plan = rkl.Plan([lib_desc(n, h, 3, inputs.SPITZER_MC)], precision="fp64", smax=64)
    T = torch.from_numpy(T0.copy()).to("cuda:0")
    bg = torch.from_numpy(b).to("cuda:0")
    dt = inputs.midpoint_ratio(20) * plan.dt_par(T)
    s_dev = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    plan.superstep_async(T, bg, dt, s_cap=12, s_out=s_dev)
    assert int(s_dev.item()) == 20
    assert torch.equal(T.cpu(), torch.from_numpy(T0))
    s, _, flags = plan.query()
    assert s == 20 and flags & rkl.RKL_FLAG_STAGES
    with pytest.raises(rkl.RklError):
        plan.superstep_async(T, bg, dt, s_cap=65)   # above the plan's smax
    with pytest.raises(rkl.RklError):
        plan.superstep_async(T, bg, dt, s_cap=1)
    plan.close()


def test_async_in_a_captured_graph(torch_cuda):
    # captured once into a torch CUDA graph, replayed five times with eager
    # library work in between; every replay equals the eager super-step
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n = (48, 40, 24)
    h = tuple(1.0 / v for v in n)
    T0, b = fields(n, 9)
    plan = rkl.Plan([lib_desc(n, h, 3, inputs.SPITZER_MC_SAT)], precision="mixed", smax=64)
    ref_plan = rkl.Plan([lib_desc(n, h, 3, inputs.SPITZER_MC_SAT)], precision="mixed", smax=64)
    T = torch.from_numpy(T0.copy()).to("cuda:0")
    bg = torch.from_numpy(b.astype(np.float32)).to("cuda:0")
    dt = inputs.midpoint_ratio(10) * plan.dt_par(T)
    s_dev = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    Tref = T.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        plan.superstep_async(T, bg, dt, s_cap=14, s_out=s_dev)   # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(side)
    ref_plan.superstep(Tref, bg, dt)
    assert torch.equal(T, Tref)
    with torch.cuda.graph(graph):
        plan.superstep_async(T, bg, dt, s_cap=14, s_out=s_dev)
    for rep in range(5):
        graph.replay()
        ref_plan.superstep(Tref, bg, dt)      # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(T, Tref), rep
        assert int(s_dev.item()) == ref_plan.query()[0]
    plan.close()
    ref_plan.close()
