"""RKL1 super-steps (plan scheme RKL_RKL1) vs the oracle's, through the C ABI.

Bars as for RKL2: FP64 rel-L1 <= 1e-12, mixed <= 1e-5, identical stage
counts (s = 1, a forward-Euler step, included); every variant, one- or
two-stage, gives the same bits."""
import numpy as np
import pytest

import oracle
from helpers import lib_desc, oracle_grid, rel_l1
from test_gpu_parity import make_case, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1702_05487_amd import rkl
    rkl.load(build_if_missing=False)
    return torch


def pair(torch, name, precision, ratio, steps=1, variant=-1):
    from paper_1702_05487_amd import rkl
    n, h, ndim, p, T, b = make_case(name)
    g = oracle_grid(n, h, ndim, p)
    bg = b.astype(np.float32) if precision == "mixed" else b
    plan = rkl.Plan([lib_desc(n, h, ndim, p)], precision=precision, variant=variant, scheme="rkl1")
    Td = to_dev(torch, T, torch.float64)
    bd = to_dev(torch, bg, torch.float32 if precision == "mixed" else torch.float64)
    To = T.copy()
    svals = []
    for _ in range(steps):
        dt = ratio * oracle.dt_par(g, To)
        To, s_ref, _ = oracle.superstep_rkl1(g, To, bg.astype(np.float64), dt)
        s = plan.superstep(Td, bd, dt)
        assert s == s_ref
        svals.append(s)
    plan.close()
    return Td.cpu().numpy(), To, T, svals


@pytest.mark.parametrize("name,ratio,steps", [
    ("tangled_mc", 40.0, 2), ("tangled_mc_sat", 12.0, 1), ("gauss2d", 50.0, 3), ("iso1d", 20.0, 2),
    ("flat2d_ragged", 9.0, 1), ("tiny3d", 0.6, 2), ("tangled_mc", 1.5, 1),
])
def test_rkl1_fp64(torch_cuda, name, ratio, steps):
    print("rkl1 fp64", name, ratio, steps, flush=True)
    g, o, T0, s = pair(torch_cuda, name, "fp64", ratio, steps)
    assert s[0] == oracle.stages_rkl1(ratio)
    assert rel_l1(g, o) <= 1e-12
    assert rel_l1(g - T0, o - T0) <= 1e-10


def test_rkl1_one_stage_is_forward_euler(torch_cuda):
    g, o, T0, s = pair(torch_cuda, "tangled_mc_sat", "fp64", 0.7)
    assert s == [1]
    assert rel_l1(g, o) <= 1e-12


@pytest.mark.parametrize("name,ratio", [("tangled_mc", 40.0), ("tangled_mc_sat", 90.0), ("gauss2d", 50.0)])
def test_rkl1_mixed(torch_cuda, name, ratio):
    g, o, T0, s = pair(torch_cuda, name, "mixed", ratio)
    err = rel_l1(g, o)
    print("rkl1 mixed", name, s, "rel-L1 %.3e" % err, flush=True)
    assert err <= 1e-5


def test_rkl1_every_variant_gives_the_same_bits(torch_cuda):
    ref = pair(torch_cuda, "tangled_mc_sat", "mixed", 30.0, variant=0)[0]
    for v in (1, 4, 8, 9, 10, 11):
        assert np.array_equal(pair(torch_cuda, "tangled_mc_sat", "mixed", 30.0, variant=v)[0], ref), v


def test_rkl1_batched_is_rejected_but_per_grid_works(torch_cuda):
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n, h, ndim, p, T, b = make_case("tiny3d")
    plan = rkl.Plan([lib_desc(n, h, ndim, p)] * 2, scheme="rkl1")
    T2 = to_dev(torch, np.concatenate([T.ravel(), T.ravel()]), torch.float64)
    b2 = to_dev(torch, np.concatenate([b.ravel(), b.ravel()]), torch.float64)
    dt = torch.full((2,), 1e-3, dtype=torch.float64, device="cuda:0")
    with pytest.raises(rkl.RklError) as e:
        plan.superstep_batched(T2, b2, dt)
    assert e.value.status == rkl.RKL_EINVAL
    Td = to_dev(torch, T, torch.float64)
    bd = to_dev(torch, b, torch.float64)
    g = oracle_grid(n, h, ndim, p)
    dtv = 5.0 * oracle.dt_par(g, T)
    s = plan.superstep(Td, bd, dtv, grid=1)
    To, s_ref, _ = oracle.superstep_rkl1(g, T, b, dtv)
    assert s == s_ref and rel_l1(Td.cpu().numpy(), To) <= 1e-12
    plan.close()
