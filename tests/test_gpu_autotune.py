"""The autotuner (rkl_autotune through the C ABI, and the JSON cache of
tune.py) on the GPU."""
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


def case(torch, precision):
    n = (40, 36, 34)
    h = tuple(1.0 / v for v in n)
    p = dict(inputs.SPITZER_MC_SAT, phi=0.01)
    T = inputs.noisy_temperature(n, 21, kmax=6)
    b = inputs.tangled_b(n, 22, kmax=6)
    bdt = torch.float32 if precision == "mixed" else torch.float64
    bh = b.astype(np.float32) if precision == "mixed" else b
    return n, h, p, T, bh, torch.from_numpy(T).to("cuda:0"), torch.from_numpy(bh).to("cuda:0", dtype=bdt)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotune_picks_a_usable_variant_and_keeps_results(torch_cuda, precision):
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n, h, p, T, bh, Td, bd = case(torch, precision)
    plan = rkl.Plan([lib_desc(n, h, 3, p)], precision=precision)
    dt = inputs.midpoint_ratio(9) * plan.dt_par(Td)
    T_before = Td.clone()
    v, ms = rkl.rkl_autotune(plan.handle, 0, *plan._tb(0, Td, bd), dt, 1,
                             rkl.ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert torch.equal(Td, T_before)               # the caller's T is not touched
    assert 0 <= v < rkl.rkl_variant_count() and ms > 0
    if precision == "fp64":
        assert rkl.rkl_variant_info(v)[3] == 1     # two-stage variants need RKL_MIXED
    # the plan now runs the chosen variant; the answer is the oracle's
    s = plan.superstep(Td, bd, dt)
    g = oracle_grid(n, h, 3, p)
    To, s_ref, _ = oracle.superstep(g, T, bh.astype(np.float64), dt)
    assert s == s_ref == 9
    assert rel_l1(Td.cpu().numpy(), To) <= (1e-12 if precision == "fp64" else 1e-5)
    with pytest.raises(rkl.RklError) as e:
        rkl.rkl_autotune(plan.handle, 0, *plan._tb(0, Td, bd), dt, 0,
                         rkl.ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert e.value.status == rkl.RKL_EINVAL
    plan.close()


def test_tune_cache_round_trip(torch_cuda, tmp_path):
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n, h, p, T, bh, Td, bd = case(torch, "mixed")
    cache = str(tmp_path / "tune.json")
    plan = rkl.Plan([lib_desc(n, h, 3, p)], precision="mixed")
    dt = inputs.midpoint_ratio(7) * plan.dt_par(Td)
    v1, ms1, cached1 = plan.autotune(Td, bd, dt, reps=1, cache=cache)
    assert not cached1
    plan2 = rkl.Plan([lib_desc(n, h, 3, p)], precision="mixed")
    v2, ms2, cached2 = plan2.autotune(Td, bd, dt, reps=1, cache=cache)
    assert cached2 and v2 == v1 and ms2 == ms1
    plan.close()
    plan2.close()
