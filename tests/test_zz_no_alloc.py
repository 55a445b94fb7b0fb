"""rkl_superstep_noalloc (static scratch, no plan, no allocation) against
rkl_superstep on the same fields: two calls in a row, the second on a
smaller grid, each compared with a plan's super-step (stencil variant 0).

Bars: FP64 rel-L1 <= 1e-12 and mixed <= 1e-5 (both run the same kernels in
the same order, so the results are in fact the same bits, also checked);
identical stage counts.  Sizes beyond the static scratch are refused before
anything runs on the device."""
import numpy as np
import pytest

from helpers import lib_desc, rel_l1
from paper_1702_05487_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1702_05487_amd import rkl
    rkl.load(build_if_missing=False)
    return torch


def run_pair(torch, n, ndim, params, precision, s):
    from paper_1702_05487_amd import rkl
    h = tuple(1.0 / v for v in n)
    T0 = inputs.noisy_temperature(n, 11, kmax=6)
    b = inputs.tangled_b(n, 12, kmax=6)
    bd = b.astype(np.float32) if precision == "mixed" else b
    desc = lib_desc(n, h, ndim, params)
    plan = rkl.Plan([desc], precision=precision, variant=0)
    Tn = torch.from_numpy(T0.copy()).to("cuda:0")
    Tp = Tn.clone()
    bg = torch.from_numpy(np.ascontiguousarray(bd)).to("cuda:0")
    dt = inputs.midpoint_ratio(s) * plan.dt_par(Tp)
    s_dev = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
    rkl.superstep_noalloc(desc, Tn, bg, dt, s_cap=s + 4, s_out=s_dev, precision=precision)
    s_ref = plan.superstep(Tp, bg, dt)
    torch.cuda.synchronize()
    err = rel_l1(Tn.cpu().numpy(), Tp.cpu().numpy())
    print("noalloc %s %s: s %d/%d, rel-L1 vs rkl_superstep %.3e" % (precision, n, int(s_dev.item()), s_ref, err))
    assert int(s_dev.item()) == s_ref == s
    assert err <= (1e-12 if precision == "fp64" else 1e-5)
    assert torch.equal(Tn, Tp)
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_two_calls_second_smaller(torch_cuda, precision):
    torch = torch_cuda
    # 2^21 cells (the limit) first, then a ragged smaller grid with outflow axes
    run_pair(torch, (128, 128, 128), 3, inputs.SPITZER_MC_SAT, precision, 9)
    run_pair(torch, (37, 29, 23), 3, dict(inputs.SPITZER_MC, boundary=(1, 0, 1)), precision, 6)


def test_noalloc_refuses_beyond_its_limits(torch_cuda):
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    big = lib_desc((128, 128, 129), (1 / 128, 1 / 128, 1 / 129), 3, inputs.SPITZER_MC)
    T = torch.ones(128 * 128 * 129, dtype=torch.float64, device="cuda:0")
    b = torch.zeros(3 * 128 * 128 * 129, dtype=torch.float64, device="cuda:0")
    with pytest.raises(rkl.RklError) as e:
        rkl.superstep_noalloc(big, T, b, 1e-6, s_cap=8)
    assert "RKL_NOALLOC_MAX_CELLS" in str(e.value)
    small = lib_desc((8, 8, 8), (1 / 8,) * 3, 3, inputs.SPITZER_MC)
    with pytest.raises(rkl.RklError) as e:
        rkl.superstep_noalloc(small, T[:512], b[:1536], 1e-6, s_cap=257)
    assert "RKL_NOALLOC_MAX_STAGES" in str(e.value)
