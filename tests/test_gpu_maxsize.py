"""A grid beyond 2^31 cells (2048 x 2048 x 520 = 2.18e9 cells, 17 GB per FP64
field; the descriptor limit is 2^32 cells): one super-step through the C
ABI, checked against the oracle at sampled cells whose linear index is
above 2^31, so every address computation must be 64-bit.  Mixed precision
with a one-stage and a two-stage variant (same bits), and FP64."""
import math

import numpy as np
import pytest

import oracle
from helpers import lib_desc, rel_l1
from paper_1702_05487_amd import inputs

pytestmark = pytest.mark.gpu

N = (2048, 2048, 520)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1702_05487_amd import rkl
    rkl.load(build_if_missing=False)
    return torch


def fields(torch, bdtype):
    """smooth periodic T and b built from broadcast 1-D factors on the GPU"""
    n0, n1, n2 = N
    dev = "cuda:0"
    x = (torch.arange(n0, device=dev, dtype=torch.float64) + 0.5) / n0
    y = (torch.arange(n1, device=dev, dtype=torch.float64) + 0.5) / n1
    z = (torch.arange(n2, device=dev, dtype=torch.float64) + 0.5) / n2
    tp = 2 * math.pi
    T = torch.empty((n2, n1, n0), dtype=torch.float64, device=dev)
    torch.add(0.05 * torch.sin(tp * (x[None, None, :] + 2 * y[None, :, None])),
              1.0 + 0.05 * torch.cos(tp * (3 * z[:, None, None] + y[None, :, None])), out=T)
    th = (tp * (x[None, None, :] + z[:, None, None])).to(bdtype)          # (n2, 1, n0)
    ph = (math.pi / 3 + 0.3 * torch.sin(tp * y)).to(bdtype)[None, :, None]  # (1, n1, 1)
    b = torch.empty((3, n2, n1, n0), dtype=bdtype, device=dev)
    torch.mul(torch.cos(th), torch.sin(ph), out=b[0])
    torch.mul(torch.sin(th), torch.sin(ph), out=b[1])
    b[2].copy_(torch.cos(ph).expand(n2, n1, n0))
    return T, b


def window(torch, t, center, r):
    lead = t.dim() - 3
    a = t
    for ax, c in enumerate(center):
        n = t.shape[lead + ax]
        idx = torch.arange(c - r, c + r + 1, device=t.device) % n
        a = a.index_select(lead + ax, idx)
    return a.double().cpu().numpy()


CENTERS = [(519, 2047, 2047), (300, 5, 1000), (519, 0, 0), (260, 1024, 7), (10, 10, 10)]   # (k, j, i)


def check(torch, precision, variants):
    from paper_1702_05487_amd import rkl
    params = dict(inputs.SPITZER_MC_SAT, phi=0.01)
    h = tuple(1.0 / v for v in N)
    T0, b = fields(torch, torch.float32 if precision == "mixed" else torch.float64)
    plan = rkl.Plan([lib_desc(N, h, 3, params)], precision=precision)
    dt = inputs.midpoint_ratio(4) * plan.dt_par(T0)
    s = 4
    r = s + 1
    plane = N[0] * N[1]
    assert max(k * plane + j * N[0] + i for k, j, i in CENTERS) > 2 ** 31
    ref = []
    for c in CENTERS:
        win = oracle.Grid(n=(2 * r + 1,) * 3, h=h, ndim=3, **params)
        ref.append(oracle.rkl2_fixed(win, window(torch, T0, c, r), window(torch, b, c, r), s, dt)[r, r, r])
    ref = np.array(ref)
    idx = tuple(torch.tensor(np.array(CENTERS).T, device="cuda:0"))
    t0 = T0[idx].cpu().numpy()
    first = None
    for v in variants:
        plan.set_variant(v)
        T = T0.clone()
        assert plan.superstep(T, b, dt) == s
        got = T[idx].cpu().numpy()
        print("  %s variant %d: max |diff| %.3e, max |change| %.3e, change rel-L1 %.3e"
              % (precision, v, np.abs(got - ref).max(), np.abs(ref - t0).max(), rel_l1(got - t0, ref - t0)),
              flush=True)
        # the change over one super-step at h = 1/2048 is ~3e-8 of T, so one
        # FP64 rounding of T (~2e-16) is already ~1e-8 of the change, and the
        # FP32 flux arithmetic (2^-24 of the offset temperatures, ~6e-9 here)
        # a few 1e-3 of it (3.9e-3 measured; 1e-10 absolute)
        if precision == "mixed":
            assert np.abs(got - ref).max() <= 1e-8
            assert rel_l1(got - t0, ref - t0) <= 1e-2
        else:
            assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
            assert rel_l1(got - t0, ref - t0) <= 1e-6
        if first is None:
            first = T
        else:
            assert torch.equal(first, T)
            del T
    plan.close()
    del T0, b, first
    torch.cuda.empty_cache()


def test_beyond_2_31_cells_mixed(torch_cuda):
    print("2048x2048x520 mixed", flush=True)
    check(torch_cuda, "mixed", [0, 8])


def test_beyond_2_31_cells_fp64(torch_cuda):
    print("2048x2048x520 fp64", flush=True)
    check(torch_cuda, "fp64", [0])
