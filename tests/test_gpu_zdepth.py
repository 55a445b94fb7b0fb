"""Thin and ragged z-depths of the 3-D stage kernels against the oracle.

The 3-D stage kernels walk each tile's z-chunk (16, 32 or 64 planes,
by variant) plane by plane with the loop unrolled six-fold; a chunk whose
length is not a multiple of six ends in a shorter remainder, and the
temperature planes ahead of the current one wrap around a periodic z axis
(or repeat the edge plane of an outflow one).  The depths below give chunk
lengths of every remainder modulo six, down to a single plane, where the
planes k-1, k and k+1 are all one plane.  x and y are ragged too (37 x 11
against tiles of 16, 32 and 64 cells across).

  - FP64: the same bits in every one-stage variant, super-step rel-L1 <=
    1e-12 against the oracle and the change over it <= 1e-10 (Appendix A,
    Sec. 3.3 Eq. RKL-s for the stage count, which must agree);
  - mixed: the same bits in every one-stage variant, rel-L1 <= 1e-5, and
    of the change <= 1e-5, against the oracle fed the FP32-rounded unit
    vectors (measured: about 2e-10 and 2e-7);
  - rkl_supersteps_async: the bits of the same number of single calls.
"""
import numpy as np
import pytest

import oracle
from helpers import lib_desc, oracle_grid, rel_l1
from paper_1702_05487_amd import inputs

pytestmark = pytest.mark.gpu

# chunk lengths (16/32/64-plane chunks) cover every remainder modulo 6
DEPTHS = (1, 2, 3, 4, 5, 6, 7, 11, 17, 23, 35, 70)
ZEDGES = {"periodic": (0, 0, 0), "outflow": (0, 0, 1)}
H = (0.03, 0.04, 0.05)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1702_05487_amd import rkl
    rkl.load(build_if_missing=False)
    return torch


def case(depth, zedge):
    n = (37, 11, depth)
    rng = np.random.default_rng(1000 + depth)
    shape = (n[2], n[1], n[0])
    T = 1.0 + 0.2 * rng.random(shape)
    b = inputs.unit_vectors(rng.standard_normal((3,) + shape))
    p = dict(inputs.SPITZER_MC_SAT, phi=0.003, boundary=ZEDGES[zedge])
    return n, p, T, b


def one_stage_variants():
    from paper_1702_05487_amd import rkl
    return [v for v in range(rkl.rkl_variant_count()) if rkl.rkl_variant_info(v)[3] == 1]


def library_superstep(torch, n, p, T, b, precision, variant, dt):
    from paper_1702_05487_amd import rkl
    plan = rkl.Plan([lib_desc(n, H, 3, p)], precision=precision, variant=variant)
    Td = torch.from_numpy(T).to("cuda:0")
    bd = torch.from_numpy(b).to("cuda:0", torch.float32 if precision == "mixed" else torch.float64)
    s = plan.superstep(Td, bd, dt)
    plan.close()
    return Td.cpu().numpy(), s


@pytest.mark.parametrize("zedge", sorted(ZEDGES))
@pytest.mark.parametrize("depth", DEPTHS)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_depth_every_variant(torch_cuda, precision, depth, zedge):
    print("z-depth", precision, depth, zedge, flush=True)
    n, p, T, b = case(depth, zedge)
    bo = b.astype(np.float32).astype(np.float64) if precision == "mixed" else b
    g = oracle_grid(n, H, 3, p)
    dt = inputs.midpoint_ratio(7) * oracle.dt_par(g, T)
    ref, s_ref, _ = oracle.superstep(g, T, bo, dt)
    base = None
    for v in one_stage_variants():
        got, s = library_superstep(torch_cuda, n, p, T, b, precision, v, dt)
        assert s == s_ref, v
        if base is None:
            base = got
            err = rel_l1(got, ref)
            chg = rel_l1(got - T, ref - T)
            print("  rel-L1 %.3e, change %.3e" % (err, chg))
            if precision == "fp64":
                assert err <= 1e-12 and chg <= 1e-10
            else:
                assert err <= 1e-5 and chg <= 1e-5
        else:
            assert np.array_equal(got, base), v


@pytest.mark.parametrize("zedge", sorted(ZEDGES))
@pytest.mark.parametrize("depth", (1, 2, 5, 17, 70))
def test_depth_chained_supersteps(torch_cuda, depth, zedge):
    """three super-steps in one rkl_supersteps_async call against three
    rkl_superstep_async calls (mixed, the 64 x 4 x 64 tile)"""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n, p, T, b = case(depth, zedge)
    g = oracle_grid(n, H, 3, p)
    dt = inputs.midpoint_ratio(7) * oracle.dt_par(g, T)
    bd = torch.from_numpy(b).to("cuda:0", torch.float32)
    plan = rkl.Plan([lib_desc(n, H, 3, p)], precision="mixed", variant=3)
    one = torch.from_numpy(T).to("cuda:0")
    s_one = torch.zeros(3, dtype=torch.int32, device="cuda:0")
    for i in range(3):
        plan.superstep_async(one, bd, dt, 12, s_one[i:i + 1])
    many = torch.from_numpy(T).to("cuda:0")
    s_many = torch.zeros(3, dtype=torch.int32, device="cuda:0")
    plan.supersteps_async(many, bd, dt, 3, 12, s_many)
    torch.cuda.synchronize()
    plan.close()
    assert s_one.tolist() == s_many.tolist()
    assert all(1 <= s <= 12 for s in s_one.tolist())
    assert torch.equal(one, many)
