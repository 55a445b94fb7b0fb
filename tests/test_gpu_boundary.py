"""Outflow boundaries (per axis: ghost cells repeat the edge cell's T and b
at every stage) on the GPU through the C ABI, against the oracle's outflow
form.

Bars: FP64 rel-L1 <= 1e-12, mixed <= 1e-5, identical stage counts (RKL2,
and RKL1, AAG and sub-cycling in FP64); every
one-stage variant and the batched launch give the same bits; two-stage
variants are refused for grids that are not periodic.
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


def make_case(name):
    """(n, h, ndim, params, T, b) of a small case with outflow axes"""
    if name == "3d_xz_open_ragged":      # several tiles, ragged x/y tails, z chunks
        n = (45, 27, 40)
        p = dict(inputs.SPITZER_MC_SAT, phi=0.003, boundary=(1, 0, 1))
        return n, (0.03, 0.04, 0.05), 3, p, inputs.noisy_temperature(n, 4, kmax=4), inputs.tangled_b(n, 3, kmax=4)
    if name == "3d_all_open_upwind":
        n = (33, 20, 17)
        p = dict(inputs.SPITZER_MC_SAT, saturation=2, phi=0.01, boundary=(1, 1, 1))
        return n, (0.04, 0.03, 0.05), 3, p, inputs.noisy_temperature(n, 6, kmax=4), inputs.tangled_b(n, 5, kmax=4)
    if name == "3d_y_open_mean":
        n = (30, 26, 21)
        p = dict(inputs.BASE, kappa_exp=2.5, kperp_ratio=0.02, boundary=(0, 1, 0))
        return n, (0.05, 0.04, 0.03), 3, p, inputs.noisy_temperature(n, 8, kmax=5), inputs.tangled_b(n, 7, kmax=5)
    if name == "2d_both_open":
        rng = np.random.default_rng(17)
        n = (45, 29, 1)
        T = inputs.noisy_temperature(n, 6, kmax=6)
        B = rng.standard_normal((3, 1, 29, 45))
        B[2] = 0.0
        p = dict(inputs.SPITZER_MC_SAT, kperp_ratio=0.05, boundary=(1, 1, 0))
        return n, (0.02, 0.03, 1.0), 2, p, T, inputs.unit_vectors(B)
    if name == "1d_open":
        rng = np.random.default_rng(19)
        n = (50, 1, 1)
        T = 1.0 + 0.5 * rng.random((1, 1, 50))
        b = np.zeros((3, 1, 1, 50))
        b[0] = 1.0
        return n, (0.02, 1.0, 1.0), 1, dict(inputs.BASE, kappa_exp=2.5, boundary=(1, 0, 0)), T, b
    if name == "tiny3d_open":           # narrower than every tile
        rng = np.random.default_rng(23)
        n = (5, 3, 4)
        T = 1.0 + 0.2 * rng.random((4, 3, 5))
        b = inputs.unit_vectors(rng.standard_normal((3, 4, 3, 5)))
        return n, (0.2, 0.3, 0.25), 3, dict(inputs.SPITZER_MC_SAT, phi=0.01, boundary=(1, 1, 1)), T, b
    raise KeyError(name)


CASES = ["3d_xz_open_ragged", "3d_all_open_upwind", "3d_y_open_mean", "2d_both_open", "1d_open", "tiny3d_open"]


def to_dev(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda:0", dtype=dtype)


def run(torch, name, precision, ratio, steps=1, variant=-1):
    from paper_1702_05487_amd import rkl
    n, h, ndim, p, T, b = make_case(name)
    bg = b.astype(np.float32) if precision == "mixed" else b
    plan = rkl.Plan([lib_desc(n, h, ndim, p)], precision=precision, variant=variant)
    Td = to_dev(torch, T, torch.float64)
    bd = to_dev(torch, bg, torch.float32 if precision == "mixed" else torch.float64)
    g = oracle_grid(n, h, ndim, p)
    To, svals = T.copy(), []
    for _ in range(steps):
        dt = ratio * oracle.dt_par(g, To)
        s = plan.superstep(Td, bd, dt)
        To, s_ref, _ = oracle.superstep(g, To, bg.astype(np.float64), dt)
        svals.append((s, s_ref))
    plan.close()
    return Td.cpu().numpy(), To, T, svals


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
@pytest.mark.parametrize("name", CASES)
def test_outflow_flux_div(torch_cuda, name, precision, tol):
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n, h, ndim, p, T, b = make_case(name)
    bg = b.astype(np.float32) if precision == "mixed" else b
    ref = oracle.flux_div(oracle_grid(n, h, ndim, p), T, bg.astype(np.float64))
    per = oracle.flux_div(oracle_grid(n, h, ndim, dict(p, boundary=(0, 0, 0))), T, bg.astype(np.float64))
    assert rel_l1(per, ref) > 1e-4                 # the boundaries matter here
    plan = rkl.Plan([lib_desc(n, h, ndim, p)], precision=precision)
    got = plan.flux_div(to_dev(torch, T, torch.float64),
                        to_dev(torch, bg, torch.float32 if precision == "mixed" else torch.float64)).cpu().numpy()
    plan.close()
    print("outflow flux_div", name, precision, "rel-L1 %.3e" % rel_l1(got, ref))
    assert rel_l1(got, ref) <= tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
@pytest.mark.parametrize("name,steps,s", [
    ("3d_xz_open_ragged", 2, 9), ("3d_all_open_upwind", 1, 7), ("3d_y_open_mean", 1, 11),
    ("2d_both_open", 2, 6), ("1d_open", 2, 12), ("tiny3d_open", 2, 4),
])
def test_outflow_superstep(torch_cuda, name, steps, s, precision, tol):
    print("outflow superstep", name, precision, flush=True)
    g, o, T0, svals = run(torch_cuda, name, precision, inputs.midpoint_ratio(s), steps)
    assert all(a == b for a, b in svals) and svals[0][0] == s
    print("  rel-L1 %.3e  change rel-L1 %.3e" % (rel_l1(g, o), rel_l1(g - T0, o - T0)))
    assert rel_l1(g, o) <= tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_outflow_every_variant_same_bits(torch_cuda, precision):
    from paper_1702_05487_amd import rkl
    ratio = inputs.midpoint_ratio(8)
    base = run(torch_cuda, "3d_xz_open_ragged", precision, ratio, variant=0)[0]
    for v in range(1, rkl.rkl_variant_count()):
        if rkl.rkl_variant_info(v)[3] >= 2:
            continue
        assert np.array_equal(run(torch_cuda, "3d_xz_open_ragged", precision, ratio, variant=v)[0], base), v


def test_two_stage_variants_refused_for_outflow(torch_cuda):
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n, h, ndim, p, T, b = make_case("3d_xz_open_ragged")
    with pytest.raises(rkl.RklError) as e:
        rkl.Plan([lib_desc(n, h, ndim, p)], precision="mixed", variant=8)
    assert e.value.status == rkl.RKL_EINVAL
    plan = rkl.Plan([lib_desc(n, h, ndim, p)], precision="mixed")
    Td = to_dev(torch, T, torch.float64)
    bd = to_dev(torch, b, torch.float32)
    v, _ = rkl.rkl_autotune(plan.handle, 0, *plan._tb(0, Td, bd), inputs.midpoint_ratio(8) * plan.dt_par(Td), 1,
                            rkl.ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rkl.rkl_variant_info(v)[3] == 1
    plan.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_outflow_batched(torch_cuda, precision, tol):
    """patches with their own boundaries (periodic, partly and fully open)
    in one batched super-step, against the oracle patch by patch"""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    ps = inputs.patch_set(9, seed=31, lo=8, hi=32, smin=2, smax=12)
    bnds = [(0, 0, 0), (1, 0, 0), (0, 1, 1), (1, 1, 1)]
    bdt = np.float32 if precision == "mixed" else np.float64
    descs, refs, svals, dts = [], [], [], []
    for k, n in enumerate(ps.n):
        p = dict(ps.params, boundary=bnds[k % len(bnds)])
        g = oracle_grid(n, (1 / 64,) * 3, 3, p)
        bk = ps.b[k].astype(bdt).astype(np.float64)
        dt = ps.ratio[k] * oracle.dt_par(g, ps.T[k])
        To, s, _ = oracle.superstep(g, ps.T[k], bk, dt)
        descs.append(lib_desc(n, (1 / 64,) * 3, 3, p))
        refs.append(To)
        svals.append(s)
        dts.append(dt)
    plan = rkl.Plan(descs, precision=precision, smax=16)
    T = torch.from_numpy(np.concatenate([t.ravel() for t in ps.T])).to("cuda:0")
    b = torch.from_numpy(np.concatenate([bb.astype(bdt).ravel() for bb in ps.b])).to("cuda:0")
    s_out = torch.zeros(len(ps.n), dtype=torch.int32, device="cuda:0")
    plan.superstep_batched(T, b, torch.tensor(dts, dtype=torch.float64, device="cuda:0"), s_out)
    got = T.cpu().numpy()
    off = plan.offsets()
    plan.close()
    assert list(s_out.cpu().numpy()) == svals
    for k in range(len(ps.n)):
        assert rel_l1(got[off[k]:off[k + 1]].reshape(refs[k].shape), refs[k]) <= tol, k


def test_outflow_96_full_grid(torch_cuda):
    """96^3, x and z outflow, y periodic, Spitzer conduction with MC and
    saturation, s = 16, FP64: the whole grid against the oracle"""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n = (96, 96, 96)
    h = tuple(1.0 / v for v in n)
    p = dict(inputs.SPITZER_MC_SAT, phi=0.01, boundary=(1, 0, 1))
    T = inputs.noisy_temperature(n, 2)
    b = inputs.tangled_b(n, 1)
    plan = rkl.Plan([lib_desc(n, h, 3, p)], precision="fp64")
    Td = to_dev(torch, T, torch.float64)
    dt = inputs.midpoint_ratio(16) * plan.dt_par(Td)
    assert plan.superstep(Td, to_dev(torch, b, torch.float64), dt) == 16
    plan.close()
    ref, s, _ = oracle.superstep(oracle_grid(n, h, 3, p), T, b, dt)
    got = Td.cpu().numpy()
    print("outflow 96^3: rel-L1 %.3e, change rel-L1 %.3e" % (rel_l1(got, ref), rel_l1(got - T, ref - T)))
    assert s == 16
    assert rel_l1(got, ref) <= 1e-12


@pytest.mark.parametrize("method", ["rkl1", "aag", "subcycle"])
def test_outflow_other_integrators(torch_cuda, method):
    """RKL1, AAG and explicit sub-cycling on a grid with outflow axes, FP64,
    against the oracle's same integrator"""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n, h, ndim, p, T, b = make_case("3d_all_open_upwind")
    g = oracle_grid(n, h, ndim, p)
    plan = rkl.Plan([lib_desc(n, h, ndim, p)], scheme="rkl1" if method == "rkl1" else "rkl2")
    Td = to_dev(torch, T, torch.float64)
    bd = to_dev(torch, b, torch.float64)
    dt = 9.0 * oracle.dt_par(g, T)
    if method == "rkl1":
        c = plan.superstep(Td, bd, dt)
        ref, c_ref, _ = oracle.superstep_rkl1(g, T, b, dt)
    elif method == "aag":
        c = plan.aag(Td, bd, dt, 0.01)
        ref, c_ref = oracle.aag_superstep(g, T, b, dt, 0.01)
    else:
        c = plan.subcycle(Td, bd, dt)
        ref, c_ref = oracle.subcycle(g, T, b, dt)
    plan.close()
    got = Td.cpu().numpy()
    print("outflow", method, c, "rel-L1 %.3e" % rel_l1(got, ref))
    assert c == c_ref
    assert rel_l1(got, ref) <= 1e-12
