"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Tolerances (rel-L1 = sum|gpu - oracle| / sum|oracle|):
  FP64 plans: super-step rel-L1 <= 1e-12, flux divergence <= 1e-12 with
  max |diff| <= 1e-11 max |ref|; identical stage counts.
  Mixed plans (FP32 flux, FP64 stage recurrence): super-step rel-L1 <= 1e-5.
"""
import zlib

import numpy as np
import pytest

import oracle
from helpers import lib_desc, oracle_grid, rel_l1, sampled_superstep
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
    """(n, h, ndim, params, T, b) for a named small case"""
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    if name == "gauss2d":
        w = inputs.gaussian_pulse_2d(64)
        return w.n, w.h, 2, dict(w.params), w.T, w.b
    if name == "tangled_mc":
        n = (48, 40, 36)
        return n, tuple(1.0 / v for v in n), 3, dict(inputs.SPITZER_MC), \
            inputs.noisy_temperature(n, 2, kmax=8), inputs.tangled_b(n, 1, kmax=8)
    if name == "tangled_mc_sat":
        n = (37, 23, 19)
        p = dict(inputs.SPITZER_MC_SAT, phi=0.003)   # saturation active in a fraction of faces
        return n, (0.03, 0.04, 0.05), 3, p, \
            inputs.noisy_temperature(n, 4, kmax=4), inputs.tangled_b(n, 3, kmax=4)
    if name == "iso1d":
        n = (50, 1, 1)
        T = 1.0 + 0.5 * rng.random((1, 1, 50))
        b = np.zeros((3, 1, 1, 50))
        b[0] = 1.0
        return n, (0.02, 1.0, 1.0), 1, dict(inputs.BASE, kappa_exp=2.5), T, b
    if name == "flat2d_ragged":
        n = (45, 29, 1)
        T = inputs.noisy_temperature(n, 6, kmax=6)
        b = inputs.unit_vectors(rng.standard_normal((3, 1, 29, 45)))
        return n, (0.02, 0.03, 1.0), 2, dict(inputs.SPITZER_MC_SAT, kperp_ratio=0.05), T, b
    if name == "tiny3d":
        n = (5, 3, 4)          # narrower than every tile: wrap inside one tile
        T = 1.0 + 0.2 * rng.random((4, 3, 5))
        b = inputs.unit_vectors(rng.standard_normal((3, 4, 3, 5)))
        return n, (0.2, 0.3, 0.25), 3, dict(inputs.SPITZER_MC_SAT, phi=0.01), T, b
    raise KeyError(name)


CASES = ["gauss2d", "tangled_mc", "tangled_mc_sat", "iso1d", "flat2d_ragged", "tiny3d"]


def to_dev(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda:0", dtype=dtype)


def run_plan(torch, n, h, ndim, params, precision, variant=-1):
    from paper_1702_05487_amd import rkl
    return rkl.Plan([lib_desc(n, h, ndim, params)], precision=precision, variant=variant)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("variant", [0, 2, 4])
def test_flux_div_fp64(torch_cuda, name, variant):
    torch = torch_cuda
    n, h, ndim, p, T, b = make_case(name)
    print("flux_div fp64", name, n, "variant", variant, flush=True)
    ref = oracle.flux_div(oracle_grid(n, h, ndim, p), T, b)
    plan = run_plan(torch, n, h, ndim, p, "fp64", variant)
    out = plan.flux_div(to_dev(torch, T, torch.float64), to_dev(torch, b, torch.float64)).cpu().numpy()
    assert rel_l1(out, ref) <= 1e-12
    assert np.abs(out - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("name", CASES)
def test_flux_div_mixed(torch_cuda, name):
    torch = torch_cuda
    n, h, ndim, p, T, b = make_case(name)
    print("flux_div mixed", name, n, flush=True)
    b32 = b.astype(np.float32)
    ref = oracle.flux_div(oracle_grid(n, h, ndim, p), T, b32.astype(np.float64))
    plan = run_plan(torch, n, h, ndim, p, "mixed")
    out = plan.flux_div(to_dev(torch, T, torch.float64), to_dev(torch, b32, torch.float32)).cpu().numpy()
    assert rel_l1(out, ref) <= 1e-4


def superstep_pair(torch, name, precision, steps, ratio, variant=-1):
    n, h, ndim, p, T, b = make_case(name)
    g = oracle_grid(n, h, ndim, p)
    bg = b.astype(np.float32) if precision == "mixed" else b
    bo = bg.astype(np.float64)
    plan = run_plan(torch, n, h, ndim, p, precision, variant)
    Td = to_dev(torch, T, torch.float64)
    bd = to_dev(torch, bg, torch.float32 if precision == "mixed" else torch.float64)
    To = T.copy()
    for _ in range(steps):
        dt = ratio * oracle.dt_par(g, To)
        To, s_ref, _ = oracle.superstep(g, To, bo, dt)
        s = plan.superstep(Td, bd, dt)
        assert s == s_ref
    return Td.cpu().numpy(), To, T


@pytest.mark.parametrize("name,steps,ratio", [
    ("gauss2d", 5, 50.0), ("tangled_mc", 2, inputs.midpoint_ratio(16)),
    ("tangled_mc_sat", 2, inputs.midpoint_ratio(9)), ("iso1d", 3, 20.0),
    ("flat2d_ragged", 2, 30.0), ("tiny3d", 2, inputs.midpoint_ratio(5)),
])
def test_superstep_fp64(torch_cuda, name, steps, ratio):
    print("superstep fp64", name, steps, ratio, flush=True)
    g, o, T0 = superstep_pair(torch_cuda, name, "fp64", steps, ratio)
    assert rel_l1(g, o) <= 1e-12
    # the change over the step is matched too, not only the background
    assert rel_l1(g - T0, o - T0) <= 1e-10


@pytest.mark.parametrize("name,steps,ratio", [
    ("tangled_mc", 2, inputs.midpoint_ratio(16)), ("tangled_mc_sat", 2, inputs.midpoint_ratio(24)),
    ("gauss2d", 5, 50.0), ("flat2d_ragged", 2, 30.0),
])
def test_superstep_mixed(torch_cuda, name, steps, ratio):
    print("superstep mixed", name, steps, ratio, flush=True)
    g, o, T0 = superstep_pair(torch_cuda, name, "mixed", steps, ratio)
    err = rel_l1(g, o)
    print("  rel-L1 %.3e  Linf %.3e" % (err, np.abs(g - o).max()))
    assert err <= 1e-5


@pytest.mark.parametrize("variant", range(8))
def test_superstep_every_variant(torch_cuda, variant):
    print("variant", variant, flush=True)
    g, o, _ = superstep_pair(torch_cuda, "tangled_mc_sat", "fp64", 1, inputs.midpoint_ratio(6), variant)
    assert rel_l1(g, o) <= 1e-12


def test_every_variant_gives_the_same_bits(torch_cuda):
    """Each variant computes every face once, with the same operations in the
    same order (no automatic contraction), so the tile shape chosen by the
    autotuner never changes the result."""
    ref, _, _ = superstep_pair(torch_cuda, "tangled_mc_sat", "fp64", 1, inputs.midpoint_ratio(6), 0)
    for v in range(1, 8):
        g, _, _ = superstep_pair(torch_cuda, "tangled_mc_sat", "fp64", 1, inputs.midpoint_ratio(6), v)
        assert np.array_equal(g, ref), v


def test_superstep_is_deterministic(torch_cuda):
    torch = torch_cuda
    n, h, ndim, p, T, b = make_case("tangled_mc")
    plan = run_plan(torch, n, h, ndim, p, "fp64")
    outs = []
    for _ in range(2):
        Td = to_dev(torch, T, torch.float64)
        plan.superstep(Td, to_dev(torch, b, torch.float64), 1e-3)
        outs.append(Td.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_superstep_conserves_energy_on_gpu(torch_cuda):
    torch = torch_cuda
    n, h, ndim, p, T, b = make_case("tangled_mc_sat")
    plan = run_plan(torch, n, h, ndim, p, "fp64")
    Td = to_dev(torch, T, torch.float64)
    bd = to_dev(torch, b, torch.float64)
    e0 = T.sum()
    for _ in range(3):
        s = plan.superstep(Td, bd, 40 * plan.dt_par(Td))
    assert abs(Td.sum().item() - e0) <= 1e-13 * e0 * 3 * s


def test_dt_par_and_stage_count_match_oracle(torch_cuda):
    torch = torch_cuda
    for name in CASES:
        n, h, ndim, p, T, b = make_case(name)
        plan = run_plan(torch, n, h, ndim, p, "fp64")
        Td = to_dev(torch, T, torch.float64)
        assert plan.dt_par(Td) == oracle.dt_par(oracle_grid(n, h, ndim, p), T)


def test_flags_and_errors(torch_cuda):
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n, h, ndim, p, T, b = make_case("tiny3d")
    plan = rkl.Plan([lib_desc(n, h, ndim, p)], smax=8)
    Td = to_dev(torch, T, torch.float64)
    bd = to_dev(torch, b, torch.float64)
    # stage count above smax: error, T untouched
    with pytest.raises(rkl.RklError) as e:
        plan.superstep(Td, bd, 1000 * plan.dt_par(Td))
    assert e.value.status == rkl.RKL_ESTAGES
    assert np.array_equal(Td.cpu().numpy(), T)
    s, dtp, fl = plan.query()
    assert fl & rkl.RKL_FLAG_STAGES
    # a tiny super-step still takes the minimum two stages
    assert plan.superstep(Td, bd, 1e-12) == 2
    # non-positive and non-finite temperatures are flagged
    T2 = T.copy()
    T2[0, 0, 0] = -1.0
    plan.superstep(to_dev(torch, T2, torch.float64), bd, 1e-6)
    assert plan.query()[2] & rkl.RKL_FLAG_NONPOS
    T2[0, 0, 0] = np.nan
    plan.flux_div(to_dev(torch, T2, torch.float64), bd)
    assert plan.query()[2] & rkl.RKL_FLAG_NONFINITE
    with pytest.raises(ValueError):
        plan.superstep(Td[:-1].clone(), bd, 1e-6)
    with pytest.raises(TypeError):
        plan.superstep(Td.float(), bd, 1e-6)
    with pytest.raises(rkl.RklError):
        plan.superstep(Td, bd, float("nan"))
    # aliased fields are refused before any launch
    stream = rkl.ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    tp, bp = rkl.ctypes.c_void_p(Td.data_ptr()), rkl.ctypes.c_void_p(bd.data_ptr())
    before = Td.cpu().numpy()
    for call in (lambda: rkl.rkl_superstep(plan.handle, 0, tp, tp, 1e-6, stream),
                 lambda: rkl.rkl_subcycle(plan.handle, 0, tp, tp, 1e-6, 100, stream),
                 lambda: rkl.rkl_aag(plan.handle, 0, tp, tp, 1e-6, 0.01, 100, stream),
                 lambda: rkl.rkl_flux_div(plan.handle, 0, tp, bp, bp, stream),
                 lambda: rkl.rkl_flux_div(plan.handle, 0, tp, bp, tp, stream)):
        with pytest.raises(rkl.RklError) as e:
            call()
        assert e.value.status == rkl.RKL_EINVAL
    assert np.array_equal(Td.cpu().numpy(), before)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_spitzer_256_sampled_full_size(torch_cuda, precision, tol):
    """256^3 tangled field, kappa = T^2.5, kappa_perp = 1e-3, MC, s = 16: one
    full-size super-step on the GPU against the oracle at sampled cells,
    with every variant the plan can use (bench.py's autotuned pick among
    them), all giving the same bits."""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    w = inputs.spitzer_256()
    g = oracle_grid(w.n, w.h, 3, w.params)
    dt = w.ratio * oracle.dt_par(g, w.T)
    bg = w.b.astype(np.float32) if precision == "mixed" else w.b
    plan = run_plan(torch, w.n, w.h, 3, w.params, precision)
    bd = to_dev(torch, bg, torch.float32 if precision == "mixed" else torch.float64)
    rng = np.random.default_rng(5)
    centers = [tuple(int(v) for v in rng.integers(0, 256, 3)) for _ in range(6)] + [(0, 0, 0), (255, 255, 255)]
    ref = sampled_superstep(w.T, bg.astype(np.float64), w.params, w.h, 16, dt, centers)
    T0 = w.T[tuple(np.array(centers).T)]
    first = None
    for v in range(rkl.rkl_variant_count()):
        if rkl.rkl_variant_info(v)[3] >= 2 and precision != "mixed":
            continue
        plan.set_variant(v)
        Td = to_dev(torch, w.T, torch.float64)
        s = plan.superstep(Td, bd, dt)
        assert s == oracle.stages(w.ratio) == 16
        got = Td.cpu().numpy()[tuple(np.array(centers).T)]
        print("  %s variant %d: max |diff| %.3e, change rel-L1 %.3e"
              % (precision, v, np.abs(got - ref).max(), rel_l1(got - T0, ref - T0)), flush=True)
        # mixed: T ~ 1, FP32 flux arithmetic on temperatures offset to their
        # mean leaves ~1e-7 at the worst cell of the whole field (1.8e-7
        # measured there), so 1e-6 absolute and 1e-5 of the change
        assert np.abs(got - ref).max() <= (4e-12 if precision == "fp64" else 1e-6), v
        assert rel_l1(got - T0, ref - T0) <= (1e-9 if precision == "fp64" else 1e-5), v
        if first is None:
            first = Td
        else:
            assert torch.equal(first, Td), v
    plan.close()


def _window_t(torch, t, center, r):
    """periodic window of half-width r of a [n2][n1][n0] (or (3, ...)) torch
    tensor, copied to the host as float64"""
    lead = t.dim() - 3
    a = t
    for ax, c in enumerate(center):
        idx = torch.arange(c - r, c + r + 1, device=t.device) % t.shape[lead + ax]
        a = a.index_select(lead + ax, idx)
    return a.double().cpu().numpy()


@pytest.mark.parametrize("precision,variants", [("mixed", (0, 1)), ("fp64", (1,))])
def test_saturated_512_sampled_full_size(torch_cuda, precision, variants):
    """512^3 tangled field, kappa = T^2.5, kappa_perp = 1e-3, MC, saturation,
    s = 24: one full-size super-step with the one-stage variants bench.py
    times (32x8 tiles, z-chunks 32 and 64) against the oracle at sampled
    cells (periodic windows of half-width s+1, which hold the centre cell's
    whole dependency cone).  Mixed: max |diff| <= 1e-6 (T ~ 1; FP32 flux
    arithmetic on offset temperatures leaves ~1e-7 at the worst cell) and
    rel-L1 of the change <= 1e-5; FP64: rounding level, max |diff| <=
    1e-12 |T|."""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    w = inputs.saturated_512(fields=False)
    T0 = inputs.noisy_temperature(w.n, 2, device="cuda:0")
    b = inputs.tangled_b(w.n, 1, device="cuda:0")
    b = b.float() if precision == "mixed" else b.double()
    plan = rkl.Plan([lib_desc(w.n, w.h, 3, w.params)], precision=precision)
    dt = w.ratio * plan.dt_par(T0)
    s_target = 24
    rng = np.random.default_rng(13)
    centers = [tuple(int(v) for v in rng.integers(0, 512, 3)) for _ in range(3)] + [(0, 511, 0), (511, 0, 511)]
    r = s_target + 1
    ref = []
    for c in centers:
        win = oracle.Grid(n=(2 * r + 1,) * 3, h=tuple(w.h), ndim=3, **w.params)
        ref.append(oracle.rkl2_fixed(win, _window_t(torch, T0, c, r), _window_t(torch, b, c, r), s_target, dt)[r, r, r])
    ref = np.array(ref)
    idx = tuple(torch.tensor(np.array(centers).T, device="cuda:0"))
    t0 = T0[idx].cpu().numpy()
    for v in variants:
        plan.set_variant(v)
        T = T0.clone()
        assert plan.superstep(T, b, dt) == s_target
        got = T[idx].cpu().numpy()
        print("  %s variant %d: max |diff| %.3e" % (precision, v, np.abs(got - ref).max()), flush=True)
        if precision == "mixed":
            assert np.abs(got - ref).max() <= 1e-6
            assert rel_l1(got - t0, ref - t0) <= 1e-5
        else:
            assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
            assert rel_l1(got - t0, ref - t0) <= 1e-9
        del T
    plan.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_current_sheets(torch_cuda, precision, tol):
    """b flips sign between random neighbouring cells (b_L + b_R = 0 on
    many faces: the face direction vanishes and only kappa_perp conducts
    there), 3D, Spitzer + MC + saturation, against the oracle"""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    n = (33, 21, 18)
    h = (0.03, 0.04, 0.05)
    rng = np.random.default_rng(41)
    u = inputs.unit_vectors(rng.standard_normal((3, 1, 1, 1)) * np.ones((3,) + (n[2], n[1], n[0])))
    b = u * np.where(rng.random((n[2], n[1], n[0])) < 0.5, 1.0, -1.0)[None]
    T = inputs.noisy_temperature(n, 9, kmax=5)
    p = dict(inputs.SPITZER_MC_SAT, phi=0.01, kperp_ratio=0.05)
    bg = b.astype(np.float32) if precision == "mixed" else b
    g = oracle_grid(n, h, 3, p)
    plan = rkl.Plan([lib_desc(n, h, 3, p)], precision=precision)
    bd = to_dev(torch, bg, torch.float32 if precision == "mixed" else torch.float64)
    out = plan.flux_div(to_dev(torch, T, torch.float64), bd).cpu().numpy()
    ref = oracle.flux_div(g, T, bg.astype(np.float64))
    assert rel_l1(out, ref) <= tol
    dt = inputs.midpoint_ratio(8) * oracle.dt_par(g, T)
    Td = to_dev(torch, T, torch.float64)
    s = plan.superstep(Td, bd, dt)
    To, s_ref, _ = oracle.superstep(g, T, bg.astype(np.float64), dt)
    plan.close()
    assert s == s_ref == 8
    assert rel_l1(Td.cpu().numpy(), To) <= tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_degenerate_inputs(torch_cuda, precision):
    """no conduction (kappa0 = 0: dt_par is infinite, s = 2), a uniform
    temperature (every gradient zero), single-cell grids in 1, 2 and 3
    dimensions, and dt_hyp = 0: stage counts and results as the oracle's,
    the flux divergence exactly zero where no heat can flow"""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    tol = 1e-12 if precision == "fp64" else 1e-5
    bt = torch.float32 if precision == "mixed" else torch.float64
    rng = np.random.default_rng(43)
    cases = []
    n = (20, 12, 9)
    b = inputs.unit_vectors(rng.standard_normal((3, 9, 12, 20)))
    cases.append(("kappa0=0", n, 3, dict(inputs.SPITZER_MC_SAT, kappa0=0.0), 1.0 + rng.random((9, 12, 20)), b, 1e-3, True))
    cases.append(("uniform T", n, 3, dict(inputs.SPITZER_MC_SAT), np.full((9, 12, 20), 1.7), b, 1e-4, True))
    for nd, nn in ((1, (1, 1, 1)), (2, (1, 1, 1)), (3, (1, 1, 1))):
        cases.append(("one cell %dD" % nd, nn, nd, dict(inputs.SPITZER_MC_SAT), np.full((1, 1, 1), 1.3),
                      inputs.unit_vectors(rng.standard_normal((3, 1, 1, 1))), 1e-3, True))
    cases.append(("dt_hyp=0", n, 3, dict(inputs.SPITZER_MC), 1.0 + rng.random((9, 12, 20)), b, 0.0, False))
    for name, n, nd, p, T, b, dt, zero_div in cases:
        h = (0.1, 0.2, 0.3)
        bg = b.astype(np.float32) if precision == "mixed" else b
        g = oracle_grid(n, h, nd, p)
        plan = rkl.Plan([lib_desc(n, h, nd, p)], precision=precision)
        bd = to_dev(torch, bg, bt)
        div = plan.flux_div(to_dev(torch, T, torch.float64), bd).cpu().numpy()
        if zero_div:
            assert np.all(div == 0.0), name
        Td = to_dev(torch, T, torch.float64)
        s = plan.superstep(Td, bd, dt)
        To, s_ref, _ = oracle.superstep(g, T, bg.astype(np.float64), dt)
        plan.close()
        print("%-10s s=%d rel-L1 %.2e" % (name, s, rel_l1(Td.cpu().numpy(), To)), flush=True)
        assert s == s_ref == 2, name
        assert rel_l1(Td.cpu().numpy(), To) <= tol, name
        assert np.abs(Td.cpu().numpy() - T).max() <= 1e-14 * np.abs(T).max(), name


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_kernel_symmetries(torch_cuda, precision, tol):
    """The library against itself: x and z faces run different code (LDS
    exchange vs the register-carried z face), so exchanging axes x and z, or
    reflecting y, must transform the flux divergence and the super-step
    accordingly (up to the order of the three direction sums)."""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    from test_oracle_symmetry import reflect, swap
    n, h = (37, 23, 29), (0.03, 0.04, 0.05)
    p = dict(inputs.SPITZER_MC_SAT, phi=0.01, kperp_ratio=0.05)
    T = inputs.noisy_temperature(n, 12, amp=0.3, kmax=4)
    b = inputs.tangled_b(n, 13, kmax=4)
    bt = torch.float32 if precision == "mixed" else torch.float64
    if precision == "mixed":
        b = b.astype(np.float32).astype(np.float64)

    def run(n_, h_, T_, b_, dt=None):
        plan = rkl.Plan([lib_desc(n_, h_, 3, p)], precision=precision)
        Td = to_dev(torch, T_, torch.float64)
        bd = to_dev(torch, b_, bt)
        div = plan.flux_div(Td, bd).cpu().numpy()
        s = plan.superstep(Td, bd, dt) if dt else 0
        out = Td.cpu().numpy()
        plan.close()
        return div, out, s

    dt = inputs.midpoint_ratio(9) * oracle.dt_par(oracle_grid(n, h, 3, p), T)
    div0, out0, s0 = run(n, h, T, b, dt)
    T2, b2, h2, n2, perm = swap(T, b, h, n, 0, 2)
    div1, out1, s1 = run(n2, h2, T2, b2, dt)
    T3, b3 = reflect(T, b, 1)
    div2, out2, s2 = run(n, h, T3, b3, dt)
    assert s0 == s1 == s2 == 9
    scale, chg = np.abs(div0).max(), np.abs(out0 - T).max()
    gaps = [np.abs(np.transpose(div1, perm) - div0).max() / scale,
            np.abs(np.flip(div2, axis=1) - div0).max() / scale,
            np.abs(np.transpose(out1, perm) - out0).max() / chg,
            np.abs(np.flip(out2, axis=1) - out0).max() / chg]
    print(precision, "relative gaps (div x<->z, div y-mirror, step x<->z, step y-mirror):",
          " ".join("%.1e" % v for v in gaps))
    # mixed: the three FP32 direction sums are added in another order
    assert max(gaps) <= tol


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_full_size_conserves_energy(torch_cuda, precision, bar):
    """256^3 periodic workload, two super-steps: every face flux enters its
    two cells with opposite signs, so the sum of T is conserved up to
    rounding -- |sum dT| / sum |dT| within the bar (FP64: rounding of the
    stage sums; mixed: FP32 face fluxes)"""
    torch = torch_cuda
    from paper_1702_05487_amd import rkl
    w = inputs.spitzer_256(fields=False)
    T0 = inputs.noisy_temperature(w.n, 2, device="cuda:0")
    b = inputs.tangled_b(w.n, 1, device="cuda:0")
    b = b.float() if precision == "mixed" else b.double()
    plan = rkl.Plan([lib_desc(w.n, w.h, 3, w.params)], precision=precision)
    T = T0.clone()
    dt = w.ratio * plan.dt_par(T)
    for _ in range(2):
        assert plan.superstep(T, b, dt) >= 15
    plan.close()
    d = (T - T0)
    drift = abs(float(d.sum())) / float(d.abs().sum())
    print("%s: sum |dT| %.3e, |sum dT| / sum |dT| %.3e" % (precision, float(d.abs().sum()), drift))
    assert drift <= bar
