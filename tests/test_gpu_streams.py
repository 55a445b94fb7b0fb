"""Every entry point on a caller's non-default stream (created right after
the plan, torch's default priority): the same bits as on the default
stream -- plan set-up is complete when rkl_plan returns and every launch
and copy goes to the stream passed."""
import numpy as np
import pytest

from helpers import lib_desc
from paper_1702_05487_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1702_05487_amd import rkl
    rkl.load(build_if_missing=False)
    return torch


def run_all(torch, precision, side):
    """flux_div, dt_par, super-step, sub-cycling and AAG of one grid, and a
    batched graph super-step of three, on `side` (a stream) or the default
    stream (None); returns the host results"""
    from paper_1702_05487_amd import rkl
    n = (24, 18, 14)
    p = dict(inputs.SPITZER_MC_SAT, phi=0.05)
    bt = torch.float32 if precision == "mixed" else torch.float64
    T0 = torch.from_numpy(inputs.noisy_temperature(n, 5, kmax=4)).to("cuda:0")
    b = torch.from_numpy(inputs.tangled_b(n, 6, kmax=4)).to("cuda:0", dtype=bt)
    ps = inputs.patch_set(3, seed=12, lo=8, hi=20, smin=3, smax=9)
    Tb0 = torch.from_numpy(np.concatenate([t.ravel() for t in ps.T])).to("cuda:0")
    bb = torch.from_numpy(np.concatenate([x.ravel() for x in ps.b])).to("cuda:0", dtype=bt)
    torch.cuda.synchronize()
    out = {}
    ctx = torch.cuda.stream(side) if side is not None else torch.cuda.stream(torch.cuda.current_stream())
    with ctx:
        plan = rkl.Plan([lib_desc(n, (0.04, 0.05, 0.06), 3, p)], precision=precision)
        out["div"] = plan.flux_div(T0, b)
        dtp = plan.dt_par(T0)
        T = T0.clone()
        out["s"] = plan.superstep(T, b, inputs.midpoint_ratio(9) * dtp)
        out["T"] = T
        T = T0.clone()
        out["nsub"] = plan.subcycle(T, b, 5.5 * dtp)
        out["Tsub"] = T
        T = T0.clone()
        out["saag"] = plan.aag(T, b, 6.0 * dtp, 0.05)
        out["Taag"] = T
        plan.close()
        bplan = rkl.Plan([lib_desc(m, (1 / 64,) * 3, 3, ps.params) for m in ps.n], precision=precision, smax=16)
        off = bplan.offsets()
        dt = torch.tensor([ps.ratio[k] * bplan.dt_par(Tb0[off[k]:off[k + 1]], grid=k) for k in range(3)],
                          dtype=torch.float64, device="cuda:0")
        Tb = Tb0.clone()
        s_out = torch.zeros(3, dtype=torch.int32, device="cuda:0")
        bplan.graph_capture(Tb, bb, dt, s_out)
        bplan.graph_launch()
        bplan.graph_launch()
        out["Tb"], out["sb"] = Tb, s_out
        Te = Tb0.clone()
        bplan.superstep_batched(Te, bb, dt)
        out["Te"] = Te
    torch.cuda.synchronize()
    bplan.close()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_side_stream_gives_the_same_bits(torch_cuda, precision):
    torch = torch_cuda
    ref = run_all(torch, precision, None)
    side = torch.cuda.Stream()
    got = run_all(torch, precision, side)
    for k in ref:
        assert np.array_equal(np.asarray(ref[k]), np.asarray(got[k])), k
    assert ref["s"] == 9 and ref["nsub"] == 6


def test_two_plans_on_two_threads(torch_cuda):
    """two plans used at once from two host threads, each on its own
    stream (the library keeps no state outside a plan; rkl_last_error is per
    thread): the same bits as one after the other"""
    torch = torch_cuda
    from concurrent.futures import ThreadPoolExecutor
    from paper_1702_05487_amd import rkl

    def work(seed):
        n = (28, 20, 16)
        p = dict(inputs.SPITZER_MC_SAT, phi=0.05)
        T0 = torch.from_numpy(inputs.noisy_temperature(n, seed, kmax=4)).to("cuda:0")
        b = torch.from_numpy(inputs.tangled_b(n, seed + 1, kmax=4)).to("cuda:0")
        torch.cuda.synchronize()
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            plan = rkl.Plan([lib_desc(n, (0.04, 0.05, 0.06), 3, p)])
            T = T0.clone()
            dt = inputs.midpoint_ratio(11) * plan.dt_par(T)
            ss = [plan.superstep(T, b, dt) for _ in range(4)]
            side.synchronize()
            plan.close()
        return ss, T.cpu().numpy()

    seq = [work(s) for s in (21, 31)]
    with ThreadPoolExecutor(2) as ex:
        par = list(ex.map(work, (21, 31)))
    for (s1, t1), (s2, t2) in zip(seq, par):
        assert s1 == s2
        assert np.array_equal(t1, t2)
