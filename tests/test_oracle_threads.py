"""The oracle's cell loops on several threads give the same bits as the
serial run (each cell's value is computed on its own from inputs the loop
does not write), for periodic and outflow grids, both limiters and both
saturation forms."""
import numpy as np
import pytest

import oracle
from paper_1702_05487_amd import inputs


@pytest.mark.parametrize("params,bc", [
    (inputs.SPITZER_MC_SAT, (0, 0, 0)),
    (dict(inputs.SPITZER_MC, saturation=2), (1, 0, 1)),
    (dict(inputs.BASE, kappa_exp=2.5, kperp_ratio=0.1), (0, 1, 0)),
])
def test_threads_give_the_serial_bits(params, bc):
    n = (23, 19, 13)
    T = inputs.noisy_temperature(n, 4, kmax=4)
    b = inputs.tangled_b(n, 5, kmax=4)
    g = oracle.Grid(n=n, h=(0.04, 0.05, 0.07), ndim=3, **dict(params, boundary=bc))
    dt = inputs.midpoint_ratio(7) * oracle.dt_par(g, T)
    try:
        assert oracle.set_threads(1) == 1
        ref, s_ref, _ = oracle.superstep(g, T, b, dt)
        div_ref = oracle.flux_div(g, T, b)
        assert oracle.set_threads(4) == 4
        got, s, _ = oracle.superstep(g, T, b, dt)
        div = oracle.flux_div(g, T, b)
    finally:
        oracle.set_threads(1)
    assert s == s_ref == 7
    assert np.array_equal(got, ref)
    assert np.array_equal(div, div_ref)
