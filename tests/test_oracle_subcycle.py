"""Pins of the oracle's explicit sub-cycling (the conduction operator applied
N_sub = ceil(dt_hyp/dt_par) times with forward-Euler steps of dt_hyp/N_sub):
the exact amplification (1 + tau lambda)^N of a Fourier mode, the sub-step
count rule and its degenerate cases, conservation, and first-order
convergence to a fine-step reference.  CPU only."""
import numpy as np
import pytest

import oracle
from paper_1702_05487_amd import inputs
from test_oracle_convergence import rk4
from test_oracle_operator import CASES, cell_coords, fourier_symbol, uniform_b


@pytest.mark.parametrize("case", CASES[:4])
@pytest.mark.parametrize("ratio", [0.7, 3.4, 17.2])
def test_fourier_mode_amplification(case, ratio):
    n, h, ndim, bv, kr, m = case
    g = oracle.Grid(n=n, h=h, ndim=ndim, kappa0=0.9, kappa_exp=0.0, kperp_ratio=kr, gamma=2.0, rho=1.0)
    i0, i1, i2 = cell_coords(n)
    theta = [2 * np.pi * m[d] / n[d] for d in range(3)]
    phase = theta[0] * i0 + theta[1] * i1 + theta[2] * i2
    lam = fourier_symbol(g, bv, theta)
    T = 3.0 + 0.5 * np.cos(phase)
    # dt_par for constant kappa: cp / ((gamma-1)/rho kappa0 sum_d h_d^-2)
    dtp = 0.5 / (1.0 * 0.9 * sum(1.0 / h[d] ** 2 for d in range(ndim)))
    dt_hyp = ratio * dtp
    Y, nsub = oracle.subcycle(g, T, uniform_b(n, bv), dt_hyp)
    assert nsub == int(np.ceil(ratio - 1e-12))
    tau = dt_hyp / nsub
    assert tau <= dtp * (1 + 1e-14)
    amp = (1.0 + tau * lam) ** nsub
    np.testing.assert_allclose(Y, 3.0 + 0.5 * amp * np.cos(phase), rtol=0, atol=1e-13 * nsub)


def test_substep_count_and_degenerate_cases():
    n = (6, 5, 4)
    g = oracle.Grid(n=n, h=(0.1, 0.1, 0.1), ndim=3, kappa0=1.0, kappa_exp=2.5, kperp_ratio=0.01, limiter=1)
    T = inputs.noisy_temperature(n, 3, kmax=2)
    b = inputs.tangled_b(n, 4, kmax=2)
    dtp = oracle.dt_par(g, T)
    for r in (0.3, 1.5, 9.9):
        _, nsub = oracle.subcycle(g, T, b, r * dtp)
        assert nsub == int(np.ceil(r))
    Y, nsub = oracle.subcycle(g, T, b, 0.0)
    assert nsub == 0 and np.array_equal(Y, T)
    g0 = oracle.Grid(n=n, h=(0.1, 0.1, 0.1), ndim=3, kappa0=0.0)
    Y, nsub = oracle.subcycle(g0, T, b, 1.0)
    assert nsub == 0 and np.array_equal(Y, T)
    _, nsub = oracle.subcycle(g, T, b, 50 * dtp, max_sub=10)
    assert nsub == -1


@pytest.mark.parametrize("sat", [0, 1])
def test_subcycling_conserves_energy(sat):
    n = (10, 9, 8)
    g = oracle.Grid(n=n, h=(0.1,) * 3, ndim=3, kappa0=1.0, kappa_exp=2.5, kperp_ratio=1e-3, limiter=1,
                    saturation=sat, phi=0.05)
    T = inputs.noisy_temperature(n, 5, kmax=2)
    b = inputs.tangled_b(n, 6, kmax=2)
    Y, nsub = oracle.subcycle(g, T, b, 12.3 * oracle.dt_par(g, T))
    assert nsub == 13
    assert abs(Y.sum() - T.sum()) <= 1e-13 * T.sum() * nsub


def test_first_order_against_fine_rk4():
    """kappa = T^2.5, MC limiter on an 8^3 tangled field: halving the
    Courant number (so doubling the sub-steps) halves the error against a
    brute-force RK4 reference."""
    n = (8, 8, 8)
    b = inputs.tangled_b(n, 11, kmax=2)
    T0 = inputs.noisy_temperature(n, 12, kmax=2)
    g = oracle.Grid(n=n, h=(1 / 8,) * 3, ndim=3, kappa0=1.0, kappa_exp=2.5, kperp_ratio=1e-3, limiter=1)
    t_end = 20 * oracle.dt_par(g, T0)
    ref = rk4(g, T0, b, t_end, 2000)
    errs = []
    for cp in (0.5, 0.25, 0.125):
        gc = oracle.Grid(n=n, h=(1 / 8,) * 3, ndim=3, kappa0=1.0, kappa_exp=2.5, kperp_ratio=1e-3, limiter=1,
                         cp=cp)
        Y, _ = oracle.subcycle(gc, T0, b, t_end)
        errs.append(np.abs(Y - ref).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all((ratios > 1.7) & (ratios < 2.3)), (errs, ratios)
