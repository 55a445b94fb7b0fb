"""Pins of the oracle's RKL1 super-step (first-order Legendre scheme): the
Legendre amplification P_s(1 + w1 tau lambda) of Fourier modes, s = 1 as
forward Euler, the stage-count rule, first-order convergence against the
matrix exponential, positivity and conservation.  CPU only."""
import numpy as np
import pytest
from scipy.linalg import expm
from scipy.special import eval_legendre

import oracle
from paper_1702_05487_amd import inputs
from test_oracle_operator import CASES, cell_coords, fourier_symbol, uniform_b


@pytest.mark.parametrize("case", CASES[:4])
@pytest.mark.parametrize("s", [1, 2, 5, 13, 30])
def test_fourier_mode_legendre_amplification(case, s):
    n, h, ndim, bv, kr, m = case
    g = oracle.Grid(n=n, h=h, ndim=ndim, kappa0=0.9, kappa_exp=0.0, kperp_ratio=kr, gamma=2.0, rho=1.0)
    i0, i1, i2 = cell_coords(n)
    theta = [2 * np.pi * m[d] / n[d] for d in range(3)]
    phase = theta[0] * i0 + theta[1] * i1 + theta[2] * i2
    lam = fourier_symbol(g, bv, theta)
    lam_max = max(abs(fourier_symbol(g, bv, [2 * np.pi * a / n[0], 2 * np.pi * c / n[1], 2 * np.pi * e / n[2]]))
                  for a in range(n[0]) for c in range(n[1]) for e in range(n[2]))
    w1 = 2.0 / (s * s + s)
    tau = 0.9 * 2.0 / (lam_max * w1)            # inside the stable interval of every mode
    T = 3.0 + 0.5 * np.cos(phase)
    Y = oracle.rkl1_fixed(g, T, uniform_b(n, bv), s, tau)
    R = eval_legendre(s, 1 + w1 * tau * lam)
    np.testing.assert_allclose(Y, 3.0 + 0.5 * R * np.cos(phase), rtol=0, atol=1e-14 * s * (1 + abs(tau * lam)))


def test_one_stage_is_forward_euler():
    n = (9, 7, 6)
    g = oracle.Grid(n=n, h=(0.1, 0.12, 0.09), ndim=3, kappa0=1.0, kappa_exp=2.5, kperp_ratio=0.05, limiter=1,
                    saturation=1, phi=0.05)
    T = inputs.noisy_temperature(n, 31, kmax=2)
    b = inputs.tangled_b(n, 32, kmax=2)
    tau = 0.8 * oracle.dt_par(g, T)
    np.testing.assert_allclose(oracle.rkl1_fixed(g, T, b, 1, tau), T + tau * oracle.flux_div(g, T, b),
                               rtol=0, atol=1e-15)


def test_stage_count_rule():
    # dt_hyp = dt_par (s^2 + s)/2; the root is rounded up as 1 + floor(root)
    for r, s in [(0.0, 1), (0.4, 1), (0.999, 1), (1.0, 2), (2.99, 2), (3.0, 3), (6.0, 4), (5.9, 3), (55.0, 11)]:
        assert oracle.stages_rkl1(r) == s, r
    for r in np.geomspace(1.3, 5e4, 40):
        s = oracle.stages_rkl1(r)
        assert (s * s + s) / 2.0 >= r              # tau = dt_hyp stays inside the stability bound
        assert ((s - 1) ** 2 + (s - 1)) / 2.0 <= r  # and s is the smallest such count
        assert abs(s - np.sqrt(2 * r)) < 1.5


def test_first_order_against_matrix_exponential():
    """Linear operator on a tiny 2D grid: halving the super-step at fixed end
    time halves the error of RKL1 (ratio -> 2), where RKL2 gains about 4."""
    n = (6, 5, 1)
    g = oracle.Grid(n=n, h=(0.2, 0.25, 1.0), ndim=2, kappa0=1.0, kperp_ratio=0.1, gamma=2.0)
    N = n[0] * n[1]
    b = np.zeros((3, 1, n[1], n[0]))
    b[:] = (np.array([0.6, 0.7, 0.4]) / np.linalg.norm([0.6, 0.7, 0.4]))[:, None, None, None]
    M = np.zeros((N, N))
    for i in range(N):
        e = np.zeros(N)
        e[i] = 1.0
        M[:, i] = oracle.flux_div(g, e.reshape(1, n[1], n[0]), b).ravel()
    T0 = np.random.default_rng(0).uniform(0.5, 1.5, N)
    lam_max = np.max(np.abs(np.linalg.eigvalsh(0.5 * (M + M.T))))
    t_end = 4.0 / lam_max
    exact = expm(t_end * M) @ T0
    errs = []
    for nsteps in (4, 8, 16, 32):
        T = T0.reshape(1, n[1], n[0])
        for _ in range(nsteps):
            T = oracle.rkl1_fixed(g, T, b, 8, t_end / nsteps)
        errs.append(np.abs(T.ravel() - exact).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all((ratios > 1.8) & (ratios < 2.3)), (errs, ratios)


def test_positive_through_a_large_super_step():
    """A narrow Gaussian pulse on a zero background plus 1e-6, s = 40 RKL1
    stages at the stability limit: the temperature stays positive (the
    Legendre polynomials are bounded by one on [-1, 1])."""
    n = (128, 1, 1)
    g = oracle.Grid(n=n, h=(1 / 128, 1.0, 1.0), ndim=1, kappa0=1.0, gamma=2.0)
    x = (np.arange(128) + 0.5) / 128
    T = (1e-6 + np.exp(-((x - 0.5) / 0.01) ** 2))[None, None]
    b = np.zeros((3, 1, 1, 128))
    b[0] = 1.0
    s = 40
    tau = (s * s + s) / 2.0 * oracle.dt_par(g, T)
    Y = oracle.rkl1_fixed(g, T, b, s, tau)
    assert Y.min() > 0.0
    assert abs(Y.sum() - T.sum()) <= 1e-13 * T.sum() * s


@pytest.mark.parametrize("sat", [0, 1])
def test_rkl1_superstep_conserves_energy(sat):
    n = (10, 9, 8)
    g = oracle.Grid(n=n, h=(0.1,) * 3, ndim=3, kappa0=1.0, kappa_exp=2.5, kperp_ratio=1e-3, limiter=1,
                    saturation=sat, phi=0.05)
    T = inputs.noisy_temperature(n, 5, kmax=2)
    b = inputs.tangled_b(n, 6, kmax=2)
    Y, s, _ = oracle.superstep_rkl1(g, T, b, 30.0 * oracle.dt_par(g, T))
    assert s == oracle.stages_rkl1(30.0) == 8
    assert abs(Y.sum() - T.sum()) <= 1e-13 * T.sum() * s
