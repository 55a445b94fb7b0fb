"""Pins of the oracle's RKL2 time integrator (coefficients, stage count,
amplification polynomial) against what the paper prints and what the
mathematics fixes.  CPU only."""
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import eval_legendre

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "rkl2_s3_worked_example.txt")


def _golden():
    rows = []
    for line in open(GOLD):
        line = line.split("#")[0].split()
        if line:
            rows.append((line[0], int(line[1]), [Fraction(v) for v in line[2:]]))
    return rows


def amplification(s, z):
    """R_s(z) measured through the oracle: a two-cell periodic 1D grid with
    constant kappa = 1 and h = 1 has the alternating mode with eigenvalue -4,
    so tau = -z/4 gives tau*lambda = z; the mode amplitude after one
    super-step is R_s(z)."""
    g = oracle.Grid(n=(2, 1, 1), h=(1.0, 1.0, 1.0), ndim=1, kappa0=1.0)
    b = np.zeros((3, 1, 1, 2))
    b[0] = 1.0
    T = np.array([[[2.0, 0.0]]])
    Y = oracle.rkl2_fixed(g, T, b, s, -z / 4.0)
    return 0.5 * (Y[0, 0, 0] - Y[0, 0, 1])


def legendre_form(s, z):
    """a_s + b_s P_s(1 + w1 z) with the closed forms of Appendix A."""
    bs = (s * s + s - 2.0) / (2.0 * s * (s + 1.0))
    w1 = 4.0 / (s * s + s - 2.0)
    return (1.0 - bs) + bs * eval_legendre(s, 1.0 + w1 * z)


def test_s3_coefficients_match_worked_example():
    w1, mu, nu, mut, gt = oracle.coeffs(3)
    table = {"mu": mu, "nu": nu, "mut": mut, "gt": gt}
    seen = 0
    for name, j, vals in _golden():
        if name == "w1":
            assert w1 == pytest.approx(float(vals[0]), rel=1e-15)
            seen += 1
        elif name in table:
            assert table[name][j] == pytest.approx(float(vals[0]), rel=1e-15, abs=1e-16), (name, j)
            seen += 1
        elif name == "y0w":
            assert 1.0 - mu[j] - nu[j] == pytest.approx(float(vals[0]), rel=1e-15)
            seen += 1
    assert seen == 11


def test_s3_stability_polynomial_matches_worked_example():
    rows = {(n, j): v for n, j, v in _golden()}
    poly = [float(c) for c in rows[("R", 3)]]
    for z in np.linspace(-5.0, 0.0, 21):
        want = sum(c * z ** k for k, c in enumerate(poly))
        assert amplification(3, z) == pytest.approx(want, abs=2e-14)
    # the Legendre form with the printed a_3, b_3 and w1 = 2/5
    a3, b3 = float(rows[("a", 3)][0]), float(rows[("b", 3)][0])
    for z in np.linspace(-5.0, 0.0, 11):
        assert amplification(3, z) == pytest.approx(a3 + b3 * eval_legendre(3, 1 + 0.4 * z), abs=2e-14)
    # stable range -5 <= z <= 0 and the end point
    zmin = float(rows[("zmin", 3)][0])
    zs = np.linspace(zmin, 0.0, 501)
    assert max(abs(amplification(3, z)) for z in zs[::10]) <= 1.0 + 1e-14
    # at z = -5 the Legendre argument is -1: R_3 = a_3 - b_3 = 1/6
    assert amplification(3, zmin) == pytest.approx(a3 - b3, abs=1e-14)
    # far outside the interval the polynomial grows without bound
    assert abs(amplification(3, 2 * zmin)) > 1.0


def test_two_stage_is_textbook_rk2():
    # s = 2: R_2(z) = 1 + z + z^2/2, the two-stage second-order RK polynomial
    for z in np.linspace(-2.0, 0.0, 9):
        assert amplification(2, z) == pytest.approx(1 + z + z * z / 2, abs=1e-14)


@pytest.mark.parametrize("s", [2, 3, 4, 5, 7, 10, 16, 24, 32, 40, 64])
def test_amplification_is_legendre_polynomial(s):
    w1 = 4.0 / (s * s + s - 2.0)
    zs = np.linspace(-2.0 / w1, 0.0, 37)
    got = np.array([amplification(s, z) for z in zs])
    want = legendre_form(s, zs)
    assert np.max(np.abs(got - want)) < 1e-12 * max(1, s)
    # |R_s| <= 1 over the whole stable interval (argument of P_s in [-1, 1])
    assert np.max(np.abs(got)) <= 1.0 + 1e-12


@pytest.mark.parametrize("s", [2, 3, 4, 5, 6, 8])
def test_second_order_taylor_match(s):
    # R_s(0) = R_s'(0) = R_s''(0) = 1: recover the polynomial's coefficients
    # exactly from s+1 samples and compare with 1, 1, 1/2
    zs = -np.cos(np.pi * (np.arange(s + 1) + 0.5) / (s + 1)) - 1.0   # in [-2, 0]
    vals = np.array([amplification(s, z) for z in zs])
    c = np.linalg.solve(np.vander(zs, s + 1, increasing=True), vals)
    assert c[0] == pytest.approx(1.0, abs=1e-11)
    assert c[1] == pytest.approx(1.0, abs=1e-10)
    assert c[2] == pytest.approx(0.5, abs=1e-9)
    if s >= 3:
        # not third order: the z^3 coefficient differs from 1/6
        assert abs(c[3] - 1.0 / 6.0) > 1e-3


def test_stage_count_rule():
    # r = dt_hyp/dt_par; root of r = (s^2+s-2)/4 rounded to 1 + floor(root)
    assert oracle.stages(0.0) == 2          # root 1 -> 2
    assert oracle.stages(1.0) == 3          # exact root 2 is bumped to 3
    assert oracle.stages(50.0) == 14        # root 13.72
    for s in range(2, 200):
        exact = (s * s + s - 2) / 4.0       # root exactly s
        assert oracle.stages(exact) == s + 1
        assert oracle.stages(exact * (1 - 1e-9)) == s
    # the effective parabolic Courant number dt_h/(2 dt_p) tends to s^2/8
    for s in (100, 1000, 10000):
        r = (s * s + s - 2) / 4.0 * 0.999999
        assert oracle.stages(r) == s
        assert (r / 2.0) / (s * s / 8.0) == pytest.approx(1.0, rel=2.0 / s)


def test_stage_count_stays_within_stability_bound():
    # with s from the rule, tau = r dt_par satisfies tau <= 2/(|lambda|max w1)
    # whenever dt_par |lambda|max <= 2 (the explicit limit)
    for r in np.concatenate([np.linspace(0, 5, 51), np.geomspace(5, 1e6, 200)]):
        s = oracle.stages(r)
        w1 = 4.0 / (s * s + s - 2.0)
        assert r * 2.0 * w1 <= 2.0 + 1e-12
