"""Pins of the oracle's fixed (Dirichlet) ghost boundaries.  CPU only.

A fixed axis takes the temperatures beyond its edges from caller layers,
held over the super-step, as the Gaussian test of Sec. 4.1.1 takes its
edge values from the exact solution.  Pinned by:
  - the periodic image: ghost layers holding the periodic neighbours (and a
    field direction that does not vary along the axis, since b repeats the
    edge cell's) give the periodic flux divergence bit for bit, per axis;
  - a linear temperature with linear ghosts (edges and corners included) is
    a steady state of the constant-conductivity flux, for one, two and
    three fixed axes at once, where zero-gradient ghosts are not;
  - the layer of the lowest fixed axis is the one read at a position beyond
    several edges: entries the rule never reads change nothing;
  - the Gaussian of Sec. 4.1.1 off-centre with exact-solution ghosts at the
    super-step's midpoint converges at second order.
"""
import numpy as np
import pytest

import oracle


def image_layers(T, n, d):
    """ghost layers of axis d holding the periodic neighbours of the edges"""
    a, bb = [e for e in range(3) if e != d]
    lo = np.zeros(oracle.ghost_shape(n, d))
    hi = np.zeros_like(lo)
    for jb in range(-1, n[bb] + 1):
        for ja in range(-1, n[a] + 1):
            c = [0, 0, 0]
            c[a], c[bb] = ja % n[a], jb % n[bb]
            cl, ch = list(c), list(c)
            cl[d], ch[d] = n[d] - 1, 0
            lo[jb + 1, ja + 1] = T[cl[2], cl[1], cl[0]]
            hi[jb + 1, ja + 1] = T[ch[2], ch[1], ch[0]]
    return lo, hi


def unit_b_const_along(rng, n, d):
    b = rng.standard_normal((3, n[2], n[1], n[0]))
    sl = [slice(None)] * 4
    sl[3 - d] = slice(0, 1)
    b = np.broadcast_to(b[tuple(sl)], b.shape).copy()
    return b / np.sqrt((b ** 2).sum(0))


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("limiter,saturation", [(0, 0), (1, 1), (1, 2)])
def test_periodic_image(d, limiter, saturation):
    rng = np.random.default_rng(10 * d + limiter + 3 * saturation)
    n = (7, 6, 5)
    T = 1.0 + 0.3 * rng.random((n[2], n[1], n[0]))
    b = unit_b_const_along(rng, n, d)
    base = dict(n=n, h=(0.1, 0.12, 0.09), ndim=3, limiter=limiter, saturation=saturation, phi=0.01,
                kappa_exp=2.5, kperp_ratio=0.01)
    ref = oracle.flux_div(oracle.Grid(**base), T, b)
    bnd, gh = [0, 0, 0], [None, None, None]
    bnd[d], gh[d] = 2, image_layers(T, n, d)
    out = oracle.flux_div(oracle.Grid(**base, boundary=tuple(bnd), ghosts=tuple(gh)), T, b)
    assert np.array_equal(out, ref)
    # and the layers matter: one changed ghost value changes the edge cells
    lo = gh[d][0].copy()
    lo[2, 2] += 0.1
    gh[d] = (lo, gh[d][1])
    out2 = oracle.flux_div(oracle.Grid(**base, boundary=tuple(bnd), ghosts=tuple(gh)), T, b)
    assert not np.array_equal(out2, ref)


def test_periodic_image_1d_2d():
    rng = np.random.default_rng(5)
    for n, ndim in (((12, 1, 1), 1), ((9, 8, 1), 2)):
        T = 1.0 + 0.3 * rng.random((n[2], n[1], n[0]))
        b = unit_b_const_along(rng, n, 0)
        base = dict(n=n, h=(0.1, 0.12, 1.0), ndim=ndim, limiter=1, saturation=1, phi=0.02, kappa_exp=2.5,
                    kperp_ratio=0.05)
        ref = oracle.flux_div(oracle.Grid(**base), T, b)
        g = oracle.Grid(**base, boundary=(2, 0, 0), ghosts=(image_layers(T, n, 0), None, None))
        assert np.array_equal(oracle.flux_div(g, T, b), ref)


def linear_layers(f, n, d):
    """ghost layers of axis d from the function f(i, j, k) of cell indices"""
    a, bb = [e for e in range(3) if e != d]
    out = []
    for pos in (-1, n[d]):
        L = np.zeros(oracle.ghost_shape(n, d))
        for jb in range(-1, n[bb] + 1):
            for ja in range(-1, n[a] + 1):
                c = [0, 0, 0]
                c[d], c[a], c[bb] = pos, ja, jb
                L[jb + 1, ja + 1] = f(*c)
        out.append(L)
    return tuple(out)


@pytest.mark.parametrize("fixed", [(2, 0, 0), (0, 2, 0), (0, 0, 2), (2, 2, 0), (2, 0, 2), (0, 2, 2), (2, 2, 2)])
@pytest.mark.parametrize("limiter", [0, 1])
def test_linear_steady_state(fixed, limiter):
    """T = 1 + g.r with linear ghosts: the face gradient is g everywhere, so
    every face flux is the same and the divergence vanishes (to rounding);
    non-fixed axes are outflow where fixed would be needed for the steady
    state, so they get g = 0 along them."""
    n, h = (6, 5, 4), (0.1, 0.15, 0.2)
    grad = [0.7 if fixed[e] == 2 else 0.0 for e in range(3)]
    grad = [grad[0], -0.4 * (fixed[1] == 2), 0.3 * (fixed[2] == 2)]

    def f(i, j, k):
        return 1.0 + grad[0] * (i + 0.5) * h[0] + grad[1] * (j + 0.5) * h[1] + grad[2] * (k + 0.5) * h[2]

    kk, jj, ii = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    T = f(ii, jj, kk).astype(np.float64)
    b = np.zeros((3,) + T.shape)
    bdir = np.array([0.6, -0.48, 0.64])
    for e in range(3):
        b[e] = bdir[e]
    bnd = tuple(2 if fixed[e] == 2 else 1 for e in range(3))
    gh = tuple(linear_layers(f, n, e) if fixed[e] == 2 else None for e in range(3))
    base = dict(n=n, h=h, ndim=3, limiter=limiter, kappa0=1.3, kperp_ratio=0.2)
    out = oracle.flux_div(oracle.Grid(**base, boundary=bnd, ghosts=gh), T, b)
    assert np.abs(out).max() <= 1e-11
    # zero-gradient ghosts on the same axes are not a steady state
    zg = oracle.flux_div(oracle.Grid(**base, boundary=(1, 1, 1)), T, b)
    assert np.abs(zg).max() > 1e-2
    # a super-step keeps the steady state
    T1, s, _ = oracle.superstep(oracle.Grid(**base, boundary=bnd, ghosts=gh), T, b,
                                20 * oracle.dt_par(oracle.Grid(**base, boundary=bnd, ghosts=gh), T))
    assert s > 2 and np.abs(T1 - T).max() <= 1e-12


def test_lowest_fixed_axis_layer_is_read():
    """x and y fixed: a position beyond both an x and a y edge reads the x
    layer (at its y extension).  The y layer's x-extension entries are never
    read; the x layer's y-extension entries are, at the cells next to the
    tile corners."""
    rng = np.random.default_rng(8)
    n = (5, 4, 3)
    T = 1.0 + 0.3 * rng.random((n[2], n[1], n[0]))
    b = rng.standard_normal((3,) + T.shape)
    b /= np.sqrt((b ** 2).sum(0))
    gx = tuple(1.0 + 0.3 * rng.random(oracle.ghost_shape(n, 0)) for _ in range(2))
    gy = tuple(1.0 + 0.3 * rng.random(oracle.ghost_shape(n, 1)) for _ in range(2))
    base = dict(n=n, h=(0.1, 0.1, 0.1), ndim=3, limiter=1, saturation=1, phi=0.01, kappa_exp=2.5,
                kperp_ratio=0.01, boundary=(2, 2, 0))
    ref = oracle.flux_div(oracle.Grid(**base, ghosts=(gx, gy, None)), T, b)
    gy2 = tuple(L.copy() for L in gy)
    for L in gy2:
        L[:, 0] += 5.0          # x = -1 column of the y layers
        L[:, -1] += 5.0         # x = n0 column
    assert np.array_equal(oracle.flux_div(oracle.Grid(**base, ghosts=(gx, gy2, None)), T, b), ref)
    gx2 = tuple(L.copy() for L in gx)
    gx2[0][:, 0] += 0.5         # y = -1 row of the low x layer
    out = oracle.flux_div(oracle.Grid(**base, ghosts=(gx2, gy, None)), T, b)
    changed = np.argwhere(out != ref)
    assert len(changed) > 0
    assert set(changed[:, 2]) == {0} and set(changed[:, 1]) <= {0, 1}   # cells (0, 0..1, k) only


def gaussian_run(N, t_end, dx0, sigma=0.4, x0=0.6, L=4.0, when=0.5):
    """Sec. 4.1.1's Gaussian (kappa = 1 on [-2, 2]) shifted to x0, ghosts
    from the exact solution at t_n + when * dt of each super-step"""
    dx = L / N
    x = -L / 2 + (np.arange(N) + 0.5) * dx

    def exact(xx, t):
        var = sigma ** 2 + 2 * t
        return sigma / np.sqrt(var) * np.exp(-(xx - x0) ** 2 / (2 * var))

    b = np.zeros((3, 1, 1, N))
    b[0] = 1.0
    T = exact(x, 0.0)[None, None]
    nsteps = int(np.ceil(t_end / (0.45 * dx0 * dx) - 1e-12))
    dt = t_end / nsteps
    for m in range(nsteps):
        t = (m + when) * dt
        lo = np.full(oracle.ghost_shape((N, 1, 1), 0), exact(-L / 2 - dx / 2, t))
        hi = np.full(oracle.ghost_shape((N, 1, 1), 0), exact(L / 2 + dx / 2, t))
        g = oracle.Grid(n=(N, 1, 1), h=(dx, 1.0, 1.0), ndim=1, kappa0=1.0, boundary=(2, 0, 0), ghosts=((lo, hi), None, None))
        T, s, _ = oracle.superstep(g, T, b, dt)
    return np.mean(np.abs(T[0, 0] - exact(x, t_end)))


def test_gaussian_exact_ghosts_second_order():
    """the edge values carry the solution in and out (the off-centre pulse
    reaches the right edge at ~5 % of its peak): L1 error four-fold smaller
    per doubling with midpoint ghosts; ghosts frozen at the super-step's
    start lag by O(dt) = O(dx) here (dt/dx fixed) and lose the order"""
    t_end, dx0 = 0.08, 4.0 / 64
    mid = [gaussian_run(N, t_end, dx0) for N in (64, 128, 256, 512)]
    ratios = np.array(mid[:-1]) / np.array(mid[1:])
    assert np.all(ratios > 3.5) and np.all(ratios < 4.6), (mid, ratios)
    start = [gaussian_run(N, t_end, dx0, when=0.0) for N in (256, 512)]
    assert start[0] / start[1] < 3.0 and start[1] > 1.5 * mid[-1], (start, mid)
