"""Pins of the oracle's outflow boundaries (boundary[d] = 1: the cells beyond
an edge repeat the edge cell's T and b).  CPU only.

An outflow axis of N cells reads, beyond each edge, copies of the edge
cell.  A periodic axis of 2N cells holding the field and its mirror image
(T and b copied, not reflected) puts exactly those copies next to the
edges.  So one flux divergence on the outflow grid equals the first N cells
along each outflow axis of the flux divergence on the mirror-extended
periodic grid, up to rounding order -- for any conductivity law, limiter,
saturation form and field direction.  A whole super-step keeps that
equality when the mirrored problem stays mirror-symmetric from stage to
stage, i.e. when b has no component along an open axis or lies along a
single axis: then each stage's result beyond the edge is again the copy."""
import numpy as np
import pytest

import oracle
from paper_1702_05487_amd import inputs


def mirror(f, axes):
    """periodic mirror extension of a [n2][n1][n0] field (or (3, ...) vector
    field) along the given grid axes (0 = x)"""
    lead = f.ndim - 3
    for ax in axes:
        a = lead + 2 - ax
        f = np.concatenate([f, np.flip(f, axis=a)], axis=a)
    return np.ascontiguousarray(f)


def block(f, n):
    return f[..., :n[2], :n[1], :n[0]]


CASES = [
    # name, n, ndim, open axes, params
    ("1d_spitzer_sat", (40, 1, 1), 1, (0,), dict(inputs.SPITZER_MC_SAT, phi=0.01)),
    ("2d_x_open_mc", (24, 18, 1), 2, (0,), dict(inputs.SPITZER_MC, kperp_ratio=0.05)),
    ("2d_both_open_mean_upwind", (20, 22, 1), 2, (0, 1), dict(inputs.SPITZER_MC_SAT, limiter=0, saturation=2, phi=0.02)),
    ("3d_xz_open_mc_sat", (14, 12, 10), 3, (0, 2), dict(inputs.SPITZER_MC_SAT, phi=0.01)),
    ("3d_all_open_const", (10, 9, 8), 3, (0, 1, 2), dict(inputs.BASE, kperp_ratio=0.1)),
]


def case_fields(name, n, ndim):
    rng = np.random.default_rng(abs(hash(name)) % (1 << 32))
    shape = (n[2], n[1], n[0])
    T = 1.0 + 0.3 * rng.random(shape)
    B = rng.standard_normal((3,) + shape)
    if ndim < 3:
        B[2] = 0.0
    b = inputs.unit_vectors(B)
    return T, b


def grids(n, ndim, open_axes, p):
    h = (0.05, 0.04, 0.06)
    bnd = tuple(1 if d in open_axes else 0 for d in range(3))
    g_open = oracle.Grid(n=n, h=h, ndim=ndim, boundary=bnd, **p)
    n_ext = tuple(2 * n[d] if d in open_axes else n[d] for d in range(3))
    g_per = oracle.Grid(n=n_ext, h=h, ndim=ndim, **p)
    return g_open, g_per


@pytest.mark.parametrize("name,n,ndim,open_axes,p", CASES)
def test_outflow_flux_div_is_the_mirrored_periodic_one(name, n, ndim, open_axes, p):
    T, b = case_fields(name, n, ndim)
    g_open, g_per = grids(n, ndim, open_axes, p)
    got = oracle.flux_div(g_open, T, b)
    ref = block(oracle.flux_div(g_per, mirror(T, open_axes), mirror(b, open_axes)), n)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # and the boundary matters: the periodic result differs
    g_p = oracle.Grid(n=n, h=g_open.h, ndim=ndim, **p)
    assert np.abs(oracle.flux_div(g_p, T, b) - got).max() > 1e-6 * np.abs(got).max()


@pytest.mark.parametrize("name,n,ndim,open_axes,p", CASES)
def test_outflow_superstep_is_the_mirrored_periodic_one(name, n, ndim, open_axes, p):
    T, b = case_fields(name, n, ndim)
    if ndim == 1:
        b[:] = 0.0
        b[0] = 1.0
    else:
        for ax in open_axes:        # no field component along an open axis
            b[ax] = 0.0
        nb = np.sqrt((b * b).sum(axis=0))
        b = np.where(nb > 0, b / np.where(nb > 0, nb, 1.0), 0.0)
        if not (nb > 0).any():
            b[2 if 2 not in open_axes else 1] = 1.0
    g_open, g_per = grids(n, ndim, open_axes, p)
    dt = inputs.midpoint_ratio(7) * oracle.dt_par(g_open, T)
    got, s, _ = oracle.superstep(g_open, T, b, dt)
    ref, s_ref, _ = oracle.superstep(g_per, mirror(T, open_axes), mirror(b, open_axes), dt)
    assert s == s_ref == 7
    assert np.abs(got - block(ref, n)).max() <= 1e-12 * np.abs(got - T).max()


def test_outflow_1d_is_insulated():
    """b along x in 1D: the boundary faces see no gradient, so the total heat
    is conserved to rounding by an outflow super-step."""
    n = (64, 1, 1)
    T, b = case_fields("1d_insulated", n, 1)
    b[:] = 0.0
    b[0] = 1.0
    g = oracle.Grid(n=n, h=(0.02, 1, 1), ndim=1, boundary=(1, 0, 0), **dict(inputs.SPITZER_MC_SAT, phi=0.02))
    out, s, _ = oracle.superstep(g, T, b, inputs.midpoint_ratio(9) * oracle.dt_par(g, T))
    assert abs(out.sum() - T.sum()) <= 1e-13 * T.sum() * s


def test_outflow_lets_heat_cross_a_tilted_field_boundary():
    """with the field oblique to an open edge the transverse gradients drive
    a flux through it, so the total heat changes (it cannot with periodic
    axes)"""
    n = (24, 18, 1)
    T, b = case_fields("2d_x_open_mc", n, 2)
    p = dict(inputs.SPITZER_MC, kperp_ratio=0.05)
    dt = 3.0 * oracle.dt_par(oracle.Grid(n=n, h=(0.05, 0.04, 1.0), ndim=2, **p), T)
    per, _, _ = oracle.superstep(oracle.Grid(n=n, h=(0.05, 0.04, 1.0), ndim=2, **p), T, b, dt)
    opn, _, _ = oracle.superstep(oracle.Grid(n=n, h=(0.05, 0.04, 1.0), ndim=2, boundary=(1, 0, 0), **p), T, b, dt)
    assert abs(per.sum() - T.sum()) <= 1e-13 * T.sum() * 10
    assert abs(opn.sum() - T.sum()) > 1e-9 * T.sum()
