"""Shared test helpers: build oracle grids / library descriptors from one
parameter set, sample oracle values in periodic windows, error norms."""
import numpy as np

import oracle


def oracle_grid(n, h, ndim, params):
    return oracle.Grid(n=tuple(n), h=tuple(h), ndim=ndim, **params)


def lib_desc(n, h, ndim, params):
    from paper_1702_05487_amd import rkl
    return rkl.grid_desc(n, h, ndim=ndim, **params)


def rel_l1(a, ref):
    return float(np.abs(a - ref).sum() / np.abs(ref).sum())


def window(f, center, r):
    """periodic window of half-width r around center (k, j, i) of a [n2][n1][n0]
    field (or (3, n2, n1, n0) vector field)"""
    idx = [np.arange(c - r, c + r + 1) for c in center]
    vec = f.ndim == 4
    a = f
    for ax, ix in enumerate(idx):
        a = np.take(a, ix, axis=ax + (1 if vec else 0), mode="wrap")
    return np.ascontiguousarray(a)


def sampled_superstep(T, b, params, h, s, tau, centers):
    """Y_s at the given cells by running the oracle on periodic windows of
    half-width s + 1: the stencil reaches one cell per stage, so the window's
    wrap-around error cannot reach the centre within s stages."""
    r = s + 1
    out = []
    for c in centers:
        Tw = window(T, c, r)
        bw = window(b, c, r)
        w = 2 * r + 1
        g = oracle.Grid(n=(w, w, w), h=tuple(h), ndim=3, **params)
        Y = oracle.rkl2_fixed(g, Tw, bw, s, tau)
        out.append(Y[r, r, r])
    return np.array(out)
