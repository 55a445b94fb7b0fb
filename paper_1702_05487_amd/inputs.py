"""Seeded synthetic inputs for the RKL2 conduction workloads.

This module only makes input data (temperature fields, magnetic-field unit
vectors, grid parameters and super-step ratios).  It holds none of the
method's arithmetic and is the one piece of code that both the HIP path's
callers and the CPU oracle's callers use.

Fields are numpy float64 arrays with layout [n2][n1][n0] (axis 0 fastest);
vector fields are (3, n2, n1, n0), component-major.

Random fields.  A band-limited random field is a sum of Fourier modes with
integer wave numbers m = (m0, m1, m2), kmin <= |m| <= kmax, over the periodic
box; mode amplitudes are complex Gaussians scaled by |m|^(slope/2) so that the
3D power spectrum goes as |m|^slope (slope = -11/3 here).  The Gaussians are
drawn for the full cube |m_d| <= 16 in one fixed order, so a given seed gives
the same continuous field at every resolution.  Vector fields have each mode
projected perpendicular to its physical wave vector (divergence-free).  The
field is evaluated at cell centres by three separable complex contractions,
which is exact (no FFT aliasing) and cheap because the band is narrow.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

KCUBE = 16           # wave numbers are drawn for |m_d| <= KCUBE
SLOPE = -11.0 / 3.0  # 3D power-spectrum slope


def _phases(n: int, ks: np.ndarray):
    """exp(2 pi i m x) at the cell centres x = (i + 1/2)/n, shape (len(ks), n)."""
    x = (np.arange(n) + 0.5) / n
    return np.exp(2j * np.pi * np.outer(ks, x))


def band_limited_field(n, seed: int, ncomp: int = 1, kmin: float = 2.0,
                       kmax: float = 16.0, slope: float = SLOPE,
                       solenoidal: bool = False, box=(1.0, 1.0, 1.0),
                       device=None):
    """Random band-limited periodic field sampled at cell centres.

    n: (n0, n1, n2) cells; box: physical box lengths (used only for the
    divergence-free projection).  Returns (ncomp, n2, n1, n0) float64: a
    numpy array when ``device`` is None, else a torch tensor on ``device``
    (the contraction then runs there; the coefficients are always drawn with
    numpy, so the field is the same function either way).
    """
    import torch
    n0, n1, n2 = (int(v) for v in n)
    K = KCUBE
    ks = np.arange(-K, K + 1)
    rng = np.random.default_rng(seed)
    shape = (ncomp, 2 * K + 1, 2 * K + 1, 2 * K + 1)   # [comp][m2][m1][m0]
    coef = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    m2, m1, m0 = np.meshgrid(ks, ks, ks, indexing="ij")
    mag = np.sqrt(m0 ** 2 + m1 ** 2 + m2 ** 2).astype(np.float64)
    keep = (mag >= kmin) & (mag <= kmax)
    amp = np.zeros_like(mag)
    amp[keep] = mag[keep] ** (slope / 2.0)
    coef *= amp[None]
    if solenoidal:
        if ncomp != 3:
            raise ValueError("solenoidal fields need 3 components")
        k = np.stack([m0 / box[0], m1 / box[1], m2 / box[2]])   # physical wave vector
        k2 = (k ** 2).sum(0)
        k2[k2 == 0] = 1.0
        kc = (k * coef).sum(0)
        coef = coef - k * (kc / k2)[None]
    dev = torch.device("cpu") if device is None else torch.device(device)
    out = torch.zeros((ncomp, n2, n1, n0), dtype=torch.float64, device=dev)
    act = np.nonzero(amp.reshape(-1) > 0)[0]
    if act.size:
        # only wave numbers inside the band matter
        idx = np.unravel_index(act, amp.shape)
        used = ks[np.unique(np.concatenate(idx))]
        sel = np.searchsorted(ks, used)
        coef = coef[:, sel][:, :, sel][:, :, :, sel]
        u = used.size
        E0 = torch.from_numpy(_phases(n0, used)).to(dev)
        E1 = torch.from_numpy(_phases(n1, used)).to(dev)
        E2 = torch.from_numpy(_phases(n2, used)).to(dev)
        E0r = torch.cat([E0.real, -E0.imag], 0)                       # (2u, n0)
        zchunk = max(1, min(n2, (1 << 25) // max(1, n1 * n0)))
        for c in range(ncomp):
            C = torch.from_numpy(np.ascontiguousarray(coef[c])).to(dev)  # [m2][m1][m0]
            A = (C.reshape(u, u * u).T @ E2).reshape(u, u, n2)          # [m1][m0][z]
            for z0 in range(0, n2, zchunk):
                z1 = min(n2, z0 + zchunk)
                Az = A[:, :, z0:z1].permute(2, 1, 0).reshape((z1 - z0) * u, u)  # [z][m0] x [m1]
                B = (Az @ E1).reshape(z1 - z0, u, n1).permute(0, 2, 1)     # [z][y][m0]
                Bc = torch.cat([B.real, B.imag], 2).reshape(-1, 2 * u)
                out[c, z0:z1] = (Bc @ E0r).reshape(z1 - z0, n1, n0)
    return out.numpy() if device is None else out


def unit_vectors(B):
    """B/|B| per cell (float64, numpy or torch); cells with |B| == 0 get (1, 0, 0)."""
    mag = (B * B).sum(0) ** 0.5
    zero = mag == 0
    out = B / (mag + zero)[None]
    out[0][zero] = 1.0
    return out


def tangled_b(n, seed: int, kmax: float = 16.0, box=(1.0, 1.0, 1.0), device=None):
    """Unit vectors of a divergence-free k^-11/3 random field, 2 <= |m| <= kmax."""
    B = band_limited_field(n, seed, ncomp=3, kmin=2.0, kmax=kmax,
                           solenoidal=True, box=box, device=device)
    return unit_vectors(B)


def noisy_temperature(n, seed: int, amp: float = 0.1, kmax: float = 16.0, device=None):
    """T = 1 + amp * phi / max|phi| with phi a k^-11/3 scalar field."""
    phi = band_limited_field(n, seed, ncomp=1, kmin=2.0, kmax=kmax, device=device)[0]
    return 1.0 + amp * phi / abs(phi).max()


def midpoint_ratio(s: int) -> float:
    """Super-step ratio dt_hyp/dt_par chosen so that the stage-count root of the
    RKL2 rule lands at s - 1/2, half-way between integers (no rounding ties):
    r = ((s - 1/2)^2 + (s - 1/2) - 2) / 4."""
    x = s - 0.5
    return (x * x + x - 2.0) / 4.0


# --------------------------------------------------------------------------
# The workloads.  Each is one periodic grid (or a set of them) plus the ratio
# dt_hyp/dt_par that fixes the super-step; the harness turns the ratio into
# dt_hyp with whichever dt_par it has (the oracle's, or the library's own).
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n: tuple                  # (n0, n1, n2)
    ndim: int
    params: dict              # limiter, saturation, phi, kappa0, kappa_exp, kperp_ratio, rho, gamma, cp
    ratio: float              # dt_hyp / dt_par
    steps: int
    precision: str            # "fp64" or "mixed"
    T: np.ndarray = field(default=None, repr=False)
    b: np.ndarray = field(default=None, repr=False)

    @property
    def h(self):
        return tuple(1.0 / v for v in self.n)

    @property
    def cells(self):
        return int(np.prod(self.n))


BASE = dict(limiter=0, saturation=0, phi=0.3, kappa0=1.0, kappa_exp=0.0,
            kperp_ratio=0.0, rho=1.0, gamma=2.0, cp=0.5)
SPITZER_MC = dict(BASE, limiter=1, kappa_exp=2.5, kperp_ratio=1e-3)
SPITZER_MC_SAT = dict(SPITZER_MC, saturation=1)


def gaussian_pulse_2d(n: int = 64, fields: bool = True) -> Workload:
    """2D n x n periodic unit box, uniform b at 45 degrees, kappa_par = 1,
    kappa_perp = 0, T = 1 + exp(-r^2/0.01) about the box centre,
    dt_hyp = 50 dt_par, 5 super-steps, FP64."""
    w = Workload("gaussian2d_%d" % n, (n, n, 1), 2, dict(BASE), 50.0, 5, "fp64")
    if fields:
        x = (np.arange(n) + 0.5) / n
        X = x[None, :]
        Y = x[:, None]
        r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2
        w.T = (1.0 + np.exp(-r2 / 0.01))[None].copy()
        b = np.zeros((3, 1, n, n))
        b[0] = b[1] = 1.0 / np.sqrt(2.0)
        w.b = b
    return w


def tangled_3d(n: int, precision: str, saturation: bool, s: int, steps: int,
               seed_b: int = 1, seed_T: int = 2, fields: bool = True, device=None) -> Workload:
    """3D n^3 periodic unit box, tangled k^-11/3 b, T = 1 + 0.1 noise,
    kappa_par = T^2.5, kappa_perp = 1e-3 kappa_par, MC-limited transverse
    gradients, optional saturation (phi = 0.3, rho = 1)."""
    p = dict(SPITZER_MC_SAT if saturation else SPITZER_MC)
    w = Workload("tangled3d_%d_%s%s" % (n, precision, "_sat" if saturation else ""),
                 (n, n, n), 3, p, midpoint_ratio(s), steps, precision)
    if fields:
        w.b = tangled_b((n, n, n), seed_b, device=device)
        w.T = noisy_temperature((n, n, n), seed_T, device=device)
    return w


def spitzer_256(fields: bool = True, device=None) -> Workload:
    """256^3 FP64, no saturation, s = 16, 10 super-steps."""
    return tangled_3d(256, "fp64", False, 16, 10, fields=fields, device=device)


def saturated_512(fields: bool = True, device=None) -> Workload:
    """512^3 mixed precision with saturation, s = 24, 10 super-steps."""
    return tangled_3d(512, "mixed", True, 24, 10, fields=fields, device=device)


def saturated_512_upwind(fields: bool = True, device=None) -> Workload:
    """saturated_512 with the upwind saturated flux (q of the upwind cell)."""
    w = tangled_3d(512, "mixed", True, 24, 10, fields=fields, device=device)
    w.name += "_upwind"
    w.params["saturation"] = 2
    return w


def fused_768(fields: bool = True, device=None) -> Workload:
    """768^3 mixed precision with saturation, s = 32, 20 super-steps."""
    return tangled_3d(768, "mixed", True, 32, 20, fields=fields, device=device)


@dataclass
class PatchSet:
    """Independent periodic patches with cells of width 1/64."""
    n: list                     # per patch (n0, n1, n2)
    s: list                     # per patch target stage count
    ratio: list                 # per patch dt_hyp/dt_par
    params: dict
    T: list = field(default=None, repr=False)
    b: list = field(default=None, repr=False)

    @property
    def cells(self):
        return [int(np.prod(v)) for v in self.n]


def patch_set(npatch: int = 2000, seed: int = 7, fields: bool = True,
              lo: int = 16, hi: int = 64, smin: int = 4, smax: int = 40, device=None) -> PatchSet:
    """Patch edges i.i.d. log-uniform in [lo, hi] per axis (rounded); each patch
    has its own tangled b (seed 1000+2p) and T = 1 + 0.1 noise (seed 1001+2p)
    with 2 <= |m| <= min(16, n_min/4), and a stage count drawn uniformly in
    [smin, smax]."""
    rng = np.random.default_rng(seed)
    edges = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=(npatch, 3)))).astype(int)
    svals = rng.integers(smin, smax + 1, size=npatch)
    ps = PatchSet([tuple(int(v) for v in e) for e in edges], [int(v) for v in svals],
                  [midpoint_ratio(int(v)) for v in svals], dict(SPITZER_MC))
    if fields:
        ps.T, ps.b = [], []
        for p, n in enumerate(ps.n):
            kmax = min(16.0, float(min(n) // 4))
            box = tuple(v / 64.0 for v in n)
            ps.b.append(tangled_b(n, 1000 + 2 * p, kmax=kmax, box=box, device=device))
            ps.T.append(noisy_temperature(n, 1001 + 2 * p, kmax=kmax, device=device))
    return ps


# --------------------------------------------------------------------------
# The paper's validation problems (Sec. 4.1.2 and 4.1.3).  Both are periodic;
# only the initial fields and parameters are made here.
# --------------------------------------------------------------------------

RING_PARAMS = dict(BASE)              # kappa_par = 1, kappa_perp = 0, no saturation


def ring(N: int):
    """Ring diffusion (Sec. 4.1.3): [-1, 1]^2 with N x N cells, circular field
    lines b = (y, -x)/r, T = 12 inside the arc 11pi/12 <= theta <= 13pi/12,
    0.5 <= r <= 0.7, else 10.  Returns (T (1, N, N), b (3, 1, N, N), h)."""
    h = 2.0 / N
    x = -1.0 + (np.arange(N) + 0.5) * h
    X, Y = np.meshgrid(x, x)
    r = np.hypot(X, Y)
    th = np.mod(np.arctan2(Y, X), 2.0 * np.pi)
    arc = (th >= 11.0 * np.pi / 12.0) & (th <= 13.0 * np.pi / 12.0) & (r >= 0.5) & (r <= 0.7)
    T = np.where(arc, 12.0, 10.0)
    b = np.zeros((3, 1, N, N))
    b[0, 0] = Y / r
    b[1, 0] = -X / r
    return T[None], b, h


SAWTOOTH_PARAMS = dict(BASE, kappa0=40.0, saturation=1, phi=0.3)


def sawtooth(N: int = 400, L: float = 20.0):
    """Saw-tooth profile (Sec. 4.1.2): x in [-L/2, L/2) with N cells,
    T = 10 + 20 (x/10 - floor(x/10 + 1/2)) (period 10, range [0, 20)), field
    along x.  Returns (T (1, 1, N), b (3, 1, 1, N), h)."""
    h = L / N
    x = -L / 2.0 + (np.arange(N) + 0.5) * h
    T = 10.0 + 20.0 * (x / 10.0 - np.floor(x / 10.0 + 0.5))
    b = np.zeros((3, 1, 1, N))
    b[0] = 1.0
    return T[None, None], b, h
