"""ctypes front end of the serial FP64 oracle (``rkl_oracle.c``).

TEST INFRASTRUCTURE ONLY.  This module compiles and calls the plain C oracle;
it shares nothing with the HIP library and imports nothing from it.  Arrays
are numpy float64, C-contiguous, layout [n2][n1][n0] (axis 0 fastest); ``b``
is shaped (3, n2, n1, n0).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rkl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


class _CGrid(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("h", ctypes.c_double * 3),
        ("limiter", ctypes.c_int),
        ("saturation", ctypes.c_int),
        ("phi", ctypes.c_double),
        ("kappa0", ctypes.c_double),
        ("kappa_exp", ctypes.c_double),
        ("kperp_ratio", ctypes.c_double),
        ("rho", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("cp", ctypes.c_double),
        ("boundary", ctypes.c_int * 3),
        ("ghost", (ctypes.POINTER(ctypes.c_double) * 2) * 3),
    ]


@dataclass
class Grid:
    """Grid + conduction parameters (same meaning as in rkl_oracle.c);
    boundary[d] = 0 periodic, 1 outflow, 2 fixed.  ghosts[d] (fixed axes):
    (low, high) layers of ghost temperatures, each of shape (n_b+2, n_a+2)
    for the other two axes a < b (see ghost_shape)."""
    n: tuple                      # (n0, n1, n2), axis 0 fastest
    h: tuple = (1.0, 1.0, 1.0)
    ndim: int = 3
    limiter: int = 0
    saturation: int = 0
    phi: float = 0.3
    kappa0: float = 1.0
    kappa_exp: float = 0.0
    kperp_ratio: float = 0.0
    rho: float = 1.0
    gamma: float = 2.0
    cp: float = 0.5
    boundary: tuple = (0, 0, 0)
    ghosts: tuple = (None, None, None)
    _c: _CGrid = field(default=None, repr=False, compare=False)

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    def c(self) -> _CGrid:
        g = _CGrid()
        g.ndim = int(self.ndim)
        for d in range(3):
            g.n[d] = int(self.n[d])
            g.h[d] = float(self.h[d])
        g.limiter = int(self.limiter)
        g.saturation = int(self.saturation)
        g.phi = float(self.phi)
        g.kappa0 = float(self.kappa0)
        g.kappa_exp = float(self.kappa_exp)
        g.kperp_ratio = float(self.kperp_ratio)
        g.rho = float(self.rho)
        g.gamma = float(self.gamma)
        g.cp = float(self.cp)
        keep = []
        for d in range(3):
            g.boundary[d] = int(self.boundary[d])
            if self.boundary[d] != 2:
                continue
            if self.ghosts is None or self.ghosts[d] is None:
                raise ValueError("axis %d is fixed but has no ghost layers" % d)
            for side in range(2):
                a = np.ascontiguousarray(self.ghosts[d][side], dtype=np.float64)
                if a.shape != ghost_shape(self.n, d):
                    raise ValueError("ghost layer of axis %d has shape %s, not %s" % (d, a.shape, ghost_shape(self.n, d)))
                keep.append(a)
                g.ghost[d][side] = _ptr(a)
        g._keep = keep          # the layers live as long as the structure
        return g


def ghost_shape(n, d: int):
    """shape of one ghost layer of axis d of a grid of n = (n0, n1, n2)
    cells: (n_b + 2, n_a + 2), a < b the other two axes"""
    a, b = [e for e in range(3) if e != d]
    return (n[b] + 2, n[a] + 2)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, no fast-math)."""
    stale = (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-fPIC", "-shared", "-o", tmp, _SRC, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


def load():
    """Load the oracle library: the one built from rkl_oracle.c, or the one
    named by $RKL_ORACLE_LIB (the mutation tests use this to run the pins
    against deliberately broken copies of the oracle)."""
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(os.environ.get("RKL_ORACLE_LIB") or build())
        dp = ctypes.POINTER(ctypes.c_double)
        gp = ctypes.POINTER(_CGrid)
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = None
        lib.orc_get_threads.argtypes = []
        lib.orc_get_threads.restype = ctypes.c_int
        lib.orc_mc.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.orc_mc.restype = ctypes.c_double
        lib.orc_stages.argtypes = [ctypes.c_double]
        lib.orc_stages.restype = ctypes.c_int
        lib.orc_coeffs.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp]
        lib.orc_coeffs.restype = None
        lib.orc_dt_par.argtypes = [gp, dp]
        lib.orc_dt_par.restype = ctypes.c_double
        lib.orc_flux_div.argtypes = [gp, dp, dp, dp]
        lib.orc_flux_div.restype = None
        lib.orc_face_flux.argtypes = [gp, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.orc_face_flux.restype = ctypes.c_double
        lib.orc_rkl2_fixed.argtypes = [gp, dp, dp, ctypes.c_int, ctypes.c_double]
        lib.orc_rkl2_fixed.restype = None
        lib.orc_superstep.argtypes = [gp, dp, dp, ctypes.c_double, dp]
        lib.orc_subcycle.argtypes = [gp, dp, dp, ctypes.c_double, ctypes.c_long]
        lib.orc_aag_gain.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.orc_aag_gain.restype = ctypes.c_double
        lib.orc_aag_stages.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int]
        lib.orc_aag_stages.restype = ctypes.c_int
        lib.orc_aag_taus.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
        lib.orc_aag_taus.restype = None
        lib.orc_aag_fixed.argtypes = [gp, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        lib.orc_aag_fixed.restype = None
        lib.orc_aag_superstep.argtypes = [gp, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int]
        lib.orc_aag_superstep.restype = ctypes.c_int
        lib.orc_stages_rkl1.argtypes = [ctypes.c_double]
        lib.orc_stages_rkl1.restype = ctypes.c_int
        lib.orc_rkl1_fixed.argtypes = [gp, dp, dp, ctypes.c_int, ctypes.c_double]
        lib.orc_rkl1_fixed.restype = None
        lib.orc_superstep_rkl1.argtypes = [gp, dp, dp, ctypes.c_double, dp]
        lib.orc_superstep_rkl1.restype = ctypes.c_int
        lib.orc_subcycle.restype = ctypes.c_long
        lib.orc_superstep.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _field(g: Grid, a, name):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != g.shape:
        raise ValueError(f"{name}: shape {a.shape} != {g.shape}")
    return a


def _bfield(g: Grid, b):
    b = np.ascontiguousarray(b, dtype=np.float64)
    if b.shape != (3,) + g.shape:
        raise ValueError(f"b: shape {b.shape} != {(3,) + g.shape}")
    return b


def set_threads(n: int) -> int:
    """Threads of the oracle's cell loops (1 = serial, the default).  The
    result is the same bits for any count; returns the count in effect."""
    lib = load()
    lib.orc_set_threads(int(n))
    return lib.orc_get_threads()


def threads() -> int:
    return load().orc_get_threads()


def mc(a: float, b: float) -> float:
    return load().orc_mc(a, b)


def stages(r: float) -> int:
    return load().orc_stages(r)


def coeffs(s: int):
    """(w1, mu, nu, mut, gt) with arrays indexed by stage j = 0..s (s >= 2)."""
    if int(s) < 2:
        raise ValueError("RKL2 needs s >= 2, got %d" % s)
    arrs = [np.zeros(s + 1) for _ in range(4)]
    w1 = ctypes.c_double()
    load().orc_coeffs(s, ctypes.byref(w1), *[_ptr(a) for a in arrs])
    return (w1.value, *arrs)


def dt_par(g: Grid, T) -> float:
    T = _field(g, T, "T")
    cg = g.c()
    return load().orc_dt_par(ctypes.byref(cg), _ptr(T))


def flux_div(g: Grid, T, b) -> np.ndarray:
    T = _field(g, T, "T")
    b = _bfield(g, b)
    out = np.empty(g.shape)
    cg = g.c()
    load().orc_flux_div(ctypes.byref(cg), _ptr(T), _ptr(b), _ptr(out))
    return out


def face_flux(g: Grid, T, b, cell, d: int) -> float:
    """Component d of the flux through the +e_d face of cell (i, j, k)."""
    T = _field(g, T, "T")
    b = _bfield(g, b)
    cg = g.c()
    i, j, k = (int(v) for v in cell)
    return load().orc_face_flux(ctypes.byref(cg), _ptr(T), _ptr(b), i, j, k, int(d))


def rkl2_fixed(g: Grid, T, b, s: int, tau: float) -> np.ndarray:
    """s RKL2 stages of length tau; returns Y_s (input is not modified)."""
    if int(s) < 2:
        raise ValueError("RKL2 needs s >= 2, got %d" % s)
    T = _field(g, T, "T").copy()
    b = _bfield(g, b)
    cg = g.c()
    load().orc_rkl2_fixed(ctypes.byref(cg), _ptr(T), _ptr(b), int(s), float(tau))
    return T


def superstep(g: Grid, T, b, dt_hyp: float):
    """One super-step; returns (T_new, s, dt_par)."""
    T = _field(g, T, "T").copy()
    b = _bfield(g, b)
    cg = g.c()
    dtp = ctypes.c_double()
    s = load().orc_superstep(ctypes.byref(cg), _ptr(T), _ptr(b), float(dt_hyp), ctypes.byref(dtp))
    return T, s, dtp.value


def subcycle(g: Grid, T, b, dt_hyp: float, max_sub: int = 1 << 20):
    """Explicit sub-cycling over dt_hyp; returns (T_new, n_sub)."""
    T = _field(g, T, "T").copy()
    b = _bfield(g, b)
    cg = g.c()
    n = load().orc_subcycle(ctypes.byref(cg), _ptr(T), _ptr(b), float(dt_hyp), int(max_sub))
    return T, n


def stages_rkl1(r: float) -> int:
    """RKL1 stage count for dt_hyp/dt_par = r."""
    return load().orc_stages_rkl1(float(r))


def rkl1_fixed(g: Grid, T, b, s: int, tau: float) -> np.ndarray:
    """s stages of RKL1 over tau; returns Y_s."""
    T = _field(g, T, "T").copy()
    b = _bfield(g, b)
    cg = g.c()
    load().orc_rkl1_fixed(ctypes.byref(cg), _ptr(T), _ptr(b), int(s), float(tau))
    return T


def superstep_rkl1(g: Grid, T, b, dt_hyp: float):
    """One RKL1 super-step; returns (T_new, s, dt_par)."""
    T = _field(g, T, "T").copy()
    b = _bfield(g, b)
    cg = g.c()
    dtp = ctypes.c_double()
    s = load().orc_superstep_rkl1(ctypes.byref(cg), _ptr(T), _ptr(b), float(dt_hyp), ctypes.byref(dtp))
    return T, s, dtp.value


def aag_gain(s: int, nu: float) -> float:
    """AAG-STS gain (sum of the sub-steps over dt_par), Eq. AAG-STS."""
    return load().orc_aag_gain(int(s), float(nu))


def aag_stages(r: float, nu: float, smax: int = 4096) -> int:
    return load().orc_aag_stages(float(r), float(nu), int(smax))


def aag_taus(s: int, nu: float, dt_p: float) -> np.ndarray:
    out = np.empty(s)
    load().orc_aag_taus(int(s), float(nu), float(dt_p), _ptr(out))
    return out


def aag_superstep(g: Grid, T, b, dt_hyp: float, nu: float, smax: int = 4096):
    """One AAG super-step; returns (T_new, s)."""
    T = _field(g, T, "T").copy()
    b = _bfield(g, b)
    cg = g.c()
    s = load().orc_aag_superstep(ctypes.byref(cg), _ptr(T), _ptr(b), float(dt_hyp), float(nu), int(smax))
    return T, s


def aag_fixed(g: Grid, T, b, s: int, nu: float, dt_hyp: float) -> np.ndarray:
    """s AAG sub-steps scaled to sum to dt_hyp; returns the result."""
    T = _field(g, T, "T").copy()
    b = _bfield(g, b)
    cg = g.c()
    load().orc_aag_fixed(ctypes.byref(cg), _ptr(T), _ptr(b), int(s), float(nu), float(dt_hyp))
    return T
