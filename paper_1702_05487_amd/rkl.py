"""Thin ctypes binding of librkl (include/rkl.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of librkl.so.  The C entry points are exposed under their own names
(``rkl_plan``, ``rkl_superstep``, ...); ``Plan`` wraps them for torch
tensors (PyTorch supplies device memory and the current stream).  If the
library cannot be loaded the import of this module's functions raises --
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librkl.so")

RKL_OK, RKL_EINVAL, RKL_ENOMEM, RKL_EDEVICE, RKL_ESTAGES, RKL_ESTATE = range(6)
RKL_FP64, RKL_MIXED = 0, 1
RKL_LIM_NONE, RKL_LIM_MC = 0, 1
RKL_SAT_NONE, RKL_SAT_CENTRAL, RKL_SAT_UPWIND = 0, 1, 2
RKL_BC_PERIODIC, RKL_BC_OUTFLOW, RKL_BC_FIXED = 0, 1, 2
RKL_RKL2, RKL_RKL1 = 0, 1
RKL_FLAG_NONPOS, RKL_FLAG_NONFINITE, RKL_FLAG_STAGES, RKL_FLAG_ABORTED = 1, 2, 4, 8

EXPORTS = [
    "rkl_plan", "rkl_destroy", "rkl_grid_offset", "rkl_set_ghosts", "rkl_flux_div", "rkl_dt_par",
    "rkl_superstep", "rkl_superstep_async", "rkl_supersteps_async", "rkl_superstep_noalloc", "rkl_superstep_batched", "rkl_graph_capture", "rkl_graph_launch",
    "rkl_query", "rkl_variant_count", "rkl_variant_info", "rkl_set_variant", "rkl_last_error",
    "rkl_profile", "rkl_profile_read", "rkl_autotune",
    "rkl_batch_policy_count", "rkl_batch_policy_info", "rkl_set_batch_policy", "rkl_autotune_batched",
    "rkl_set_batch_mode",
    "rkl_subcycle", "rkl_aag", "rkl_stream",
]


class rkl_grid_desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("h", ctypes.c_double * 3),
        ("limiter", ctypes.c_int32),
        ("saturation", ctypes.c_int32),
        ("phi", ctypes.c_double),
        ("kappa0", ctypes.c_double),
        ("kappa_exp", ctypes.c_double),
        ("kperp_ratio", ctypes.c_double),
        ("rho", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("cp", ctypes.c_double),
        ("boundary", ctypes.c_int32 * 3),
    ]


class rkl_options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("smax", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
    ]


class RklError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("librkl status %d: %s" % (status, msg))
        self.status = status


_lib = None


def load(build_if_missing: bool = True):
    """Load librkl.so (building it first only if no library exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise RuntimeError("librkl.so is not built (run paper_1702_05487_amd.build)")
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "rkl_plan": (i32, [P(rkl_grid_desc), i32, P(rkl_options), P(vp)]),
        "rkl_destroy": (i32, [vp]),
        "rkl_grid_offset": (i64, [vp, i32]),
        "rkl_set_ghosts": (i32, [vp, i32, i32, vp, vp]),
        "rkl_flux_div": (i32, [vp, i32, vp, vp, vp, vp]),
        "rkl_dt_par": (i32, [vp, i32, vp, P(dbl), vp]),
        "rkl_superstep": (i32, [vp, i32, vp, vp, dbl, P(i32), vp]),
        "rkl_superstep_async": (i32, [vp, i32, vp, vp, dbl, i32, vp, vp]),
        "rkl_supersteps_async": (i32, [vp, i32, vp, vp, dbl, i32, i32, vp, vp]),
        "rkl_superstep_noalloc": (i32, [P(rkl_grid_desc), i32, vp, vp, dbl, i32, vp, vp]),
        "rkl_superstep_batched": (i32, [vp, vp, vp, vp, vp, vp]),
        "rkl_graph_capture": (i32, [vp, vp, vp, vp, vp, vp]),
        "rkl_graph_launch": (i32, [vp, vp]),
        "rkl_query": (i32, [vp, i32, P(i32), P(dbl), P(ctypes.c_uint32)]),
        "rkl_variant_count": (i32, []),
        "rkl_variant_info": (i32, [i32, P(i32), P(i32), P(i32), P(i32)]),
        "rkl_set_variant": (i32, [vp, i32]),
        "rkl_last_error": (ctypes.c_char_p, []),
        "rkl_profile": (i32, [vp, i32]),
        "rkl_profile_read": (i32, [vp, i32, P(dbl), P(i64), P(i64)]),
        "rkl_autotune": (i32, [vp, i32, vp, vp, dbl, i32, P(i32), P(dbl), vp]),
        "rkl_batch_policy_count": (i32, []),
        "rkl_batch_policy_info": (i32, [i32, P(i32), P(i32)]),
        "rkl_set_batch_policy": (i32, [vp, i32]),
        "rkl_set_batch_mode": (i32, [vp, i32]),
        "rkl_autotune_batched": (i32, [vp, vp, vp, vp, i32, P(i32), P(dbl), vp]),
        "rkl_subcycle": (i32, [vp, i32, vp, vp, dbl, i64, P(i64), vp]),
        "rkl_aag": (i32, [vp, i32, vp, vp, dbl, dbl, i32, P(i32), vp]),
        "rkl_stream": (i32, [vp, vp, i64, i32, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != RKL_OK:
        raise RklError(status, load().rkl_last_error().decode())


# -------------------------------------------------- raw C entry points ----
def rkl_plan(descs, precision=RKL_FP64, variant=-1, smax=0, scheme=RKL_RKL2):
    arr = (rkl_grid_desc * len(descs))(*descs)
    opt = rkl_options(precision, variant, smax, scheme)
    h = ctypes.c_void_p()
    _check(load().rkl_plan(arr, len(descs), ctypes.byref(opt), ctypes.byref(h)))
    return h


def rkl_destroy(plan):
    _check(load().rkl_destroy(plan))


def rkl_grid_offset(plan, grid):
    return load().rkl_grid_offset(plan, grid)


def rkl_flux_div(plan, grid, T_ptr, b_ptr, out_ptr, stream):
    _check(load().rkl_flux_div(plan, grid, T_ptr, b_ptr, out_ptr, stream))


def rkl_dt_par(plan, grid, T_ptr, stream):
    v = ctypes.c_double()
    _check(load().rkl_dt_par(plan, grid, T_ptr, ctypes.byref(v), stream))
    return v.value


def rkl_superstep(plan, grid, T_ptr, b_ptr, dt_hyp, stream):
    s = ctypes.c_int32()
    _check(load().rkl_superstep(plan, grid, T_ptr, b_ptr, float(dt_hyp), ctypes.byref(s), stream))
    return s.value


def rkl_superstep_async(plan, grid, T_ptr, b_ptr, dt_hyp, s_cap, s_ptr, stream):
    _check(load().rkl_superstep_async(plan, grid, T_ptr, b_ptr, float(dt_hyp), int(s_cap), s_ptr, stream))


def rkl_supersteps_async(plan, grid, T_ptr, b_ptr, dt_hyp, nsteps, s_cap, s_ptr, stream):
    _check(load().rkl_supersteps_async(plan, grid, T_ptr, b_ptr, float(dt_hyp), int(nsteps), int(s_cap), s_ptr,
                                       stream))


NOALLOC_MAX_CELLS = 2097152
NOALLOC_MAX_STAGES = 256


def rkl_superstep_noalloc(desc, precision, T_ptr, b_ptr, dt_hyp, s_cap, s_ptr, stream):
    _check(load().rkl_superstep_noalloc(ctypes.byref(desc), int(precision), T_ptr, b_ptr, float(dt_hyp),
                                        int(s_cap), s_ptr, stream))


def superstep_noalloc(desc, T, b, dt_hyp, s_cap, s_out=None, precision="fp64"):
    """One allocation-free super-step of the grid `desc` on torch tensors
    (T in place; s lands in the int32 device tensor s_out)."""
    import torch
    prec = RKL_MIXED if precision in ("mixed", RKL_MIXED) else RKL_FP64
    n = desc.n[0] * desc.n[1] * desc.n[2]
    tp = _dev_ptr(T, torch.float64, n, "T")
    bp = _dev_ptr(b, torch.float32 if prec == RKL_MIXED else torch.float64, 3 * n, "b")
    sp = None if s_out is None else _dev_ptr(s_out, torch.int32, 1, "s_out")
    rkl_superstep_noalloc(desc, prec, tp, bp, dt_hyp, s_cap, sp, _stream())


def rkl_subcycle(plan, grid, T_ptr, b_ptr, dt_hyp, max_sub, stream):
    n = ctypes.c_int64()
    _check(load().rkl_subcycle(plan, grid, T_ptr, b_ptr, float(dt_hyp), int(max_sub), ctypes.byref(n), stream))
    return n.value


def rkl_aag(plan, grid, T_ptr, b_ptr, dt_hyp, nu, max_s, stream):
    n = ctypes.c_int32()
    _check(load().rkl_aag(plan, grid, T_ptr, b_ptr, float(dt_hyp), float(nu), int(max_s), ctypes.byref(n), stream))
    return n.value


def rkl_superstep_batched(plan, T_ptr, b_ptr, dt_ptr, s_ptr, stream):
    _check(load().rkl_superstep_batched(plan, T_ptr, b_ptr, dt_ptr, s_ptr, stream))


def rkl_graph_capture(plan, T_ptr, b_ptr, dt_ptr, s_ptr, stream):
    _check(load().rkl_graph_capture(plan, T_ptr, b_ptr, dt_ptr, s_ptr, stream))


def rkl_graph_launch(plan, stream):
    _check(load().rkl_graph_launch(plan, stream))


def rkl_query(plan, grid):
    s, dtp, fl = ctypes.c_int32(), ctypes.c_double(), ctypes.c_uint32()
    _check(load().rkl_query(plan, grid, ctypes.byref(s), ctypes.byref(dtp), ctypes.byref(fl)))
    return s.value, dtp.value, fl.value


def rkl_variant_count():
    return load().rkl_variant_count()


def rkl_variant_info(v):
    """(tile_x, tile_y, tile_z, stages per launch) of variant v."""
    x, y, z, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().rkl_variant_info(v, ctypes.byref(x), ctypes.byref(y), ctypes.byref(z), ctypes.byref(f)))
    return x.value, y.value, z.value, f.value


def rkl_set_variant(plan, v):
    _check(load().rkl_set_variant(plan, v))


def rkl_set_ghosts(plan, grid, axis, lo_ptr, hi_ptr):
    _check(load().rkl_set_ghosts(plan, grid, axis, lo_ptr, hi_ptr))


def ghost_shape(n, axis):
    """shape of one ghost layer of a fixed axis of a grid of n = (n0, n1, n2)
    cells: (n_b + 2, n_a + 2), a < b the other two axes"""
    a, b = [e for e in range(3) if e != axis]
    return (n[b] + 2, n[a] + 2)


def rkl_stream(src_ptr, dst_ptr, nbytes, mode, stream):
    _check(load().rkl_stream(src_ptr, dst_ptr, int(nbytes), int(mode), stream))


def stream_probe(src, dst, mode=0):
    """One rkl_stream sweep over the torch tensor src (mode 0/1/3: copy into
    dst, same size; mode 2: read-only, dst holds src.nbytes // 8192 doubles)."""
    import torch
    for t, name in ((src, "src"), (dst, "dst")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
            raise TypeError("%s must be a contiguous CUDA (HIP) tensor" % name)
    need = src.nbytes // 8192 * 8 if mode == 2 else src.nbytes
    if dst.nbytes < need:
        raise ValueError("dst holds %d bytes, %d needed" % (dst.nbytes, need))
    rkl_stream(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), src.nbytes, mode, _stream())


def rkl_last_error():
    return load().rkl_last_error().decode()


def rkl_autotune(plan, grid, T_ptr, b_ptr, dt_hyp, reps, stream):
    v, ms = ctypes.c_int32(), ctypes.c_double()
    _check(load().rkl_autotune(plan, grid, T_ptr, b_ptr, float(dt_hyp), int(reps), ctypes.byref(v),
                               ctypes.byref(ms), stream))
    return v.value, ms.value


def rkl_batch_policy_count():
    return load().rkl_batch_policy_count()


def rkl_batch_policy_info(policy):
    """(half_rows, tile_z) of a batched tile policy."""
    h, z = ctypes.c_int32(), ctypes.c_int32()
    _check(load().rkl_batch_policy_info(policy, ctypes.byref(h), ctypes.byref(z)))
    return h.value, z.value


def rkl_set_batch_policy(plan, policy):
    _check(load().rkl_set_batch_policy(plan, policy))


def rkl_set_batch_mode(plan, mode):
    _check(load().rkl_set_batch_mode(plan, int(mode)))


def rkl_autotune_batched(plan, T_ptr, b_ptr, dt_ptr, reps, stream):
    v, ms = ctypes.c_int32(), ctypes.c_double()
    _check(load().rkl_autotune_batched(plan, T_ptr, b_ptr, dt_ptr, int(reps), ctypes.byref(v),
                                       ctypes.byref(ms), stream))
    return v.value, ms.value


def rkl_profile(plan, enable):
    _check(load().rkl_profile(plan, int(enable)))


def rkl_profile_read(plan, fuse=1):
    ms, n, c = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().rkl_profile_read(plan, int(fuse), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(c)))
    return ms.value, n.value, c.value


# ------------------------------------------------------- torch wrapper ----
def grid_desc(n, h, ndim=3, limiter=0, saturation=0, phi=0.3, kappa0=1.0, kappa_exp=0.0,
              kperp_ratio=0.0, rho=1.0, gamma=2.0, cp=0.5, boundary=(0, 0, 0)):
    d = rkl_grid_desc()
    d.ndim = int(ndim)
    for i in range(3):
        d.n[i] = int(n[i])
        d.h[i] = float(h[i])
        d.boundary[i] = int(boundary[i])
    d.limiter, d.saturation = int(limiter), int(saturation)
    d.phi, d.kappa0, d.kappa_exp = float(phi), float(kappa0), float(kappa_exp)
    d.kperp_ratio, d.rho, d.gamma, d.cp = float(kperp_ratio), float(rho), float(gamma), float(cp)
    return d


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, dtype, numel, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.device.index != torch.cuda.current_device():
        raise ValueError("%s is on %s; the current device (the plan's) is cuda:%d"
                         % (name, t.device, torch.cuda.current_device()))
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A librkl plan over one grid or a batch of grids (descs: rkl_grid_desc list)."""

    def __init__(self, descs, precision="fp64", variant=-1, smax=0, scheme="rkl2"):
        import torch
        self.descs = list(descs)
        self.precision = RKL_MIXED if precision in ("mixed", RKL_MIXED) else RKL_FP64
        self.scheme = RKL_RKL1 if scheme in ("rkl1", RKL_RKL1) else RKL_RKL2
        self.bdtype = torch.float32 if self.precision == RKL_MIXED else torch.float64
        self.handle = rkl_plan(self.descs, self.precision, variant, smax, self.scheme)
        self.cells = [d.n[0] * d.n[1] * d.n[2] for d in self.descs]

    def close(self):
        if self.handle:
            rkl_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _tb(self, g, T, b):
        import torch
        return (_dev_ptr(T, torch.float64, self.cells[g], "T"),
                _dev_ptr(b, self.bdtype, 3 * self.cells[g], "b"))

    def flux_div(self, T, b, out=None, grid=0):
        import torch
        if out is None:
            out = torch.empty_like(T)
        tp, bp = self._tb(grid, T, b)
        rkl_flux_div(self.handle, grid, tp, bp, _dev_ptr(out, torch.float64, self.cells[grid], "out"), _stream())
        return out

    def dt_par(self, T, grid=0):
        import torch
        return rkl_dt_par(self.handle, grid, _dev_ptr(T, torch.float64, self.cells[grid], "T"), _stream())

    def superstep(self, T, b, dt_hyp, grid=0):
        """Advance T in place by one super-step; returns the stage count."""
        tp, bp = self._tb(grid, T, b)
        return rkl_superstep(self.handle, grid, tp, bp, dt_hyp, _stream())

    def superstep_async(self, T, b, dt_hyp, s_cap, s_out=None, grid=0):
        """Advance T in place by one super-step without host synchronisation
        (s_cap stage launches; s lands in the int32 device tensor s_out)."""
        import torch
        tp, bp = self._tb(grid, T, b)
        sp = None if s_out is None else _dev_ptr(s_out, torch.int32, 1, "s_out")
        rkl_superstep_async(self.handle, grid, tp, bp, dt_hyp, s_cap, sp, _stream())

    def supersteps_async(self, T, b, dt_hyp, nsteps, s_cap, s_out=None, grid=0):
        """nsteps super-steps one after another without host synchronisation
        (each super-step after the first takes the extrema its predecessor's
        last stage kept); the stage counts land in the int32 device tensor
        s_out of nsteps entries."""
        import torch
        tp, bp = self._tb(grid, T, b)
        sp = None if s_out is None else _dev_ptr(s_out, torch.int32, int(nsteps), "s_out")
        rkl_supersteps_async(self.handle, grid, tp, bp, dt_hyp, nsteps, s_cap, sp, _stream())

    def subcycle(self, T, b, dt_hyp, max_sub=1 << 20, grid=0):
        """Explicit sub-cycling over dt_hyp (T in place); returns the number of sub-steps."""
        tp, bp = self._tb(grid, T, b)
        return rkl_subcycle(self.handle, grid, tp, bp, dt_hyp, max_sub, _stream())

    def aag(self, T, b, dt_hyp, nu, max_s=4096, grid=0):
        """One AAG super-time-step with damping nu (T in place); returns the stage count."""
        tp, bp = self._tb(grid, T, b)
        return rkl_aag(self.handle, grid, tp, bp, dt_hyp, nu, max_s, _stream())

    def query(self, grid=0):
        return rkl_query(self.handle, grid)

    def set_variant(self, v):
        rkl_set_variant(self.handle, v)

    def set_ghosts(self, axis, lo, hi, grid=0):
        """Ghost temperatures beyond the low and high edge of fixed axis
        `axis`: float64 device tensors of ghost_shape(n, axis).  The plan
        reads them at every later stencil call; they are kept referenced
        here so that they stay alive."""
        import torch
        d = self.descs[grid]
        shape = ghost_shape(tuple(d.n), axis)
        ptrs = []
        for name, t in (("lo", lo), ("hi", hi)):
            if tuple(t.shape) != shape:
                raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), shape))
            ptrs.append(_dev_ptr(t, torch.float64, shape[0] * shape[1], name))
        rkl_set_ghosts(self.handle, grid, axis, ptrs[0], ptrs[1])
        if not hasattr(self, "_ghosts"):
            self._ghosts = {}
        self._ghosts[(grid, axis)] = (lo, hi)

    def autotune(self, T, b, dt_hyp, reps=2, grid=0, cache=None):
        """Pick the fastest stencil variant for this grid (see tune.py for the
        JSON cache); returns (variant, ms per super-step, from_cache)."""
        from . import tune
        return tune.autotune(self, T, b, dt_hyp, reps=reps, grid=grid, cache=cache)

    # batched: packed tensors
    def offsets(self):
        return [rkl_grid_offset(self.handle, g) for g in range(len(self.descs) + 1)]

    def superstep_batched(self, T, b, dt_hyp, s_out=None):
        import torch
        tot = sum(self.cells)
        rkl_superstep_batched(self.handle, _dev_ptr(T, torch.float64, tot, "T"),
                              _dev_ptr(b, self.bdtype, 3 * tot, "b"),
                              _dev_ptr(dt_hyp, torch.float64, len(self.descs), "dt_hyp"),
                              None if s_out is None else _dev_ptr(s_out, torch.int32, len(self.descs), "s_out"),
                              _stream())

    def graph_capture(self, T, b, dt_hyp, s_out=None):
        import torch
        tot = sum(self.cells)
        rkl_graph_capture(self.handle, _dev_ptr(T, torch.float64, tot, "T"),
                          _dev_ptr(b, self.bdtype, 3 * tot, "b"),
                          _dev_ptr(dt_hyp, torch.float64, len(self.descs), "dt_hyp"),
                          None if s_out is None else _dev_ptr(s_out, torch.int32, len(self.descs), "s_out"),
                          _stream())

    def graph_launch(self):
        rkl_graph_launch(self.handle, _stream())

    def set_batch_policy(self, policy):
        rkl_set_batch_policy(self.handle, policy)

    def set_batch_mode(self, mode):
        """0: one launch per stage; 1: one persistent launch (see rkl.h)."""
        rkl_set_batch_mode(self.handle, mode)

    def autotune_batched(self, T, b, dt_hyp, reps=2):
        """Pick the fastest batched tile policy by timing; returns (policy, ms)."""
        import torch
        tot = sum(self.cells)
        return rkl_autotune_batched(self.handle, _dev_ptr(T, torch.float64, tot, "T"),
                                    _dev_ptr(b, self.bdtype, 3 * tot, "b"),
                                    _dev_ptr(dt_hyp, torch.float64, len(self.descs), "dt_hyp"), reps, _stream())
