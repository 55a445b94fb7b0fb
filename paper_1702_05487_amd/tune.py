"""Autotuner front end: picks the stencil kernel variant (tile shape and
z-chunk length) for a grid by timing every variant on the caller's own
fields (``rkl_autotune`` in librkl), and remembers the choice in a JSON cache
keyed by everything that changes the kernel's cost or the variants a plan
may use: device name, grid shape, flux precision, limiter, saturation form,
conductivity law and boundaries.

Cache file: $RKL_TUNE_CACHE, else ~/.cache/rkl/tune.json.  Writes are atomic
(temp file + rename); a corrupt or unreadable cache is ignored.
"""
from __future__ import annotations

import json
import os
import tempfile

from . import rkl


def cache_path(path=None):
    if path:
        return path
    env = os.environ.get("RKL_TUNE_CACHE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "rkl", "tune.json")


def _load(path):
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _save(path, d):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(path) or ".", prefix=".tune")
    try:
        with os.fdopen(fd, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except BaseException:
        try:
            os.unlink(tmp)
        except OSError:
            pass
        raise


def _cached_variant(d, k):
    """the cached variant index under key k, or None if absent or malformed"""
    e = d.get(k)
    v = e.get("variant") if isinstance(e, dict) else None
    if isinstance(v, int) and not isinstance(v, bool) and 0 <= v < rkl.rkl_variant_count():
        return v
    return None


def key(plan, grid):
    import torch
    d = plan.descs[grid]
    kind = "const" if d.kappa_exp == 0.0 else ("spitzer" if d.kappa_exp == 2.5 else "power")
    return "|".join(str(x) for x in (
        torch.cuda.get_device_name(torch.cuda.current_device()), tuple(d.n), d.ndim,
        "mixed" if plan.precision == rkl.RKL_MIXED else "fp64",
        "mc" if d.limiter else "mean", ("nosat", "sat", "upwind")[d.saturation], kind,
        "bc%d%d%d" % tuple(d.boundary), rkl.rkl_variant_count()))


def autotune(plan, T, b, dt_hyp, reps=2, grid=0, cache=None):
    """Set plan's variant to the fastest one; returns (variant, ms, cached)."""
    import torch
    path = cache_path(cache)
    k = key(plan, grid)
    d = _load(path)
    v = _cached_variant(d, k)
    if v is not None:
        plan.set_variant(v)
        return v, d[k].get("ms"), True
    tp, bp = plan._tb(grid, T, b)
    v, ms = rkl.rkl_autotune(plan.handle, grid, tp, bp, dt_hyp, reps,
                             rkl.ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    d = _load(path)
    d[k] = {"variant": v, "ms": ms, "tile": list(rkl.rkl_variant_info(v))}
    try:
        _save(path, d)
    except OSError:
        pass
    return v, ms, False
