"""The C-ABI library builds, loads and exports every entry point that
include/rkl.h declares; descriptor validation answers without a GPU."""
import os
import re

import pytest

from paper_1702_05487_amd import rkl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "rkl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rkl_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = rkl.load()
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(rkl.EXPORTS)


def test_descriptor_struct_matches_header(tmp_path):
    # the ctypes mirrors have the layout the C compiler gives the header's structs
    import ctypes
    import subprocess
    fields = [f for f, _ in rkl.rkl_grid_desc._fields_]
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "rkl.h"\nint main(void){\n'
        'printf("%zu %zu\\n", sizeof(rkl_grid_desc), sizeof(rkl_options));\n'
        + "".join('printf("%%zu\\n", offsetof(rkl_grid_desc, %s));\n' % f for f in fields)
        + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    assert int(out[0]) == ctypes.sizeof(rkl.rkl_grid_desc)
    assert int(out[1]) == ctypes.sizeof(rkl.rkl_options)
    for f, off in zip(fields, out[2:]):
        assert int(off) == getattr(rkl.rkl_grid_desc, f).offset, f


@pytest.mark.parametrize("bad", [
    dict(ndim=4), dict(n=(0, 4, 4)), dict(n=(4, 4, 2), ndim=2), dict(h=(0.0, 1, 1)),
    dict(limiter=2), dict(saturation=1, phi=0.0), dict(saturation=2, phi=0.0), dict(saturation=3),
    dict(saturation=-1), dict(kappa0=-1.0), dict(kappa_exp=-0.5),
    dict(boundary=(3, 0, 0)), dict(boundary=(0, -1, 0)), dict(n=(8, 8, 1), ndim=2, boundary=(0, 0, 2)),
    dict(n=(8, 1, 1), ndim=1, boundary=(2, 2, 0)),
    dict(kperp_ratio=1.5), dict(rho=0.0), dict(gamma=1.0), dict(cp=0.6), dict(cp=0.0),
])
def test_invalid_descriptors_are_rejected(bad):
    base = dict(n=(8, 8, 8), h=(0.1, 0.1, 0.1), ndim=3)
    base.update(bad)
    d = rkl.grid_desc(**base)
    with pytest.raises(rkl.RklError) as e:
        rkl.rkl_plan([d])
    assert e.value.status == rkl.RKL_EINVAL
    assert rkl.rkl_last_error()


def test_invalid_options_are_rejected():
    d = rkl.grid_desc((8, 8, 8), (0.1,) * 3)
    for kw in (dict(precision=7), dict(smax=1), dict(smax=5000), dict(variant=999), dict(scheme=2)):
        with pytest.raises(rkl.RklError) as e:
            rkl.rkl_plan([d], **kw)
        assert e.value.status == rkl.RKL_EINVAL
    with pytest.raises(rkl.RklError):
        rkl.rkl_plan([])


def test_variant_table():
    n = rkl.rkl_variant_count()
    assert n >= 3
    fuses = set()
    for v in range(n):
        bx, by, bz, fuse = rkl.rkl_variant_info(v)
        assert bx * by <= 1024 and bz >= 1 and fuse in (1, 2, 3, 4)
        fuses.add(fuse)
        if fuse >= 2:
            # the output tile is (bx-2(F-1)) x (by-2(F-1))
            assert bx > 2 * (fuse - 1) and by > 2 * (fuse - 1)
    assert fuses == {1, 2, 3, 4}
    with pytest.raises(rkl.RklError):
        rkl.rkl_variant_info(n)


def test_batch_policy_table():
    n = rkl.rkl_batch_policy_count()
    assert n >= 2
    seen = set()
    for p in range(n):
        half, tz = rkl.rkl_batch_policy_info(p)
        assert half in (0, 1) and tz >= 1
        seen.add((half, tz))
    assert len(seen) == n           # no duplicate policies
    with pytest.raises(rkl.RklError):
        rkl.rkl_batch_policy_info(n)


def test_c_program_uses_the_abi(tmp_path):
    """A plain C program (no Python, no torch) against include/rkl.h and
    librkl.so: descriptor validation, status codes, the thread's error
    message and the variant table, all answered before any device call."""
    import subprocess
    lib = rkl.load()
    libdir = os.path.dirname(rkl.LIB_PATH)
    src = tmp_path / "use_abi.c"
    src.write_text(r'''
#include <stdio.h>
#include <string.h>
#include "rkl.h"
int main(void) {
    rkl_grid_desc g;
    memset(&g, 0, sizeof g);
    g.ndim = 3; g.n[0] = 8; g.n[1] = 8; g.n[2] = 8;
    g.h[0] = g.h[1] = g.h[2] = 0.1;
    g.kappa0 = 1.0; g.rho = 1.0; g.gamma = 2.0; g.cp = 0.5;
    g.boundary[0] = 7;                       /* not a boundary kind */
    rkl_plan_t p = (rkl_plan_t)1;
    rkl_status st = rkl_plan(&g, 1, NULL, &p);
    if (st != RKL_EINVAL || p != NULL || strstr(rkl_last_error(), "boundary[0]") == NULL) return 1;
    g.boundary[0] = RKL_BC_PERIODIC;
    g.saturation = RKL_SAT_UPWIND;           /* phi = 0 with saturation */
    if (rkl_plan(&g, 1, NULL, &p) != RKL_EINVAL || strstr(rkl_last_error(), "phi") == NULL) return 2;
    rkl_options o = {RKL_MIXED, -1, 1, RKL_RKL2};   /* smax below 2 */
    g.saturation = RKL_SAT_NONE;
    if (rkl_plan(&g, 1, &o, &p) != RKL_EINVAL) return 3;
    int n = rkl_variant_count(), tx, ty, tz, fuse, fused = 0;
    for (int v = 0; v < n; ++v) {
        if (rkl_variant_info(v, &tx, &ty, &tz, &fuse) != RKL_OK) return 4;
        fused += fuse >= 2;
    }
    if (rkl_variant_info(n, &tx, &ty, &tz, &fuse) != RKL_EINVAL) return 5;
    if (rkl_destroy(NULL) != RKL_OK) return 6;
    printf("%d %d\n", n, fused);
    return 0;
}
''')
    exe = tmp_path / "use_abi"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                           "-L", libdir, "-lrkl", "-Wl,-rpath," + libdir])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, (out.returncode, out.stderr)
    n, fused = (int(x) for x in out.stdout.split())
    assert n == rkl.rkl_variant_count() and fused >= 1


def test_noalloc_refuses_sizes_beyond_its_static_scratch():
    # checked on the host before any device call
    import ctypes
    big = rkl.grid_desc((128, 128, 129), (0.01, 0.01, 0.01), ndim=3)
    with pytest.raises(rkl.RklError) as e:
        rkl.rkl_superstep_noalloc(big, rkl.RKL_FP64, ctypes.c_void_p(256), ctypes.c_void_p(4096), 1e-6, 8,
                                  None, None)
    assert e.value.status == rkl.RKL_EINVAL and "RKL_NOALLOC_MAX_CELLS" in str(e.value)
    small = rkl.grid_desc((8, 8, 8), (0.1, 0.1, 0.1), ndim=3)
    for cap in (1, rkl.NOALLOC_MAX_STAGES + 1):
        with pytest.raises(rkl.RklError) as e:
            rkl.rkl_superstep_noalloc(small, rkl.RKL_FP64, ctypes.c_void_p(256), ctypes.c_void_p(4096), 1e-6,
                                      cap, None, None)
        assert "RKL_NOALLOC_MAX_STAGES" in str(e.value)
    with pytest.raises(rkl.RklError):
        rkl.rkl_superstep_noalloc(small, 7, ctypes.c_void_p(256), ctypes.c_void_p(4096), 1e-6, 8, None, None)
    fixed = rkl.grid_desc((8, 8, 8), (0.1, 0.1, 0.1), ndim=3, boundary=(0, rkl.RKL_BC_FIXED, 0))
    with pytest.raises(rkl.RklError) as e:
        rkl.rkl_superstep_noalloc(fixed, rkl.RKL_FP64, ctypes.c_void_p(256), ctypes.c_void_p(4096), 1e-6, 8,
                                  None, None)
    assert e.value.status == rkl.RKL_EINVAL and "RKL_BC_FIXED" in str(e.value)


def test_set_ghosts_checks_its_arguments_on_the_host():
    import ctypes
    with pytest.raises(rkl.RklError) as e:
        rkl.rkl_set_ghosts(None, 0, 0, ctypes.c_void_p(256), ctypes.c_void_p(512))
    assert e.value.status == rkl.RKL_EINVAL
    assert rkl.ghost_shape((5, 4, 3), 0) == (5, 6) and rkl.ghost_shape((5, 4, 3), 1) == (5, 7)
    assert rkl.ghost_shape((5, 4, 3), 2) == (6, 7)
