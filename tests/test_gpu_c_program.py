"""A plain C program drives one super-step through include/rkl.h and
librkl.so on the GPU -- no Python or torch in that process: it allocates
device memory with the HIP runtime, plans a 20 x 16 x 12 grid (Spitzer
conduction, MC limiter, central saturation, FP64), reads dt_par, runs
rkl_superstep on the legacy stream, queries the stage count and writes T
back.  The result must match the oracle (rel-L1 <= 1e-12, same s and
dt_par).  The program is built with the host C compiler and run as a child
process."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from helpers import oracle_grid, rel_l1
from paper_1702_05487_amd import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = "/opt/rocm"

SOURCE = r'''
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <hip/hip_runtime_api.h>
#include "rkl.h"

static int rd(const char* path, double* buf, size_t n) {
    FILE* f = fopen(path, "rb");
    if (!f) return 0;
    size_t got = fread(buf, sizeof(double), n, f);
    fclose(f);
    return got == n;
}

int main(int argc, char** argv) {
    if (argc != 8) return 10;
    rkl_grid_desc g;
    memset(&g, 0, sizeof g);
    g.ndim = 3;
    for (int d = 0; d < 3; ++d) { g.n[d] = atoi(argv[1 + d]); g.h[d] = 1.0 / g.n[d]; }
    g.limiter = RKL_LIM_MC; g.saturation = RKL_SAT_CENTRAL; g.phi = 0.3;
    g.kappa0 = 1.0; g.kappa_exp = 2.5; g.kperp_ratio = 1e-3; g.rho = 1.0; g.gamma = 2.0; g.cp = 0.5;
    const double ratio = atof(argv[4]);
    const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    double* T = malloc(N * sizeof(double));
    double* b = malloc(3 * N * sizeof(double));
    if (!T || !b || !rd(argv[5], T, N) || !rd(argv[6], b, 3 * N)) return 11;
    rkl_options o = {RKL_FP64, -1, 0, RKL_RKL2};
    rkl_plan_t p = NULL;
    if (rkl_plan(&g, 1, &o, &p) != RKL_OK) { fprintf(stderr, "%s\n", rkl_last_error()); return 12; }
    double *dT = NULL, *db = NULL;
    if (hipMalloc((void**)&dT, N * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&db, 3 * N * sizeof(double)) != hipSuccess) return 13;
    if (hipMemcpy(dT, T, N * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(db, b, 3 * N * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return 14;
    double dtp = 0.0;
    if (rkl_dt_par(p, 0, dT, &dtp, NULL) != RKL_OK) { fprintf(stderr, "%s\n", rkl_last_error()); return 15; }
    int32_t s = 0;
    if (rkl_superstep(p, 0, dT, db, ratio * dtp, &s, NULL) != RKL_OK) {
        fprintf(stderr, "%s\n", rkl_last_error());
        return 16;
    }
    if (hipMemcpy(T, dT, N * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return 17;
    uint32_t flags = 99;
    int32_t last_s = 0;
    if (rkl_query(p, 0, &last_s, NULL, &flags) != RKL_OK || last_s != s) return 18;
    FILE* f = fopen(argv[7], "wb");
    if (!f || fwrite(T, sizeof(double), N, f) != N) return 19;
    fclose(f);
    if (rkl_destroy(p) != RKL_OK) return 20;
    (void)hipFree(dT);
    (void)hipFree(db);
    printf("%d %.17g %u\n", s, dtp, flags);
    free(T);
    free(b);
    return 0;
}
'''


def test_c_program_runs_a_superstep(tmp_path):
    from paper_1702_05487_amd import rkl
    libdir = os.path.dirname(rkl.LIB_PATH)
    assert os.path.exists(rkl.LIB_PATH), "librkl.so is not built"
    src = tmp_path / "superstep.c"
    src.write_text(SOURCE)
    exe = tmp_path / "superstep"
    subprocess.check_call(["gcc", "-std=c99", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
                           "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-L", libdir, "-lrkl",
                           "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-Wl,-rpath," + libdir])
    n = (20, 16, 12)
    T = inputs.noisy_temperature(n, 3, kmax=4)
    b = inputs.tangled_b(n, 4, kmax=4)
    np.ascontiguousarray(T, dtype=np.float64).tofile(tmp_path / "T.bin")
    np.ascontiguousarray(b, dtype=np.float64).tofile(tmp_path / "b.bin")
    ratio = inputs.midpoint_ratio(7)
    print("running the C program", flush=True)
    out = subprocess.run([str(exe), *(str(v) for v in n), repr(ratio), str(tmp_path / "T.bin"),
                          str(tmp_path / "b.bin"), str(tmp_path / "out.bin")],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, (out.returncode, out.stderr)
    s, dtp, flags = out.stdout.split()
    got = np.fromfile(tmp_path / "out.bin", dtype=np.float64).reshape(T.shape)
    g = oracle_grid(n, tuple(1.0 / v for v in n), 3, inputs.SPITZER_MC_SAT)
    assert float(dtp) == oracle.dt_par(g, T)
    ref, s_ref, _ = oracle.superstep(g, T, b, ratio * float(dtp))
    print("C program: s %s, dt_par %s, flags %s, rel-L1 %.3e" % (s, dtp, flags, rel_l1(got, ref)))
    assert int(s) == s_ref == 7
    assert int(flags) == 0
    assert rel_l1(got, ref) <= 1e-12
