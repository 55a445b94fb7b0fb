// rkl_kernels.hip -- single-grid kernels of librkl for gfx950: the
// temperature min/max reduction, the finalize step that turns it into
// dt_par, the stage count s and the stage scale (Sec. 3.1 Eq. dt_exp,
// Sec. 3.3 Eq. RKL-s, Sec. 4.1 rounding), and the stencil/stage kernels that
// wrap run_tile (rkl_tile.h).
#include "rkl_stage.h"

namespace rkl {

// ------------------------------------------------------------ variants ----
// (bx, by) are compile-time tile shapes; bz is the z-chunk length per block;
// fuse is the number of stages per launch (F = 2..4: rkl_fused.hip, where
// (bx, by) is the region of a workgroup and (bx-2(F-1), by-2(F-1)) its
// output tile).
static const Variant kVariants[] = {
    {32, 8, 32, 1}, {32, 8, 64, 1}, {64, 4, 32, 1}, {64, 4, 64, 1}, {16, 16, 32, 1}, {16, 16, 64, 1},
    {32, 8, 16, 1}, {64, 4, 16, 1},
    {16, 16, 32, 2}, {16, 16, 64, 2}, {32, 8, 32, 2}, {32, 8, 64, 2},
    {16, 16, 32, 3}, {16, 16, 64, 3}, {16, 16, 32, 4}, {16, 16, 64, 4},
};
int variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
Variant variant_get(int v) { return kVariants[v]; }

// ----------------------------------------------------------- reduction ----
// per-block maximum, minimum and a non-finite flag of T
__global__ __launch_bounds__(256) void reduce_minmax_kernel(const double* __restrict__ T, int64_t N,
                                                            double* __restrict__ part,
                                                            const int32_t* __restrict__ skip) {
    if (skip && *skip) return;   // uniform: the extrema are already there
    double mx = -INFINITY, mn = INFINITY, bad = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
        const double v = T[i];
        mx = fmax(mx, v);
        mn = fmin(mn, v);
        bad = isfinite(v) ? bad : 1.0;
    }
    for (int off = 32; off > 0; off >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, off));
        mn = fmin(mn, __shfl_xor(mn, off));
        bad = fmax(bad, __shfl_xor(bad, off));
    }
    __shared__ double sm[3][4];
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    if (l == 0) { sm[0][w] = mx; sm[1][w] = mn; sm[2][w] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 4; ++i) {
            mx = fmax(mx, sm[0][i]);
            mn = fmin(mn, sm[1][i]);
            bad = fmax(bad, sm[2][i]);
        }
        part[3 * blockIdx.x + 0] = mx;
        part[3 * blockIdx.x + 1] = mn;
        part[3 * blockIdx.x + 2] = bad;
    }
}

int reduce_blocks(int64_t N) {
    int64_t b = (N + 255) / 256;
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_reduce(const double* T, int64_t N, double* partials, int nblocks, hipStream_t st,
                         const int32_t* skip) {
    reduce_minmax_kernel<<<nblocks, 256, 0, st>>>(T, N, partials, skip);
    return hipGetLastError();
}

// mode 0: super-step (computes s); mode 1: flux_div / dt_par only (s = 0).
// Four waves read the partial extrema; every lane of wave 0 then holds the
// grid's extrema and forms the same state; lane 0 stores it and the lanes
// of wave 0 share the rows of the coefficient table (coef_rows, RKL2
// super-steps with 2 <= s <= smax).
constexpr int kFinThreads = 256;
__global__ __launch_bounds__(kFinThreads) void finalize_kernel(const double* __restrict__ part, int nb, GridConst g,
                                                               double dt_hyp, int mode, GridState* st,
                                                               int32_t* s_out, int smax, double* coef_rows,
                                                               const double* __restrict__ ext_part, int ext_nb,
                                                               int32_t* ext_ok) {
    if (ext_ok) {
        const bool use = ext_part && *ext_ok;   // the same in every lane
        if (use) {
            part = ext_part;
            nb = ext_nb;
        }
    }
    double mx = -INFINITY, mn = INFINITY, bad = 0.0;
    for (int i = threadIdx.x; i < nb; i += kFinThreads) {
        mx = fmax(mx, part[3 * i]);
        mn = fmin(mn, part[3 * i + 1]);
        bad = fmax(bad, part[3 * i + 2]);
    }
    for (int off = 32; off > 0; off >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, off));
        mn = fmin(mn, __shfl_xor(mn, off));
        bad = fmax(bad, __shfl_xor(bad, off));
    }
    __shared__ double sm[3][kFinThreads / 64];
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    if (l == 0) {
        sm[0][w] = mx;
        sm[1][w] = mn;
        sm[2][w] = bad;
    }
    __syncthreads();   // also orders every lane's read of *ext_ok before its clearing below
    if (w != 0) return;
    for (int i = 1; i < kFinThreads / 64; ++i) {
        mx = fmax(mx, sm[0][i]);
        mn = fmin(mn, sm[1][i]);
        bad = fmax(bad, sm[2][i]);
    }
    const GridState o = finalize_state(g, mx, mn, bad != 0.0, dt_hyp, mode, smax);
    if (coef_rows && mode == 0 && g.scheme == 0 && o.s >= 2 && o.s <= smax) {
        for (int j = l; j <= o.s; j += 64) {
            double r[5];
            rkl2_row(o.s, j, r);
            for (int i = 0; i < 5; ++i) coef_rows[5 * j + i] = r[i];
        }
    }
    if (l != 0) return;
    *st = o;
    if (s_out) *s_out = o.s;
    if (ext_ok) *ext_ok = 0;
}

hipError_t launch_finalize(const double* partials, int nblocks, const GridConst& gc, double dt_hyp,
                           int mode, GridState* state, int32_t* s_out, int smax, hipStream_t st,
                           double* coef_rows, const double* ext_part, int ext_nb, int32_t* ext_ok) {
    finalize_kernel<<<1, kFinThreads, 0, st>>>(partials, nblocks, gc, dt_hyp, mode, state, s_out, smax, coef_rows,
                                               ext_part, ext_nb, ext_ok);
    return hipGetLastError();
}

// -------------------------------------------------------- stage kernels ----
// (instantiated in the rkl_stage_*.hip units)
template <typename R>
static hipError_t launch_prec(const StageLaunch& P, int nblocks, int bx, int by, bool lim, int sat,
                              hipStream_t st) {
    // grids with fixed axes: one runtime-shaped 16 x 16 kernel with the ghost loads
    if (P.t.fixed) return bx == 16 && by == 16 ? launch_fixed<R>(P, nblocks, lim, sat, st)
                                               : hipErrorInvalidValue;
    if (bx == 32 && by == 8) return launch_shape<R, 32, 8>(P, nblocks, lim, sat, st);
    if (bx == 64 && by == 4) return launch_shape<R, 64, 4>(P, nblocks, lim, sat, st);
    if (bx == 16 && by == 16) return launch_shape<R, 16, 16>(P, nblocks, lim, sat, st);
    return hipErrorInvalidValue;
}

int64_t stage_blocks(Variant v, const GridConst& gc) {
    if (gc.fixed) v = Variant{16, 16, v.bz, 1};
    return (int64_t)((gc.n0 + v.bx - 1) / v.bx) * ((gc.n1 + v.by - 1) / v.by) * ((gc.n2 + v.bz - 1) / v.bz);
}

hipError_t launch_stage(int precision, Variant v, const GridConst& gc, int kind, int stage,
                        const double* Yin, const double* Ym2, const double* Y0, const void* MY0in,
                        void* MY0out, double* Yout, const void* b, const GridState* state,
                        const double* coef, hipStream_t st, double sub_scale, const Route* route,
                        const ExtOut* ext) {
    if (gc.fixed) v = Variant{16, 16, v.bz, 1};   // the tile shape of the ghost-loading kernel
    StageLaunch P;
    TileArgs& a = P.t;
    a.Yin = Yin;
    a.Ym2 = Ym2;
    a.Y0 = Y0;
    a.MY0in = MY0in;
    a.MY0out = MY0out;
    a.Yout = Yout;
    a.b = b;
    a.n0 = gc.n0;
    a.n1 = gc.n1;
    a.n2 = gc.n2;
    a.ndim = gc.ndim;
    a.x0 = a.y0 = a.z0 = a.z1 = 0;
    a.bx = v.bx;
    a.by = v.by;
    a.kind = kind;
    a.bc = gc.bc;
    a.fixed = gc.fixed;
    for (int i = 0; i < 6; ++i) a.gh[i] = gc.gh[i];
    a.ih0 = gc.ih0;
    a.ih1 = gc.ih1;
    a.ih2 = gc.ih2;
    a.scale = 0.0;
    a.mu = a.nu = a.omn = a.mut = a.gt = 0.0;
    a.ext = 0;
    P.ntx = (gc.n0 + v.bx - 1) / v.bx;
    P.nty = (gc.n1 + v.by - 1) / v.by;
    P.bz = v.bz;
    const int nzc = (gc.n2 + v.bz - 1) / v.bz;
    P.state = state;
    P.coef = coef;
    P.stage = stage;
    P.kappa0 = gc.kappa0;
    P.kexp = gc.kexp;
    P.kperp = gc.kperp;
    P.satq = gc.satq;
    P.kmode = gc.kmode;
    P.fac = gc.fac;
    P.sub_scale = sub_scale;
    P.route = Route{nullptr, nullptr, 0, 0};
    P.ext = ExtOut{nullptr, nullptr};
    if (ext) {
        // the last-stage extrema: routed RKL2 stages of 3-D grids without fixed axes
        if (!route || kind != 2 || gc.ndim != 3 || gc.fixed || !ext->part || !ext->ok) return hipErrorInvalidValue;
        P.ext = *ext;
    }
    if (route) {
        // routed stages: Yout carries the caller's T to the kernel
        if ((kind != 1 && kind != 2) || !route->A || !route->B || !Yout) return hipErrorInvalidValue;
        P.route = *route;
        a.Yin = Yout;
        a.Ym2 = Yout;
        a.Y0 = Yout;
    }
    const int64_t nb = (int64_t)P.ntx * P.nty * nzc;
    if (nb <= 0 || nb > 0x7fffffff) return hipErrorInvalidValue;
    const bool lim = gc.limiter != 0;
    const int sat = gc.saturation;
    if (precision == RKL_MIXED) return launch_prec<float>(P, (int)nb, v.bx, v.by, lim, sat, st);
    return launch_prec<double>(P, (int)nb, v.bx, v.by, lim, sat, st);
}

}  // namespace rkl
