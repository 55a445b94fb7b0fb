// rkl_stage.h -- the one-stage stencil kernel of librkl (gfx950): one RKL2
// stage (or flux divergence, or explicit sub-step) over every tile of one
// grid, wrapping run_tile (rkl_tile.h).  Private to librkl; the kernel
// sources instantiate it for their tile shapes.
#pragma once
#include "rkl_internal.h"
#include "rkl_tile.h"
#include "../../include/rkl.h"

namespace rkl {

struct StageLaunch {
    TileArgs t;          // everything but the tile origin, z range and coefficients
    int ntx, nty, bz;
    const GridState* state;
    const double* coef;  // RKL2 table: 5 doubles per (s, j), row of s at s(s+1)/2
    int stage;
    double kappa0, kexp, kperp, satq;
    int kmode;
    double fac;
    double sub_scale;    // kind 3: -tau_sub (gamma-1)/rho
    Route route;         // route.A != NULL: Yin, Ym2, Yout chosen on the device (kinds 1, 2)
    ExtOut ext;          // ext.part != NULL: the launch of stage j = s keeps the extrema of Y_s
};

// MODE 1: 3-D grid, tile shape fixed at compile time (run_tile's CBX, CBY);
// MODE 0: runtime tile shape; MODE 2: runtime tile shape with the ghost
// layers of fixed axes
template <typename R, bool LIM, int SAT, int KM, int BX, int BY, int MODE>
__global__ __launch_bounds__(BX* BY) void stage_kernel(StageLaunch P) {
    constexpr int PL = (BX + 2) * (BY + 2);
    __shared__ TileLds<R, PL, (BX + 1) * BY, BX*(BY + 1)> L;
    int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int tile_x = bid % P.ntx;
    bid /= P.ntx;
    const int tile_y = bid % P.nty;
    const int zc = bid / P.nty;

    TileArgs a = P.t;
    a.bx = BX;
    a.by = BY;
    a.x0 = tile_x * BX;
    a.y0 = tile_y * BY;
    a.z0 = zc * P.bz;
    a.z1 = min(a.z0 + P.bz, a.n2);

    const GridState* st = P.state;
    double tref = 0.0;
    if (sizeof(R) == 4) tref = st->tref;
    if (a.kind == 0) {
        a.scale = -P.fac;
    } else if (a.kind == 3) {
        a.scale = P.sub_scale;
    } else {
        const int s = st->s;
        if (P.route.A) {
            // the stage sequence was launched up to s_cap without knowing s
            if (P.stage > s || s < 2 || s > P.route.s_cap) return;   // uniform over the grid
            const int j = P.stage;
            double* T = a.Yout;   // the caller's T (Y_0, and Y_s)
            double* Yj = (j & 1) ? P.route.A : P.route.B;
            if (j == 1) {
                a.Yin = T;
            } else {
                a.Yin = ((j - 1) & 1) ? P.route.A : P.route.B;
                a.Ym2 = j == 2 ? T : Yj;   // Y_{j-2} sits where Y_j goes
            }
            a.Yout = j == s ? T : Yj;
            a.ext = MODE == 1 && P.ext.part && j == s;
        }
        const double* cf = P.coef + 5 * (P.route.coef_flat ? (size_t)P.stage : (size_t)s * (s + 1) / 2 + P.stage);
        a.mu = cf[0];
        a.nu = cf[1];
        a.omn = cf[2];
        a.mut = cf[3];
        a.gt = cf[4];
        a.scale = -st->cdiv;
    }
    const FaceK<R> fk = make_facek<R>(P.kappa0, P.kexp, P.kperp, P.satq, tref);
    if constexpr (MODE == 1) {
        const TileExt e =
            run_tile<R, LIM, SAT, KM, PL, (BX + 1) * BY, BX*(BY + 1), BX, BY, false, 6, true>(a, fk, tref, L);
        if (a.ext) {   // uniform: the last stage of a routed sequence
            // the workgroup's extrema of Y_s, as one block of the reduction pass
            double mx = e.mx, mn = e.mn, bad = e.bad;
            for (int off = 32; off > 0; off >>= 1) {
                mx = fmax(mx, __shfl_xor(mx, off));
                mn = fmin(mn, __shfl_xor(mn, off));
                bad = fmax(bad, __shfl_xor(bad, off));
            }
            constexpr int NW = BX * BY / 64;
            __shared__ double esm[3][NW];
            const int w = threadIdx.x / 64, l = threadIdx.x % 64;
            if (l == 0) {
                esm[0][w] = mx;
                esm[1][w] = mn;
                esm[2][w] = bad;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                for (int i = 1; i < NW; ++i) {
                    mx = fmax(mx, esm[0][i]);
                    mn = fmin(mn, esm[1][i]);
                    bad = fmax(bad, esm[2][i]);
                }
                double* o = P.ext.part + 3 * (size_t)blockIdx.x;
                o[0] = mx;
                o[1] = mn;
                o[2] = bad;
                if (blockIdx.x == 0) *P.ext.ok = 1;   // read after this launch ends
            }
        }
    } else if constexpr (MODE == 2)
        run_tile<R, LIM, SAT, KM, PL, (BX + 1) * BY, BX*(BY + 1), 0, 0, true>(a, fk, tref, L);
    else
        run_tile<R, LIM, SAT, KM>(a, fk, tref, L);
}

// Launch helpers: the kernel of one tile shape, chosen by saturation form,
// limiter and conductivity law.
template <typename R, bool LIM, int KM, int BX, int BY, int MODE>
static void launch_sat(const StageLaunch& P, int nblocks, int sat, hipStream_t st) {
    if (sat == 2) stage_kernel<R, LIM, 2, KM, BX, BY, MODE><<<nblocks, BX * BY, 0, st>>>(P);
    else if (sat == 1) stage_kernel<R, LIM, 1, KM, BX, BY, MODE><<<nblocks, BX * BY, 0, st>>>(P);
    else stage_kernel<R, LIM, 0, KM, BX, BY, MODE><<<nblocks, BX * BY, 0, st>>>(P);
}

template <typename R, int KM, int BX, int BY, int MODE>
static void launch_fix(const StageLaunch& P, int nblocks, bool lim, int sat, hipStream_t st) {
    if (lim) launch_sat<R, true, KM, BX, BY, MODE>(P, nblocks, sat, st);
    else launch_sat<R, false, KM, BX, BY, MODE>(P, nblocks, sat, st);
}

template <typename R, int BX, int BY, int MODE>
static hipError_t launch_law(const StageLaunch& P, int nblocks, bool lim, int sat, hipStream_t st) {
    if (P.kmode == 0) launch_fix<R, 0, BX, BY, MODE>(P, nblocks, lim, sat, st);
    else if (P.kmode == 1) launch_fix<R, 1, BX, BY, MODE>(P, nblocks, lim, sat, st);
    else launch_fix<R, 2, BX, BY, MODE>(P, nblocks, lim, sat, st);
    return hipGetLastError();
}

// The kernels of one tile shape: compile-time shape for 3-D grids, runtime
// shape for 1-D and 2-D ones.  Instantiated once per precision and shape in
// the rkl_stage_*.hip units, which compile in parallel.
template <typename R, int BX, int BY>
hipError_t launch_shape(const StageLaunch& P, int nblocks, bool lim, int sat, hipStream_t st) {
    if (P.t.ndim == 3) return launch_law<R, BX, BY, 1>(P, nblocks, lim, sat, st);
    return launch_law<R, BX, BY, 0>(P, nblocks, lim, sat, st);
}

// grids with fixed axes: the runtime-shaped 16 x 16 kernel with the ghost loads
template <typename R>
hipError_t launch_fixed(const StageLaunch& P, int nblocks, bool lim, int sat, hipStream_t st) {
    return launch_law<R, 16, 16, 2>(P, nblocks, lim, sat, st);
}

#define RKL_SHAPE_ARGS const StageLaunch&, int, bool, int, hipStream_t
extern template hipError_t launch_shape<float, 32, 8>(RKL_SHAPE_ARGS);
extern template hipError_t launch_shape<float, 64, 4>(RKL_SHAPE_ARGS);
extern template hipError_t launch_shape<float, 16, 16>(RKL_SHAPE_ARGS);
extern template hipError_t launch_shape<double, 32, 8>(RKL_SHAPE_ARGS);
extern template hipError_t launch_shape<double, 64, 4>(RKL_SHAPE_ARGS);
extern template hipError_t launch_shape<double, 16, 16>(RKL_SHAPE_ARGS);
extern template hipError_t launch_fixed<float>(RKL_SHAPE_ARGS);
extern template hipError_t launch_fixed<double>(RKL_SHAPE_ARGS);

}  // namespace rkl
