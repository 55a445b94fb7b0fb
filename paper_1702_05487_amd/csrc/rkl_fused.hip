// rkl_fused.hip -- the temporally fused RKL2 kernels of librkl for gfx950:
// F = 2, 3 or 4 consecutive stages of Appendix A in one launch over
// overlapped tiles (run_fused, rkl_fused.h).  Flux arithmetic in FP32 on
// offset temperatures, stage recurrence in FP64 (RKL_MIXED plans), periodic
// 3-D grids.
#include "rkl_internal.h"
#include "rkl_fused.h"

namespace rkl {

struct FusedLaunch {
    FusedArgs f;         // everything but the tile origin, z range and coefficients
    int ntx, nty, bz;
    const GridState* state;
    const double* coef;  // RKL2 table: 5 doubles per (s, j), row of s at s(s+1)/2
    int stage;           // j, the first stage of the group
    double kappa0, kexp, kperp, satq;
    int kmode;
};

template <bool LIM, int SAT, int KM, int BX, int BY, int F>
__global__ __launch_bounds__(BX* BY) void fused_kernel(FusedLaunch P) {
    __shared__ FusedLds<float, BX, BY, F> L;
    int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int tile_x = bid % P.ntx;
    bid /= P.ntx;
    const int tile_y = bid % P.nty;
    const int zc = bid / P.nty;

    FusedArgs a = P.f;
    a.x0 = tile_x * (BX - 2 * (F - 1));
    a.y0 = tile_y * (BY - 2 * (F - 1));
    a.z0 = zc * P.bz;
    a.z1 = min(a.z0 + P.bz, a.n2);

    const GridState* st = P.state;
    const double tref = st->tref;
    const int s = st->s;
    const double* c = P.coef + 5 * ((size_t)s * (s + 1) / 2 + P.stage);
#pragma unroll
    for (int l = 0; l < F; ++l)
#pragma unroll
        for (int i = 0; i < 5; ++i) a.cf[l][i] = c[5 * l + i];
    a.scale = -st->cdiv;
    const FaceK<float> fk = make_facek<float>(P.kappa0, P.kexp, P.kperp, P.satq, tref);
    run_fused<float, LIM, SAT, KM, BX, BY, F>(a, fk, tref, L);
}

template <bool LIM, int KM, int BX, int BY, int F>
static void fused_sat(const FusedLaunch& P, int nblocks, int sat, hipStream_t st) {
    if (sat == 2) fused_kernel<LIM, 2, KM, BX, BY, F><<<nblocks, BX * BY, 0, st>>>(P);
    else if (sat == 1) fused_kernel<LIM, 1, KM, BX, BY, F><<<nblocks, BX * BY, 0, st>>>(P);
    else fused_kernel<LIM, 0, KM, BX, BY, F><<<nblocks, BX * BY, 0, st>>>(P);
}

template <int KM, int BX, int BY, int F>
static void fused_km(const FusedLaunch& P, int nblocks, bool lim, int sat, hipStream_t st) {
    if (lim) fused_sat<true, KM, BX, BY, F>(P, nblocks, sat, st);
    else fused_sat<false, KM, BX, BY, F>(P, nblocks, sat, st);
}

template <int BX, int BY, int F>
static hipError_t fused_shape(const FusedLaunch& P, int nblocks, bool lim, int sat, hipStream_t st) {
    if (P.kmode == 0) fused_km<0, BX, BY, F>(P, nblocks, lim, sat, st);
    else if (P.kmode == 1) fused_km<1, BX, BY, F>(P, nblocks, lim, sat, st);
    else fused_km<2, BX, BY, F>(P, nblocks, lim, sat, st);
    return hipGetLastError();
}

hipError_t launch_fused(Variant v, const GridConst& gc, int stage, const double* Yin, const double* Ym2,
                        const double* Y0, const void* MY0, double* Ya, double* Yb, const void* b,
                        const GridState* state, const double* coef, hipStream_t st) {
    const int F = v.fuse;
    if (F < 2 || F > kMaxFuse || gc.ndim != 3 || stage < 2 || v.bz < 1) return hipErrorInvalidValue;
    const int ox = v.bx - 2 * (F - 1), oy = v.by - 2 * (F - 1);   // output tile
    if (ox < 1 || oy < 1) return hipErrorInvalidValue;
    FusedLaunch P;
    FusedArgs& a = P.f;
    a.Yin = Yin;
    a.Ym2 = Ym2;
    a.Y0 = Y0;
    a.MY0 = MY0;
    a.b = b;
    a.Ya = Ya;
    a.Yb = Yb;
    a.n0 = gc.n0;
    a.n1 = gc.n1;
    a.n2 = gc.n2;
    a.ndim = gc.ndim;
    a.x0 = a.y0 = a.z0 = a.z1 = 0;
    a.ih0 = gc.ih0;
    a.ih1 = gc.ih1;
    a.ih2 = gc.ih2;
    a.scale = 0.0;
    for (int l = 0; l < kMaxFuse; ++l)
        for (int i = 0; i < 5; ++i) a.cf[l][i] = 0.0;
    P.ntx = (gc.n0 + ox - 1) / ox;
    P.nty = (gc.n1 + oy - 1) / oy;
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
    const int64_t nb = (int64_t)P.ntx * P.nty * nzc;
    if (nb <= 0 || nb > 0x7fffffff) return hipErrorInvalidValue;
    const bool lim = gc.limiter != 0;
    const int sat = gc.saturation;
    if (v.bx == 16 && v.by == 16 && F == 2) return fused_shape<16, 16, 2>(P, (int)nb, lim, sat, st);
    if (v.bx == 32 && v.by == 8 && F == 2) return fused_shape<32, 8, 2>(P, (int)nb, lim, sat, st);
    if (v.bx == 16 && v.by == 16 && F == 3) return fused_shape<16, 16, 3>(P, (int)nb, lim, sat, st);
    if (v.bx == 16 && v.by == 16 && F == 4) return fused_shape<16, 16, 4>(P, (int)nb, lim, sat, st);
    return hipErrorInvalidValue;
}

}  // namespace rkl
