// rkl_fused.hip -- the two-stage (temporally fused) RKL2 kernel of librkl
// for gfx950: stages j and j+1 of Appendix A in one launch over overlapped
// tiles (run_fused2, rkl_fused.h).  Flux arithmetic in FP32 on offset
// temperatures, stage recurrence in FP64 (RKL_MIXED plans), 3-D grids.
#include "rkl_internal.h"
#include "rkl_fused.h"

namespace rkl {

struct FusedLaunch {
    FusedArgs f;         // everything but the tile origin, z range and coefficients
    int ntx, nty, bz;
    const GridState* state;
    const double* coef;  // RKL2 table: 5 doubles per (s, j), row of s at s(s+1)/2
    int stage;           // j, the first stage of the pair
    double kappa0, kexp, kperp, satq;
    int kmode;
};

template <bool LIM, int SAT, int KM, int BX, int BY>
__global__ __launch_bounds__(BX* BY) void fused2_kernel(FusedLaunch P) {
    __shared__ FusedLds<float, BX, BY> L;
    int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int tile_x = bid % P.ntx;
    bid /= P.ntx;
    const int tile_y = bid % P.nty;
    const int zc = bid / P.nty;

    FusedArgs a = P.f;
    a.x0 = tile_x * (BX - 2);
    a.y0 = tile_y * (BY - 2);
    a.z0 = zc * P.bz;
    a.z1 = min(a.z0 + P.bz, a.n2);

    const GridState* st = P.state;
    const double tref = st->tref;
    const int s = st->s;
    const double* c1 = P.coef + 5 * ((size_t)s * (s + 1) / 2 + P.stage);
    const double* c2 = c1 + 5;
    a.mu1 = c1[0]; a.nu1 = c1[1]; a.omn1 = c1[2]; a.mut1 = c1[3]; a.gt1 = c1[4];
    a.mu2 = c2[0]; a.nu2 = c2[1]; a.omn2 = c2[2]; a.mut2 = c2[3]; a.gt2 = c2[4];
    a.scale = -st->cdiv;
    const FaceK<float> fk = make_facek<float>(P.kappa0, P.kexp, P.kperp, P.satq, tref);
    run_fused2<float, LIM, SAT, KM, BX, BY>(a, fk, tref, L);
}

template <bool LIM, int KM, int BX, int BY>
static void fused_sat(const FusedLaunch& P, int nblocks, int sat, hipStream_t st) {
    if (sat == 2) fused2_kernel<LIM, 2, KM, BX, BY><<<nblocks, BX * BY, 0, st>>>(P);
    else if (sat == 1) fused2_kernel<LIM, 1, KM, BX, BY><<<nblocks, BX * BY, 0, st>>>(P);
    else fused2_kernel<LIM, 0, KM, BX, BY><<<nblocks, BX * BY, 0, st>>>(P);
}

template <int KM, int BX, int BY>
static void fused_km(const FusedLaunch& P, int nblocks, bool lim, int sat, hipStream_t st) {
    if (lim) fused_sat<true, KM, BX, BY>(P, nblocks, sat, st);
    else fused_sat<false, KM, BX, BY>(P, nblocks, sat, st);
}

template <int BX, int BY>
static hipError_t fused_shape(const FusedLaunch& P, int nblocks, bool lim, int sat, hipStream_t st) {
    if (P.kmode == 0) fused_km<0, BX, BY>(P, nblocks, lim, sat, st);
    else if (P.kmode == 1) fused_km<1, BX, BY>(P, nblocks, lim, sat, st);
    else fused_km<2, BX, BY>(P, nblocks, lim, sat, st);
    return hipGetLastError();
}

hipError_t launch_fused2(Variant v, const GridConst& gc, int stage, const double* Yin, const double* Ym2,
                         const double* Y0, const void* MY0, double* Yj, double* Yj1, const void* b,
                         const GridState* state, const double* coef, hipStream_t st) {
    if (v.fuse != 2 || gc.ndim != 3 || stage < 2 || v.bz < 1) return hipErrorInvalidValue;
    FusedLaunch P;
    FusedArgs& a = P.f;
    a.Yin = Yin;
    a.Ym2 = Ym2;
    a.Y0 = Y0;
    a.MY0 = MY0;
    a.b = b;
    a.Yj = Yj;
    a.Yj1 = Yj1;
    a.n0 = gc.n0;
    a.n1 = gc.n1;
    a.n2 = gc.n2;
    a.ndim = gc.ndim;
    a.x0 = a.y0 = a.z0 = a.z1 = 0;
    a.ih0 = gc.ih0;
    a.ih1 = gc.ih1;
    a.ih2 = gc.ih2;
    a.scale = 0.0;
    a.mu1 = a.nu1 = a.omn1 = a.mut1 = a.gt1 = 0.0;
    a.mu2 = a.nu2 = a.omn2 = a.mut2 = a.gt2 = 0.0;
    P.ntx = (gc.n0 + v.bx - 3) / (v.bx - 2);
    P.nty = (gc.n1 + v.by - 3) / (v.by - 2);
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
    if (v.bx == 16 && v.by == 16) return fused_shape<16, 16>(P, (int)nb, lim, sat, st);
    if (v.bx == 32 && v.by == 8) return fused_shape<32, 8>(P, (int)nb, lim, sat, st);
    return hipErrorInvalidValue;
}

}  // namespace rkl
