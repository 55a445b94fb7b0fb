// rkl_tile.h -- device code of the conduction stencil and the RKL2 stage
// update (gfx950).  Private to librkl; included by the kernel sources only.
//
// Method: Vaidya et al. (2017), arXiv:1702.05487.  One call of run_tile
// advances one (x, y) tile of one grid over a range of z planes through one
// operation:
//   kind 0  out = (gamma-1)/rho * (-div F_c(Y))                      (Sec. 3)
//   kind 1  MY0 = tau M(Y0),  Y1 = Y0 + mut_1 MY0          (Appendix A, stage 1)
//   kind 2  Y_j = mu Y_{j-1} + nu Y_{j-2} + (1-mu-nu) Y0 + mut tau M(Y_{j-1})
//                 + gt MY0                                 (Appendix A, stage j)
//   kind 3  out = Y + tau (gamma-1)/rho (-div F_c(Y))     (one explicit sub-step)
// F_c is the face flux of Sec. 2 (Eqs. Fc, Fclass, Fsat plus the
// perpendicular term) with the transverse gradients of Appendix B.
//
// Layout: fields are [n2][n1][n0] (axis 0 fastest); b is 3 such arrays.
// Scheme: a workgroup owns a bx x by column tile and marches along z.  Three
// z planes of the stencil input (with a one-cell x/y halo: wrapped on
// periodic axes, the edge cell repeated on outflow axes) sit in an LDS ring;
// per-cell slopes and b of the current and next plane sit in a two-plane LDS
// ring.  Every face flux is computed exactly once: each cell
// computes its +x, +y and +z faces, the tile's -x and -y boundary faces are
// extra jobs, x/y faces are exchanged through (double-buffered) LDS and the
// +z face is carried in a register to the next plane.  Each thread keeps the
// three input planes of its own column (and of its halo cell), and its own
// slopes and unit vectors, in registers, so the z-slopes need no LDS, the
// low side of its faces comes from registers, and one barrier per plane
// suffices.  Flux arithmetic runs in R (double, or float on temperatures
// offset by a reference value); the stage recurrence always runs in double.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

// No automatic contraction of a*b+c: every fused multiply-add below is
// written out, so each tile shape, kernel variant and the batched kernels
// (different instantiations of the same code) round identically.
#pragma clang fp contract(off)

namespace rkl {

// ---------------------------------------------------------------- math ----
// FP32: the hardware square root / reciprocal / reciprocal square root.
// FP64: the hardware estimate y (relative error ~2^-23) corrected once to
// third order: with e = 1 - x y^2, 1/sqrt(x) = y (1 + e/2 + 3e^2/8 + O(e^3));
// with e = 1 - x y, 1/x = y (1 + e + e^2 + O(e^3)); the dropped terms are
// ~2^-66, below the rounding level.  sqrt(x) = x / sqrt(x).
__device__ __forceinline__ float r_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float r_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double r_rsqrt(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-(x * y), y, 1.0);
    return fma(y, e * fma(e, 0.375, 0.5), y);
}
// x >= 0: x times the corrected reciprocal root, whose argument is kept at or
// above 1e-300 so that the estimate stays finite and normal (exactly 0 for
// x = 0; only x < 1e-300 differs from the square root, by less than 1e-150)
__device__ __forceinline__ double r_sqrt(double x) { return x * r_rsqrt(fmax(x, 1e-300)); }
__device__ __forceinline__ float r_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double r_rcp(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, y, 1.0);
    return fma(y, fma(e, e, e), y);
}
__device__ __forceinline__ float r_pow(float x, float y) { return powf(x, y); }
__device__ __forceinline__ double r_pow(double x, double y) { return pow(x, y); }

// median of three
__device__ __forceinline__ float med3(float a, float b, float c) { return __builtin_amdgcn_fmed3f(a, b, c); }
__device__ __forceinline__ double med3(double a, double b, double c) {
    return fmax(fmin(a, b), fmin(fmax(a, b), c));
}

// Monotonized-central limiter, MC(a, b) = minmod(2a, 2b, (a+b)/2).  With
// minmod(a, b) = med3(a, b, 0) and minmod associative and positively
// homogeneous, MC(a, b) = minmod(2 minmod(a, b), (a+b)/2)
// = (1/2) med3(4 med3(a, b, 0), a + b, 0).  mc2 returns 2 MC(a, b).
template <typename R>
__device__ __forceinline__ R mc2(R a, R b) {
    return med3(R(4) * med3(a, b, R(0)), a + b, R(0));
}
// FP64 has no median instruction: where m = minmod(a, b) is not zero, a + b
// has its sign, so the outer median is that sign times min(4|m|, |a+b|);
// where m is zero, so is that product.  Same values, one emulated median.
__device__ __forceinline__ double mc2(double a, double b) {
    const double m = med3(a, b, 0.0);
    return copysign(fmin(4.0 * fabs(m), fabs(a + b)), m);
}

// Half the cell slope along one axis, from the one-sided differences
// (t0-tm)/h and (tp-t0)/h: MC-limited, or their mean (so that the mean of two
// cell slopes is the mean of the four one-sided differences of Appendix B).
// hq = 1/(4h).  The slope is stored halved so that the face's transverse
// gradient below, MC or mean of the two cells' slopes, needs no halving:
// MC and the sum are positively homogeneous and halving is exact, so the
// result has the same bits as halving at the face.
template <typename R, bool LIM>
__device__ __forceinline__ R cell_slope(R tm, R t0, R tp, R hq) {
    if (LIM) return hq * mc2(t0 - tm, tp - t0);
    return hq * (tp - tm);
}

// transverse gradient at a face from the (halved) slopes of its two cells
template <typename R, bool LIM>
__device__ __forceinline__ R face_transverse(R sL, R sR) {
    return LIM ? mc2(sL, sR) : sL + sR;
}

// per-grid constants of the face flux, in the flux precision
template <typename R>
struct FaceK {
    R kappa0, kexp;
    R r, omr;       // kappa_perp / kappa_par and 1 - r
    R r2, omr2;     // r^2 and 1 - r^2
    R satq;         // 5 phi rho
    R tref;         // added back to offset temperatures
};

template <typename R>
__device__ __forceinline__ FaceK<R> make_facek(double kappa0, double kexp, double kperp_ratio, double satq,
                                              double tref) {
    FaceK<R> k;
    k.kappa0 = R(kappa0);
    k.kexp = R(kexp);
    k.r = R(kperp_ratio);
    k.omr = R(1.0 - kperp_ratio);
    k.r2 = R(kperp_ratio * kperp_ratio);
    k.omr2 = R(1.0 - kperp_ratio * kperp_ratio);
    k.satq = R(satq);
    k.tref = R(tref);
    return k;
}

// Normal component of F_c through a face, for cells L (low) and R (high)
// along the face normal.  SAT: 0 classical flux, 1 saturated blend with q at
// the face temperature, 2 the same with q at the temperature of the upwind
// cell, the one the classical flux -kappa_par A leaves (L when A < 0).  s?1, s?2: the cells' slopes along the two
// transverse axes; b?n/b?1/b?2: the cells' unit vectors (normal, transverse
// 1, transverse 2 components).  KM: conductivity law, 0 kappa0, 1 kappa0
// T^2.5, 2 kappa0 T^kexp.
//
// With c = b_L + b_R the face direction is c/|c| (0 if |c| < 1e-12), so
// b_n (b.G) = c_n w and (b.G)^2 = (c.G) w with w = (c.G)/|c|^2.  With
// kappa_perp = r kappa_par the classical flux is
//   F = -kappa_par [r G + (1-r) b (b.G)],   F_n = -kappa_par A,
//   A = r G_n + (1-r) c_n w,
//   |F| = kappa_par B,   B^2 = r^2 |G|^2 + (1-r^2) (b.G)^2,
// and the saturated blend q F/(q + |F|) is -kappa_par A q / (q + kappa_par B).
// kappa_par = kappa0 T^2.5 is evaluated as kappa0 T (T^2/sqrt(T)) and the
// saturated flux 5 phi rho T^1.5 as satq T^2/sqrt(T) with the same T^1.5
// (one reciprocal root; T is clipped at 1e-30 instead of 0 so that the root
// stays finite, which changes kappa and q by less than 1e-75).
template <typename R, bool LIM, int SAT, int KM>
__device__ __forceinline__ R face_flux(R TL, R TR, R ihn, R sL1, R sR1, R sL2, R sR2,
                                       R bLn, R bL1, R bL2, R bRn, R bR1, R bR2,
                                       const FaceK<R>& k) {
    const R Gn = (TR - TL) * ihn;
    const R G1 = face_transverse<R, LIM>(sL1, sR1);
    const R G2 = face_transverse<R, LIM>(sL2, sR2);
    const R Tf = fmax(fma(R(0.5), TL + TR, k.tref), R(1e-30));
    const R t15 = (SAT == 1 || KM == 1) ? (Tf * Tf) * r_rsqrt(Tf) : R(0);   // T^1.5
    const R kpar = KM == 0 ? k.kappa0 : (KM == 1 ? k.kappa0 * (t15 * Tf) : k.kappa0 * r_pow(Tf, k.kexp));
    const R cn = bLn + bRn, c1 = bL1 + bR1, c2 = bL2 + bR2;
    const R cc = fma(cn, cn, fma(c1, c1, c2 * c2));
    const R cG = fma(cn, Gn, fma(c1, G1, c2 * G2));
    const R w = cc < R(1e-24) ? R(0) : cG * r_rcp(cc);     // (b.G)/|c|
    const R A = fma(k.r, Gn, k.omr * (cn * w));
    if (SAT == 0) return -(kpar * A);
    const R GG = fma(Gn, Gn, fma(G1, G1, G2 * G2));
    const R B2 = fma(k.r2, GG, k.omr2 * (cG * w));
    R q;
    if (SAT == 2) {
        const R Tu = fmax((A < R(0) ? TL : TR) + k.tref, R(1e-30));
        q = k.satq * ((Tu * Tu) * r_rsqrt(Tu));
    } else {
        q = k.satq * t15;
    }
    const R den = fma(kpar, r_sqrt(B2), q);    // q + |F|; B2 >= 0: sums of products of non-negative terms
    return den > R(0) ? -(kpar * A) * (q * r_rcp(den)) : R(0);
}

// ------------------------------------------------------------- one tile ----
struct TileArgs {
    const double* Yin;   // stencil input Y_{j-1} (Y0 for kinds 0/1)
    const double* Ym2;   // Y_{j-2} (kind 2)
    const double* Y0;    // Y0 (kind 2)
    const void* MY0in;   // tau M(Y0), type R (kind 2)
    void* MY0out;        // tau M(Y0), type R (kind 1)
    double* Yout;        // output
    const void* b;       // unit vectors, type R, 3 x N
    int n0, n1, n2, ndim;
    int x0, y0, z0, z1;  // tile origin and z range [z0, z1)
    int bx, by;          // tile shape (bx*by <= threads, 2bx+2by+4 <= threads)
    int kind;
    int bc;              // bit d set: axis d is outflow or fixed (indices clamp), else periodic
    int fixed;           // bit d set: axis d is fixed; temperatures beyond its edges from gh[2d], gh[2d+1]
    const double* gh[6]; // ghost layers of the fixed axes (runtime-shaped tiles only)
    double ih0, ih1, ih2;
    double scale;        // multiplies div F: -(gamma-1)/rho (kind 0) or -tau (gamma-1)/rho
    double mu, nu, omn, mut, gt;
    int ext;             // kind 2, compile-time tile shapes: keep the extrema of the stored output
};

// per-thread maximum, minimum and non-finite flag (0 or 1) of the stored
// stage output (TileArgs::ext)
struct TileExt {
    double mx, mn, bad;
};

template <typename R, int PLMAX, int FXMAX, int FYMAX>
struct TileLds {
    R T[3][PLMAX];      // ring of three input planes (halo 1)
    R S[2][3][PLMAX];   // slopes of two planes
    R B[2][3][PLMAX];   // unit vectors of two planes
    R FX[2][FXMAX];     // x-face fluxes, [by][bx+1], double-buffered by plane parity
    R FY[2][FYMAX];     // y-face fluxes, [by+1][bx]
};

// Workgroups are dispatched round-robin over the 8 XCDs; renumber them so that
// consecutive logical tiles (which share halo lines) land on the same XCD and
// its L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb / 8, r = nb % 8;
    const int xcd = b % 8, slot = b / 8;
    return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

__device__ __forceinline__ int wrap(int i, int n) {
    int m = i % n;
    return m < 0 ? m + n : m;
}

// index of cell i along an axis of n cells: wrapped (periodic axis) or
// clamped to the edge cell (outflow axis: the cells beyond an edge repeat it)
__device__ __forceinline__ int bidx(int i, int n, bool open) {
    return open ? min(max(i, 0), n - 1) : wrap(i, n);
}

// ---------------------------------------------- fixed (Dirichlet) axes ----
// A column of the tile beyond an x or y edge of a fixed axis reads its
// temperatures from that axis's ghost layer (the lower axis first); a column
// inside reads the field, and the ghost layer of a fixed z axis beyond the z
// edges.  Layer of axis d: (n_b + 2) x (n_a + 2) values, a < b the other
// axes, transverse index j at j + 1, wrapped on a periodic axis, clamped to
// [0, n-1] on an outflow one and to [-1, n] on a fixed one.
struct GhostCol {
    const double* lp;    // layer column: plane k at lp[(k' + 1) * ls], k' the mapped z index
    int ls;
    const double* zlo;   // field column: the fixed z axis's ghost values below and above
    const double* zhi;
};

__device__ __forceinline__ int gmap(int i, int n, bool clamp, bool fixed) {
    if (!clamp) return wrap(i, n);
    return fixed ? min(max(i, -1), n) : min(max(i, 0), n - 1);
}

__device__ inline GhostCol ghost_col(int bc, int fixed, const double* const* gh, int n0, int n1, int gi, int gj) {
    GhostCol c{nullptr, 0, nullptr, nullptr};
    const bool cx = bc & 1, cy = bc & 2, fx = fixed & 1, fy = fixed & 2;
    // constant indices only (a computed index would put the array in scratch)
    if (fx && (gi < 0 || gi >= n0)) {
        c.lp = (gi < 0 ? gh[0] : gh[1]) + (gmap(gj, n1, cy, fy) + 1);
        c.ls = n1 + 2;
    } else if (fy && (gj < 0 || gj >= n1)) {
        c.lp = (gj < 0 ? gh[2] : gh[3]) + (gmap(gi, n0, cx, fx) + 1);
        c.ls = n0 + 2;
    } else if (fixed & 4) {
        const int off = (gmap(gj, n1, cy, fy) + 1) * (n0 + 2) + gmap(gi, n0, cx, fx) + 1;
        c.zlo = gh[4] + off;
        c.zhi = gh[5] + off;
    }
    return c;
}

// temperature of column c (field index xy) at plane k, any k
__device__ inline double ghost_T(const GhostCol& c, const double* Y, int k, int n2, bool cz, bool fz, int xy,
                                 size_t plane) {
    if (c.lp) return c.lp[(size_t)(gmap(k, n2, cz, fz) + 1) * c.ls];
    if (fz && k < 0) return *c.zlo;
    if (fz && k >= n2) return *c.zhi;
    return Y[(size_t)bidx(k, n2, cz) * plane + xy];
}

template <typename R>
__device__ __forceinline__ R to_r(double v, double tref) {
    return R(v - tref);
}

// the RKL2 stage recurrence, Appendix A:
// mu Y_{j-1} + nu Y_{j-2} + (1-mu-nu) Y0 + mut tau M(Y_{j-1}) + gt tau M(Y0)
__device__ __forceinline__ double stage_combine(double mu, double nu, double omn, double mut, double gt,
                                                double ym1, double ym2, double y0, double tl, double my0) {
    return fma(gt, my0, fma(mut, tl, fma(omn, y0, fma(nu, ym2, mu * ym1))));
}

// CBX, CBY > 0: the tile shape is a compile-time constant, the grid is 3-D
// and the workgroup has exactly CBX*CBY threads (one cell each); the tile
// strides are then constants and the face code has no runtime branches.
// GH: the ghost-layer loads of fixed axes (runtime shapes only).
// UNR: the plane loop unrolled six-fold (6) or not (1); see the register
// rings below.  NT: the pointwise stage inputs and the stage output, each
// touched once per launch, bypass the caches' normal retention so that the
// lines that neighbouring tiles share (temperatures, unit vectors) stay.
// Neither changes a value.
template <typename R, bool LIM, int SAT, int KM, int PLMAX, int FXMAX, int FYMAX, int CBX = 0, int CBY = 0,
          bool GH = false, int UNR = 1, bool NT = false>
__device__ __forceinline__ TileExt run_tile(const TileArgs& a, const FaceK<R>& fk, double tref,
                                            TileLds<R, PLMAX, FXMAX, FYMAX>& L) {
    constexpr bool FIX = CBX > 0;
    static_assert(!FIX || (2 * CBX + 2 * CBY + 4 <= CBX * CBY && CBX + CBY <= CBX * CBY),
                  "the ring cells and extra faces need one thread each");
    const int tid = threadIdx.x;
    const int bx = FIX ? CBX : a.bx, by = FIX ? CBY : a.by, px = bx + 2;
    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const int plane = n0 * n1;
    const size_t N = (size_t)plane * (size_t)n2;
    const R* b0 = (const R*)a.b;
    const R* b1 = b0 + N;
    const R* b2 = b1 + N;
    const R ih0 = R(a.ih0), ih1 = R(a.ih1), ih2 = R(a.ih2);
    const R hih0 = R(0.25 * a.ih0), hih1 = R(0.25 * a.ih1), hih2 = R(0.25 * a.ih2);   // 1/(4h), see cell_slope
    const bool do_y = FIX || a.ndim >= 2, do_z = FIX || a.ndim >= 3;
    const bool ox = a.bc & 1, oy = a.bc & 2, oz = a.bc & 4;

    // own cell of this thread
    const bool own = FIX || tid < bx * by;
    const int tx = own ? tid % bx : 0, ty = own ? tid / bx : 0;
    const int oslot = (ty + 1) * px + tx + 1;
    const int oxy = bidx(a.y0 + ty, n1, oy) * n0 + bidx(a.x0 + tx, n0, ox);
    const bool store = own && (a.x0 + tx < n0) && (a.y0 + ty < n1);

    // halo cell of this thread: the 2bx+2by edge cells first (y-halo rows,
    // then x-halo columns), then the 4 corners.  An edge thread also provides
    // the slopes and unit vector of its cell (y-halo: x and z slopes; x-halo:
    // y and z slopes); corners only supply temperatures.
    const int ne = 2 * bx + 2 * by;
    const bool hjob = tid < ne + 4;
    const bool djob = tid < ne;
    bool dxh = false;
    int hslot = 0, hxy = 0, hti = 0, htj = 0;
    if (hjob) {
        int hi, hj;
        if (tid < bx) { hi = tid; hj = -1; }
        else if (tid < 2 * bx) { hi = tid - bx; hj = by; }
        else if (tid < 2 * bx + by) { hi = -1; hj = tid - 2 * bx; dxh = true; }
        else if (tid < ne) { hi = bx; hj = tid - 2 * bx - by; dxh = true; }
        else {
            const int c = tid - ne;
            hi = (c & 1) ? bx : -1;
            hj = (c & 2) ? by : -1;
        }
        hslot = (hj + 1) * px + hi + 1;
        hxy = bidx(a.y0 + hj, n1, oy) * n0 + bidx(a.x0 + hi, n0, ox);
        hti = hi;
        htj = hj;
    }
    // extra face: the tile's -x face of row j (f < by) or -y face of column i.
    // These jobs go to the last wave(s) of the workgroup while the halo jobs
    // sit in the first ones, so that no wave carries both (wave w of every
    // workgroup runs on the same SIMD).
    const int nf = by + (do_y ? bx : 0);
    const int fbase = max(0, ((FIX ? CBX * CBY : (int)blockDim.x) - nf) / 64 * 64);
    const int fid = tid - fbase;
    const bool fjob = fid >= 0 && fid < nf;
    int fdir = 0, fL = 0, fR = 0, fidx = 0;
    if (fjob) {
        if (fid < by) { fdir = 0; fL = (fid + 1) * px; fR = fL + 1; fidx = fid * (bx + 1); }
        else { const int i = fid - by; fdir = 1; fL = i + 1; fR = px + i + 1; fidx = i; }
    }

    const int z0 = a.z0, z1 = a.z1;
    // index of plane k + 4, the temperature plane prefetched at plane k
    int pz4 = bidx(z0 + 2, n2, oz);

    // fixed axes: ghost-aware temperature loads of the own and halo columns
    const bool gon = GH && !FIX && a.fixed != 0;
    GhostCol gco{nullptr, 0, nullptr, nullptr}, gch{nullptr, 0, nullptr, nullptr};
    if (gon) {
        gco = ghost_col(a.bc, a.fixed, a.gh, n0, n1, a.x0 + tx, a.y0 + ty);
        if (hjob) {
            gch = ghost_col(a.bc, a.fixed, a.gh, n0, n1, a.x0 + hti, a.y0 + htj);
        }
    }
    const bool fz = a.fixed & 4;
    // T at plane k (raw index), field index xy, through column g where ghosts apply
    auto tld = [&](const double* pp, int k, int xy, const GhostCol& g) -> double {
        return gon ? ghost_T(g, a.Yin, k, n2, oz, fz, xy, (size_t)plane) : pp[xy];
    };

    TileExt ex{-INFINITY, INFINITY, 0.0};
    if constexpr (UNR == 6) {
        const bool ext_on = a.ext != 0;
        // Register rings.  The value for plane k + m sits in slot (P + m) mod L
        // of a ring of length L, P = (k - z0 + 2) mod 6.  The loop is unrolled
        // six-fold (every L divides six) with P a compile-time constant, so each
        // value stays in one register from its load to its last use and no
        // plane-to-plane moves are left.  Loads are two planes ahead, and values
        // stay in their loaded type until they are used, so that no conversion
        // forces an early wait.
        constexpr int LT = 6;          // own FP64 input: planes k .. k+4
        constexpr int LB = 6;          // own unit vector: planes k .. k+3
        double tq[LT];                 // own input Y_{j-1}, FP64
        R oq[3];                       // the same in flux precision: planes k .. k+2
        double th[2];                  // halo cell input, FP64: planes k+2, k+3 (k+4 loaded into the slot of k+2)
        R hq[3];                       // halo cell input in flux precision: planes k .. k+2
        R ob[LB][3];                   // own unit vector
        R pbd[2][3];                   // halo unit vector: planes k+1, k+2 (k+3 loaded into the slot of k+1)
        R os[2][3];                    // own slopes: planes k, k+1
        R zf[2];                       // +z face flux: planes k-1, k
        double qym2[3], qy0[3];        // pointwise stage inputs Y_{j-2}, Y0: planes k .. k+2
        R qmy0[3];                     // tau M(Y0): planes k .. k+2
        for (int r = 0; r < LT; ++r) tq[r] = 0.0;
        for (int r = 0; r < LB; ++r) ob[r][0] = ob[r][1] = ob[r][2] = 0;
        for (int r = 0; r < 3; ++r) {
            oq[r] = hq[r] = 0;
            qym2[r] = qy0[r] = 0.0;
            qmy0[r] = 0;
        }
        for (int r = 0; r < 2; ++r) {
            th[r] = 0.0;
            zf[r] = 0;
            pbd[r][0] = pbd[r][1] = pbd[r][2] = 0;
            os[r][0] = os[r][1] = os[r][2] = 0;
        }
        const bool pw = own && a.kind == 2;

        // prologue (P = 0 at k = z0 - 2): T(z0-2 .. z0+1), b(z0-1), b(z0)
        {
            const double* p0 = a.Yin + (size_t)bidx(z0 - 2, n2, oz) * plane;
            const double* p1 = a.Yin + (size_t)bidx(z0 - 1, n2, oz) * plane;
            const double* p2 = a.Yin + (size_t)bidx(z0, n2, oz) * plane;
            const double* p3 = a.Yin + (size_t)bidx(z0 + 1, n2, oz) * plane;
            const size_t pb0 = (size_t)bidx(z0 - 1, n2, oz) * plane;
            const size_t pb1 = (size_t)bidx(z0, n2, oz) * plane;
            if (own) {
                tq[0] = tld(p0, z0 - 2, oxy, gco);
                tq[1] = tld(p1, z0 - 1, oxy, gco);
                tq[2] = tld(p2, z0, oxy, gco);
                tq[3] = tld(p3, z0 + 1, oxy, gco);
                ob[1][0] = b0[pb0 + oxy]; ob[1][1] = b1[pb0 + oxy]; ob[1][2] = b2[pb0 + oxy];
                ob[2][0] = b0[pb1 + oxy]; ob[2][1] = b1[pb1 + oxy]; ob[2][2] = b2[pb1 + oxy];
            }
            if (hjob) {
                const double h1 = tld(p0, z0 - 2, hxy, gch), h2 = tld(p1, z0 - 1, hxy, gch);
                th[0] = tld(p2, z0, hxy, gch);
                th[1] = tld(p3, z0 + 1, hxy, gch);
                hq[0] = to_r<R>(h1, tref);
                hq[1] = to_r<R>(h2, tref);
                L.T[0][hslot] = hq[0];
                L.T[1][hslot] = hq[1];
            }
            if (djob) {
                pbd[1][0] = b0[pb0 + hxy]; pbd[1][1] = b1[pb0 + hxy]; pbd[1][2] = b2[pb0 + hxy];
                pbd[0][0] = b0[pb1 + hxy]; pbd[0][1] = b1[pb1 + hxy]; pbd[0][2] = b2[pb1 + hxy];
            }
            if (own) {
                oq[0] = to_r<R>(tq[0], tref);
                oq[1] = to_r<R>(tq[1], tref);
                L.T[0][oslot] = oq[0];
                L.T[1][oslot] = oq[1];
            }
        }
        __syncthreads();

        // One plane k with phase P.  LDS rings: temperatures of planes k, k+1,
        // k+2 in slots r0, r1, r2; slopes and unit vectors of plane k+1 in
        // slot d0 and of plane k in d1; face buffers in slot d0.
        auto step = [&](auto ph, int k) __attribute__((always_inline)) {
            constexpr int P = decltype(ph)::value;
            constexpr int r0 = P % 3, r1 = (P + 1) % 3, r2 = (P + 2) % 3;   // 3-rings: planes k, k+1, k+2
            constexpr int d0 = P % 2, d1 = (P + 1) % 2;                     // 2-rings: planes k, k+1
            constexpr int t0 = r0, t1 = r1, t2 = r2, e0 = d0, e1 = d1;
            // ---- A: T(k+2) into the ring, b(k+1) into the b ring
            if (own) {
                oq[r2] = to_r<R>(tq[(P + 2) % LT], tref);
                L.T[t2][oslot] = oq[r2];
                const R* bn = ob[(P + 1) % LB];
                L.B[e0][0][oslot] = bn[0]; L.B[e0][1][oslot] = bn[1]; L.B[e0][2][oslot] = bn[2];
            }
            if (hjob) {
                hq[r2] = to_r<R>(th[d0], tref);
                L.T[t2][hslot] = hq[r2];
            }
            if (djob) { L.B[e0][0][hslot] = pbd[d1][0]; L.B[e0][1][hslot] = pbd[d1][1]; L.B[e0][2][hslot] = pbd[d1][2]; }
            // prefetch two planes ahead: T(k+4) and b(k+3), used at plane k+2
            if (k + 2 < z1) {
                const double* pt = a.Yin + (size_t)pz4 * plane;
                const int pbz = oz ? min(k + 3, n2 - 1) : (pz4 == 0 ? n2 - 1 : pz4 - 1);
                const size_t pb = (size_t)pbz * plane;
                if (own) {
                    tq[(P + 4) % LT] = tld(pt, k + 4, oxy, gco);
                    R* bl = ob[(P + 3) % LB];
                    bl[0] = b0[pb + oxy]; bl[1] = b1[pb + oxy]; bl[2] = b2[pb + oxy];
                }
                if (hjob) th[d0] = tld(pt, k + 4, hxy, gch);
                if (djob) { pbd[d1][0] = b0[pb + hxy]; pbd[d1][1] = b1[pb + hxy]; pbd[d1][2] = b2[pb + hxy]; }
                pz4 = oz ? min(k + 5, n2 - 1) : (pz4 + 1 == n2 ? 0 : pz4 + 1);
            }
            if (pw && k + 2 >= z0 && k + 2 < z1) {
                // read once and not again in this launch: streamed past the caches (NT)
                const size_t o = (size_t)(k + 2) * plane + oxy;
                if constexpr (NT) {
                    qym2[r2] = __builtin_nontemporal_load(a.Ym2 + o);
                    qy0[r2] = __builtin_nontemporal_load(a.Y0 + o);
                    qmy0[r2] = __builtin_nontemporal_load((const R*)a.MY0in + o);
                } else {
                    qym2[r2] = a.Ym2[o];
                    qy0[r2] = a.Y0[o];
                    qmy0[r2] = ((const R*)a.MY0in)[o];
                }
            }

            // ---- B: slopes of plane k+1.  In-plane neighbours of T(k+1) come from
            // the ring (written one plane earlier); z neighbours from registers.
            if (own) {
                const R* T1 = L.T[t1];
                const R s0 = cell_slope<R, LIM>(T1[oslot - 1], oq[r1], T1[oslot + 1], hih0);
                const R s1 = cell_slope<R, LIM>(T1[oslot - px], oq[r1], T1[oslot + px], hih1);
                const R s2 = cell_slope<R, LIM>(oq[r0], oq[r1], oq[r2], hih2);
                L.S[e0][0][oslot] = s0; L.S[e0][1][oslot] = s1; L.S[e0][2][oslot] = s2;
                os[d1][0] = s0; os[d1][1] = s1; os[d1][2] = s2;
            }
            if (djob) {
                const R* T1 = L.T[t1];
                if (dxh) L.S[e0][1][hslot] = cell_slope<R, LIM>(T1[hslot - px], hq[r1], T1[hslot + px], hih1);
                else     L.S[e0][0][hslot] = cell_slope<R, LIM>(T1[hslot - 1], hq[r1], T1[hslot + 1], hih0);
                L.S[e0][2][hslot] = cell_slope<R, LIM>(hq[r0], hq[r1], hq[r2], hih2);
            }

            // ---- C: faces of plane k (inputs written in earlier planes; the low
            // side of the own faces from registers)
            const R* ob0 = ob[P % LB];         // b(k)
            const R* ob1 = ob[(P + 1) % LB];   // b(k+1)
            if (k >= z0) {
                const R* Tk = L.T[t0];
                const R(*S)[PLMAX] = L.S[e1];
                const R(*Bv)[PLMAX] = L.B[e1];
                R* FX = L.FX[e0];
                R* FY = L.FY[e0];
                if (own) {
                    const int r = oslot + 1;
                    FX[ty * (bx + 1) + tx + 1] = face_flux<R, LIM, SAT, KM>(
                        oq[r0], Tk[r], ih0, os[d0][1], S[1][r], os[d0][2], S[2][r],
                        ob0[0], ob0[1], ob0[2], Bv[0][r], Bv[1][r], Bv[2][r], fk);
                    if (do_y) {
                        const int u = oslot + px;
                        FY[(ty + 1) * bx + tx] = face_flux<R, LIM, SAT, KM>(
                            oq[r0], Tk[u], ih1, os[d0][0], S[0][u], os[d0][2], S[2][u],
                            ob0[1], ob0[0], ob0[2], Bv[1][u], Bv[0][u], Bv[2][u], fk);
                    }
                }
                if (fjob) {
                    // direction-generic gather so that the wave runs one face evaluation
                    const int u1 = fdir == 0 ? 1 : 0;
                    const R f = face_flux<R, LIM, SAT, KM>(
                        Tk[fL], Tk[fR], fdir == 0 ? ih0 : ih1, S[u1][fL], S[u1][fR], S[2][fL], S[2][fR],
                        Bv[fdir][fL], Bv[u1][fL], Bv[2][fL], Bv[fdir][fR], Bv[u1][fR], Bv[2][fR], fk);
                    if (fdir == 0) FX[fidx] = f; else FY[fidx] = f;
                }
            }
            zf[d0] = 0;
            if (do_z && own && k >= z0 - 1) {
                zf[d0] = face_flux<R, LIM, SAT, KM>(oq[r0], oq[r1], ih2, os[d0][0], os[d1][0], os[d0][1], os[d1][1],
                                                    ob0[2], ob0[0], ob0[1], ob1[2], ob1[0], ob1[1], fk);
            }
            __syncthreads();

            // ---- D: divergence and the stage update of plane k
            if (k >= z0 && store) {
                const R* FX = L.FX[e0];
                const R* FY = L.FY[e0];
                const int fx = ty * (bx + 1) + tx;
                R div = (FX[fx + 1] - FX[fx]) * ih0;
                if (do_y) div = fma(FY[(ty + 1) * bx + tx] - FY[ty * bx + tx], ih1, div);
                if (do_z) div = fma(zf[d0] - zf[d1], ih2, div);
                const size_t o = (size_t)k * plane + oxy;
                const double tl = a.scale * (double)div;
                const double yk = tq[P % LT];
                if (a.kind == 0) {
                    a.Yout[o] = tl;
                } else if (a.kind == 1) {
                    const R m = R(tl);
                    ((R*)a.MY0out)[o] = m;
                    a.Yout[o] = fma(a.mut, (double)m, yk);
                } else if (a.kind == 3) {
                    a.Yout[o] = yk + tl;
                } else {
                    const double y = stage_combine(a.mu, a.nu, a.omn, a.mut, a.gt, yk, qym2[r0], qy0[r0], tl,
                                                   (double)qmy0[r0]);
                    if constexpr (NT) __builtin_nontemporal_store(y, a.Yout + o);
                    else a.Yout[o] = y;
                    if (ext_on) {
                        // as the reduction pass over T does it
                        ex.mx = fmax(ex.mx, y);
                        ex.mn = fmin(ex.mn, y);
                        ex.bad = isfinite(y) ? ex.bad : 1.0;
                    }
                }
            }
        };
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        using I3 = std::integral_constant<int, 3>;
        using I4 = std::integral_constant<int, 4>;
        using I5 = std::integral_constant<int, 5>;
        int k = z0 - 2;
        for (; k + 5 < z1; k += 6) {
            step(I0{}, k);
            step(I1{}, k + 1);
            step(I2{}, k + 2);
            step(I3{}, k + 3);
            step(I4{}, k + 4);
            step(I5{}, k + 5);
        }
        if (k < z1) step(I0{}, k);
        if (k + 1 < z1) step(I1{}, k + 1);
        if (k + 2 < z1) step(I2{}, k + 2);
        if (k + 3 < z1) step(I3{}, k + 3);
        if (k + 4 < z1) step(I4{}, k + 4);
    } else {
        static_assert(UNR == 1, "the plane loop runs unrolled six-fold or not at all");
        // Prefetch pipeline, two planes deep: set 0 is stored into LDS at this
        // plane's step A, set 1 at the next plane's.  Values stay in their loaded
        // type until they are used, so that no conversion forces an early wait.
        double pTo0 = 0.0, pTo1 = 0.0;            // T(k+2), T(k+3): own cell
        double pTh0 = 0.0, pTh1 = 0.0;            // T(k+2), T(k+3): halo cell
        R pbo00 = 0, pbo01 = 0, pbo02 = 0, pbo10 = 0, pbo11 = 0, pbo12 = 0;   // b(k+1), b(k+2): own
        R pbd00 = 0, pbd01 = 0, pbd02 = 0, pbd10 = 0, pbd11 = 0, pbd12 = 0;   // b(k+1), b(k+2): halo
        double yq0 = 0.0, yq1 = 0.0, yq2 = 0.0;   // own FP64 input, planes k, k+1, k+2
        R oq0 = 0, oq1 = 0, oq2 = 0;              // same in flux precision
        R hq0 = 0, hq1 = 0, hq2 = 0;              // halo cell input, planes k, k+1, k+2
        R ob00 = 0, ob01 = 0, ob02 = 0;           // own b, plane k
        R ob10 = 0, ob11 = 0, ob12 = 0;           // own b, plane k+1
        R os00 = 0, os01 = 0, os02 = 0;           // own slopes, plane k
        R os10 = 0, os11 = 0, os12 = 0;           // own slopes, plane k+1
        R fzp = 0;                                // +z face flux of plane k-1
        // pointwise stage inputs Y_{j-2}, Y0, tau M(Y0): plane k (cur), k+1 (q1),
        // k+2 (q2), loaded two planes ahead
        double ym2 = 0.0, y0v = 0.0;
        R my0 = 0;
        double q1ym2 = 0.0, q1y0 = 0.0, q2ym2 = 0.0, q2y0 = 0.0;
        R q1my0 = 0, q2my0 = 0;
        const bool pw = own && a.kind == 2;

        // ring slots: T(k) c0, T(k+1) c1, T(k+2) c2; slopes/b of plane k in dc, of k+1 in dn
        int c0 = 0, c1 = 1, c2 = 2, dc = 1, dn = 0, fb = 0;
        {
            const double* p0 = a.Yin + (size_t)bidx(z0 - 2, n2, oz) * plane;
            const double* p1 = a.Yin + (size_t)bidx(z0 - 1, n2, oz) * plane;
            const double* p2 = a.Yin + (size_t)bidx(z0, n2, oz) * plane;
            const double* p3 = a.Yin + (size_t)bidx(z0 + 1, n2, oz) * plane;
            const size_t pb0 = (size_t)bidx(z0 - 1, n2, oz) * plane;
            const size_t pb1 = (size_t)bidx(z0, n2, oz) * plane;
            if (own) {
                yq1 = tld(p0, z0 - 2, oxy, gco);
                yq2 = tld(p1, z0 - 1, oxy, gco);
                pTo0 = tld(p2, z0, oxy, gco);
                pTo1 = tld(p3, z0 + 1, oxy, gco);
                pbo00 = b0[pb0 + oxy]; pbo01 = b1[pb0 + oxy]; pbo02 = b2[pb0 + oxy];
                pbo10 = b0[pb1 + oxy]; pbo11 = b1[pb1 + oxy]; pbo12 = b2[pb1 + oxy];
            }
            if (hjob) {
                const double h1 = tld(p0, z0 - 2, hxy, gch), h2 = tld(p1, z0 - 1, hxy, gch);
                pTh0 = tld(p2, z0, hxy, gch);
                pTh1 = tld(p3, z0 + 1, hxy, gch);
                hq1 = to_r<R>(h1, tref);
                hq2 = to_r<R>(h2, tref);
                L.T[0][hslot] = hq1;
                L.T[1][hslot] = hq2;
            }
            if (djob) {
                pbd00 = b0[pb0 + hxy]; pbd01 = b1[pb0 + hxy]; pbd02 = b2[pb0 + hxy];
                pbd10 = b0[pb1 + hxy]; pbd11 = b1[pb1 + hxy]; pbd12 = b2[pb1 + hxy];
            }
            if (own) {
                oq1 = to_r<R>(yq1, tref);
                oq2 = to_r<R>(yq2, tref);
                L.T[0][oslot] = oq1;
                L.T[1][oslot] = oq2;
            }
        }
        __syncthreads();

        for (int k = z0 - 2; k < z1; ++k) {
            // ---- A: T(k+2) into the ring and the register queues, b(k+1) into the b ring
            if (own) {
                yq0 = yq1; yq1 = yq2; yq2 = pTo0;
                oq0 = oq1; oq1 = oq2; oq2 = to_r<R>(pTo0, tref);
                L.T[c2][oslot] = oq2;
                L.B[dn][0][oslot] = pbo00; L.B[dn][1][oslot] = pbo01; L.B[dn][2][oslot] = pbo02;
                ob00 = ob10; ob01 = ob11; ob02 = ob12;
                ob10 = pbo00; ob11 = pbo01; ob12 = pbo02;
            }
            if (hjob) {
                hq0 = hq1; hq1 = hq2; hq2 = to_r<R>(pTh0, tref);
                L.T[c2][hslot] = hq2;
            }
            if (djob) { L.B[dn][0][hslot] = pbd00; L.B[dn][1][hslot] = pbd01; L.B[dn][2][hslot] = pbd02; }
            pTo0 = pTo1; pTh0 = pTh1;
            pbo00 = pbo10; pbo01 = pbo11; pbo02 = pbo12;
            pbd00 = pbd10; pbd01 = pbd11; pbd02 = pbd12;
            // prefetch two planes ahead: T(k+4) and b(k+3), used at plane k+2
            if (k + 2 < z1) {
                const double* pt = a.Yin + (size_t)pz4 * plane;
                const int pbz = oz ? min(k + 3, n2 - 1) : (pz4 == 0 ? n2 - 1 : pz4 - 1);
                const size_t pb = (size_t)pbz * plane;
                if (own) {
                    pTo1 = tld(pt, k + 4, oxy, gco);
                    pbo10 = b0[pb + oxy]; pbo11 = b1[pb + oxy]; pbo12 = b2[pb + oxy];
                }
                if (hjob) pTh1 = tld(pt, k + 4, hxy, gch);
                if (djob) { pbd10 = b0[pb + hxy]; pbd11 = b1[pb + hxy]; pbd12 = b2[pb + hxy]; }
                pz4 = oz ? min(k + 5, n2 - 1) : (pz4 + 1 == n2 ? 0 : pz4 + 1);
            }
            ym2 = q1ym2; y0v = q1y0; my0 = q1my0;
            q1ym2 = q2ym2; q1y0 = q2y0; q1my0 = q2my0;
            if (pw && k + 2 >= z0 && k + 2 < z1) {
                const size_t o = (size_t)(k + 2) * plane + oxy;
                q2ym2 = a.Ym2[o];
                q2y0 = a.Y0[o];
                q2my0 = ((const R*)a.MY0in)[o];
            }

            // ---- B: slopes of plane k+1.  In-plane neighbours of T(k+1) come from
            // the ring (written one plane earlier); z neighbours from registers.
            if (own) {
                const R* T1 = L.T[c1];
                const R s0 = cell_slope<R, LIM>(T1[oslot - 1], oq1, T1[oslot + 1], hih0);
                const R s1 = cell_slope<R, LIM>(T1[oslot - px], oq1, T1[oslot + px], hih1);
                const R s2 = cell_slope<R, LIM>(oq0, oq1, oq2, hih2);
                L.S[dn][0][oslot] = s0; L.S[dn][1][oslot] = s1; L.S[dn][2][oslot] = s2;
                os00 = os10; os01 = os11; os02 = os12;
                os10 = s0; os11 = s1; os12 = s2;
            }
            if (djob) {
                const R* T1 = L.T[c1];
                if (dxh) L.S[dn][1][hslot] = cell_slope<R, LIM>(T1[hslot - px], hq1, T1[hslot + px], hih1);
                else     L.S[dn][0][hslot] = cell_slope<R, LIM>(T1[hslot - 1], hq1, T1[hslot + 1], hih0);
                L.S[dn][2][hslot] = cell_slope<R, LIM>(hq0, hq1, hq2, hih2);
            }

            // ---- C: faces of plane k (inputs written in earlier planes; the low
            // side of the own faces from registers)
            R fzn = 0;
            if (k >= z0) {
                const R* Tk = L.T[c0];
                const R(*S)[PLMAX] = L.S[dc];
                const R(*Bv)[PLMAX] = L.B[dc];
                R* FX = L.FX[fb];
                R* FY = L.FY[fb];
                if (own) {
                    const int r = oslot + 1;
                    FX[ty * (bx + 1) + tx + 1] = face_flux<R, LIM, SAT, KM>(
                        oq0, Tk[r], ih0, os01, S[1][r], os02, S[2][r],
                        ob00, ob01, ob02, Bv[0][r], Bv[1][r], Bv[2][r], fk);
                    if (do_y) {
                        const int u = oslot + px;
                        FY[(ty + 1) * bx + tx] = face_flux<R, LIM, SAT, KM>(
                            oq0, Tk[u], ih1, os00, S[0][u], os02, S[2][u],
                            ob01, ob00, ob02, Bv[1][u], Bv[0][u], Bv[2][u], fk);
                    }
                }
                if (fjob) {
                    // direction-generic gather so that the wave runs one face evaluation
                    const int t1 = fdir == 0 ? 1 : 0;
                    const R f = face_flux<R, LIM, SAT, KM>(
                        Tk[fL], Tk[fR], fdir == 0 ? ih0 : ih1, S[t1][fL], S[t1][fR], S[2][fL], S[2][fR],
                        Bv[fdir][fL], Bv[t1][fL], Bv[2][fL], Bv[fdir][fR], Bv[t1][fR], Bv[2][fR], fk);
                    if (fdir == 0) FX[fidx] = f; else FY[fidx] = f;
                }
            }
            if (do_z && own && k >= z0 - 1) {
                fzn = face_flux<R, LIM, SAT, KM>(oq0, oq1, ih2, os00, os10, os01, os11,
                                                 ob02, ob00, ob01, ob12, ob10, ob11, fk);
            }
            __syncthreads();

            // ---- D: divergence and the stage update of plane k
            if (k >= z0 && store) {
                const R* FX = L.FX[fb];
                const R* FY = L.FY[fb];
                const int fx = ty * (bx + 1) + tx;
                R div = (FX[fx + 1] - FX[fx]) * ih0;
                if (do_y) div = fma(FY[(ty + 1) * bx + tx] - FY[ty * bx + tx], ih1, div);
                if (do_z) div = fma(fzn - fzp, ih2, div);
                const size_t o = (size_t)k * plane + oxy;
                const double tl = a.scale * (double)div;
                if (a.kind == 0) {
                    a.Yout[o] = tl;
                } else if (a.kind == 1) {
                    const R m = R(tl);
                    ((R*)a.MY0out)[o] = m;
                    a.Yout[o] = fma(a.mut, (double)m, yq0);
                } else if (a.kind == 3) {
                    a.Yout[o] = yq0 + tl;
                } else {
                    a.Yout[o] = stage_combine(a.mu, a.nu, a.omn, a.mut, a.gt, yq0, ym2, y0v, tl, (double)my0);
                }
            }
            fzp = fzn;
            const int t = c0; c0 = c1; c1 = c2; c2 = t;
            const int d = dc; dc = dn; dn = d;
            fb ^= 1;
        }
    }
    return ex;
}

}  // namespace rkl
