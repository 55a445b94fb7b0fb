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
// F_c is the face flux of Sec. 2 (Eqs. Fc, Fclass, Fsat plus the
// perpendicular term) with the transverse gradients of Appendix B.
//
// Layout: fields are [n2][n1][n0] (axis 0 fastest); b is 3 such arrays.
// Scheme: a workgroup owns a bx x by column tile and marches along z.  Three
// z planes of the stencil input (with a one-cell x/y halo, periodic wrap) sit
// in an LDS ring; per-cell slopes and b of the current and next plane sit in
// a two-plane LDS ring.  Every face flux is computed exactly once: each cell
// computes its +x, +y and +z faces, the tile's -x and -y boundary faces are
// extra jobs, x/y faces are exchanged through LDS and the +z face is carried
// in a register to the next plane.  Flux arithmetic runs in R (double, or
// float on temperatures offset by a reference value); the stage recurrence
// always runs in double.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rkl {

// ---------------------------------------------------------------- math ----
__device__ __forceinline__ float r_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double r_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float r_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double r_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float r_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double r_div(double a, double b) { return a / b; }
__device__ __forceinline__ float r_pow(float x, float y) { return powf(x, y); }
__device__ __forceinline__ double r_pow(double x, double y) { return pow(x, y); }

// monotonized-central limiter: minmod(2a, 2b, (a+b)/2)
template <typename R>
__device__ __forceinline__ R mc(R a, R b) {
    const R m = fmin(fabs(a + b) * R(0.5), R(2) * fmin(fabs(a), fabs(b)));
    return (a * b > R(0)) ? copysign(m, a) : R(0);
}

// cell slope along one axis from the two one-sided differences: MC-limited,
// or their mean (so that the mean of two cell slopes is the mean of the four
// one-sided differences of Appendix B)
template <typename R, bool LIM>
__device__ __forceinline__ R cell_slope(R tm, R t0, R tp, R ih) {
    const R am = (t0 - tm) * ih, ap = (tp - t0) * ih;
    return LIM ? mc(am, ap) : R(0.5) * (am + ap);
}

// per-grid constants of the face flux, in the flux precision
template <typename R>
struct FaceK {
    R kappa0, kexp, kperp, satq;  // satq = 5 phi rho
    R tref;                       // added back to offset temperatures
    int kmode;                    // 0: kappa0, 1: kappa0 T^2.5, 2: kappa0 T^kexp
};

// Normal component of F_c through a face, for cells L (low) and R (high)
// along the face normal.  s?1, s?2: the cells' slopes along the two
// transverse axes; b?n/b?1/b?2: the cells' unit vectors (normal, transverse
// 1, transverse 2 components).
template <typename R, bool LIM, bool SAT>
__device__ __forceinline__ R face_flux(R TL, R TR, R ihn, R sL1, R sR1, R sL2, R sR2,
                                       R bLn, R bL1, R bL2, R bRn, R bR1, R bR2,
                                       const FaceK<R>& k) {
    const R Gn = (TR - TL) * ihn;
    const R G1 = LIM ? mc(sL1, sR1) : R(0.5) * (sL1 + sR1);
    const R G2 = LIM ? mc(sL2, sR2) : R(0.5) * (sL2 + sR2);
    R Tf = R(0.5) * (TL + TR) + k.tref;
    Tf = Tf > R(0) ? Tf : R(0);
    const R sq = (SAT || k.kmode == 1) ? r_sqrt(Tf) : R(0);
    const R kpar = k.kmode == 0 ? k.kappa0
                 : (k.kmode == 1 ? k.kappa0 * (Tf * Tf * sq) : k.kappa0 * r_pow(Tf, k.kexp));
    const R kperp = k.kperp * kpar;
    R cn = bLn + bRn, c1 = bL1 + bR1, c2 = bL2 + bR2;
    const R nb2 = cn * cn + c1 * c1 + c2 * c2;
    const R inv = nb2 < R(1e-24) ? R(0) : r_rsqrt(nb2);
    cn *= inv;
    c1 *= inv;
    c2 *= inv;
    const R bG = cn * Gn + c1 * G1 + c2 * G2;
    const R dk = kpar - kperp;
    R Fn = -(kperp * Gn + dk * cn * bG);
    if (SAT) {
        const R F1 = -(kperp * G1 + dk * c1 * bG);
        const R F2 = -(kperp * G2 + dk * c2 * bG);
        const R Fm = r_sqrt(Fn * Fn + F1 * F1 + F2 * F2);
        const R q = k.satq * (Tf * sq);
        Fn = q > R(0) ? r_div(q, q + Fm) * Fn : R(0);
    }
    return Fn;
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
    int bx, by;          // tile shape (bx*by <= threads)
    int kind;
    double ih0, ih1, ih2;
    double scale;        // multiplies div F: -(gamma-1)/rho (kind 0) or -tau (gamma-1)/rho
    double mu, nu, omn, mut, gt;
};

template <typename R, int PLMAX, int FXMAX, int FYMAX>
struct TileLds {
    R T[3][PLMAX];      // ring of three input planes (halo 1)
    R S[2][3][PLMAX];   // slopes of two planes
    R B[2][3][PLMAX];   // unit vectors of two planes
    R FX[FXMAX];        // x-face fluxes, [by][bx+1]
    R FY[FYMAX];        // y-face fluxes, [by+1][bx]
};

__device__ __forceinline__ int wrap(int i, int n) {
    int m = i % n;
    return m < 0 ? m + n : m;
}

template <typename R>
__device__ __forceinline__ R to_r(double v, double tref) {
    return R(v - tref);
}

template <typename R, bool LIM, bool SAT, int PLMAX, int FXMAX, int FYMAX>
__device__ __forceinline__ void run_tile(const TileArgs& a, const FaceK<R>& fk, double tref,
                                         TileLds<R, PLMAX, FXMAX, FYMAX>& L) {
    const int tid = threadIdx.x;
    const int bx = a.bx, by = a.by, px = bx + 2;
    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const size_t plane = (size_t)n0 * (size_t)n1;
    const size_t N = plane * (size_t)n2;
    const R* bR = (const R*)a.b;
    const R ih0 = R(a.ih0), ih1 = R(a.ih1), ih2 = R(a.ih2);
    const bool do_y = a.ndim >= 2, do_z = a.ndim >= 3;

    // own cell of this thread
    const bool own = tid < bx * by;
    const int tx = own ? tid % bx : 0, ty = own ? tid / bx : 0;
    const int oslot = (ty + 1) * px + tx + 1;
    const int oxy = wrap(a.y0 + ty, n1) * n0 + wrap(a.x0 + tx, n0);
    const bool store = own && (a.x0 + tx < n0) && (a.y0 + ty < n1);

    // halo cell whose temperature this thread loads (corners included)
    const bool hjob = tid < 2 * px + 2 * by;
    int hslot = 0, hxy = 0;
    if (hjob) {
        int hi, hj;
        if (tid < px) { hi = tid - 1; hj = -1; }
        else if (tid < 2 * px) { hi = tid - px - 1; hj = by; }
        else if (tid < 2 * px + by) { hi = -1; hj = tid - 2 * px; }
        else { hi = bx; hj = tid - 2 * px - by; }
        hslot = (hj + 1) * px + hi + 1;
        hxy = wrap(a.y0 + hj, n1) * n0 + wrap(a.x0 + hi, n0);
    }
    // halo cell whose slopes and b this thread provides (edges, no corners):
    // y-halo cells need the x and z slopes, x-halo cells the y and z slopes
    const bool djob = tid < 2 * bx + 2 * by;
    int dslot = 0, dxy = 0;
    bool dxh = false;
    if (djob) {
        int hi, hj;
        if (tid < bx) { hi = tid; hj = -1; }
        else if (tid < 2 * bx) { hi = tid - bx; hj = by; }
        else if (tid < 2 * bx + by) { hi = -1; hj = tid - 2 * bx; dxh = true; }
        else { hi = bx; hj = tid - 2 * bx - by; dxh = true; }
        dslot = (hj + 1) * px + hi + 1;
        dxy = wrap(a.y0 + hj, n1) * n0 + wrap(a.x0 + hi, n0);
    }
    // extra face: the tile's -x face of row j (tid < by) or -y face of column i
    const bool fjob = tid < by + (do_y ? bx : 0);
    int fdir = 0, fL = 0, fR = 0, fidx = 0;
    if (fjob) {
        if (tid < by) { fdir = 0; fL = (tid + 1) * px; fR = fL + 1; fidx = tid * (bx + 1); }
        else { const int i = tid - by; fdir = 1; fL = i + 1; fR = px + i + 1; fidx = i; }
    }

    auto plane_base = [&](int p) -> size_t { return (size_t)wrap(p, n2) * plane; };

    // pipeline state
    double pTo = 0.0, pTh = 0.0;            // prefetched T(k+2): own, halo
    R pbo0 = 0, pbo1 = 0, pbo2 = 0;         // prefetched b(k+1): own
    R pbd0 = 0, pbd1 = 0, pbd2 = 0;         // prefetched b(k+1): halo
    double yq0 = 0.0, yq1 = 0.0, yq2 = 0.0; // own FP64 input: planes k, k+1, k+2
    R ob00 = 0, ob01 = 0, ob02 = 0;         // own b, plane k
    R ob10 = 0, ob11 = 0, ob12 = 0;         // own b, plane k+1
    R os00 = 0, os01 = 0, os10 = 0, os11 = 0;  // own x/y slopes, planes k and k+1
    R fzp = 0;                               // +z face flux of plane k-1

    const int z0 = a.z0, z1 = a.z1;
    // ring slots: T(k) c0, T(k+1) c1, T(k+2) c2; slopes/b of plane k in dc, of k+1 in dn
    int c0 = 0, c1 = 1, c2 = 2, dc = 1, dn = 0;
    {
        const size_t pb0 = plane_base(z0 - 2), pb1 = plane_base(z0 - 1), pb2 = plane_base(z0);
        if (own) {
            yq1 = a.Yin[pb0 + oxy];
            yq2 = a.Yin[pb1 + oxy];
            L.T[0][oslot] = to_r<R>(yq1, tref);
            L.T[1][oslot] = to_r<R>(yq2, tref);
            pTo = a.Yin[pb2 + oxy];
            pbo0 = bR[pb1 + oxy];
            pbo1 = bR[N + pb1 + oxy];
            pbo2 = bR[2 * N + pb1 + oxy];
        }
        if (hjob) {
            L.T[0][hslot] = to_r<R>(a.Yin[pb0 + hxy], tref);
            L.T[1][hslot] = to_r<R>(a.Yin[pb1 + hxy], tref);
            pTh = a.Yin[pb2 + hxy];
        }
        if (djob) {
            pbd0 = bR[pb1 + dxy];
            pbd1 = bR[N + pb1 + dxy];
            pbd2 = bR[2 * N + pb1 + dxy];
        }
    }

    for (int k = z0 - 2; k < z1; ++k) {
        // ---- A: T(k+2) into the ring, b(k+1) into the b ring; prefetch the next plane
        if (own) {
            L.T[c2][oslot] = to_r<R>(pTo, tref);
            yq0 = yq1; yq1 = yq2; yq2 = pTo;
            L.B[dn][0][oslot] = pbo0; L.B[dn][1][oslot] = pbo1; L.B[dn][2][oslot] = pbo2;
            ob00 = ob10; ob01 = ob11; ob02 = ob12;
            ob10 = pbo0; ob11 = pbo1; ob12 = pbo2;
        }
        if (hjob) L.T[c2][hslot] = to_r<R>(pTh, tref);
        if (djob) { L.B[dn][0][dslot] = pbd0; L.B[dn][1][dslot] = pbd1; L.B[dn][2][dslot] = pbd2; }
        if (k + 1 < z1) {
            const size_t pt = plane_base(k + 3), pb = plane_base(k + 2);
            if (own) {
                pTo = a.Yin[pt + oxy];
                pbo0 = bR[pb + oxy]; pbo1 = bR[N + pb + oxy]; pbo2 = bR[2 * N + pb + oxy];
            }
            if (hjob) pTh = a.Yin[pt + hxy];
            if (djob) { pbd0 = bR[pb + dxy]; pbd1 = bR[N + pb + dxy]; pbd2 = bR[2 * N + pb + dxy]; }
        }
        double ym2 = 0.0, y0v = 0.0, my0 = 0.0;
        if (k >= z0 && own && a.kind == 2) {
            const size_t o = (size_t)k * plane + oxy;
            ym2 = a.Ym2[o];
            y0v = a.Y0[o];
            my0 = (double)((const R*)a.MY0in)[o];
        }
        __syncthreads();

        // ---- B: slopes of plane k+1 (needs T(k), T(k+1), T(k+2))
        if (own) {
            const R t0 = L.T[c1][oslot];
            const R s0 = cell_slope<R, LIM>(L.T[c1][oslot - 1], t0, L.T[c1][oslot + 1], ih0);
            const R s1 = cell_slope<R, LIM>(L.T[c1][oslot - px], t0, L.T[c1][oslot + px], ih1);
            const R s2 = cell_slope<R, LIM>(L.T[c0][oslot], t0, L.T[c2][oslot], ih2);
            L.S[dn][0][oslot] = s0; L.S[dn][1][oslot] = s1; L.S[dn][2][oslot] = s2;
            os00 = os10; os01 = os11; os10 = s0; os11 = s1;
        }
        if (djob) {
            const R t0 = L.T[c1][dslot];
            if (dxh) L.S[dn][1][dslot] = cell_slope<R, LIM>(L.T[c1][dslot - px], t0, L.T[c1][dslot + px], ih1);
            else     L.S[dn][0][dslot] = cell_slope<R, LIM>(L.T[c1][dslot - 1], t0, L.T[c1][dslot + 1], ih0);
            L.S[dn][2][dslot] = cell_slope<R, LIM>(L.T[c0][dslot], t0, L.T[c2][dslot], ih2);
        }
        __syncthreads();

        // ---- C: faces of plane k
        R fzn = 0;
        if (k >= z0) {
            const R* Tk = L.T[c0];
            const R(*S)[PLMAX] = L.S[dc];
            const R(*Bv)[PLMAX] = L.B[dc];
            if (own) {
                const int r = oslot + 1;
                L.FX[ty * (bx + 1) + tx + 1] = face_flux<R, LIM, SAT>(
                    Tk[oslot], Tk[r], ih0, S[1][oslot], S[1][r], S[2][oslot], S[2][r],
                    Bv[0][oslot], Bv[1][oslot], Bv[2][oslot], Bv[0][r], Bv[1][r], Bv[2][r], fk);
                if (do_y) {
                    const int u = oslot + px;
                    L.FY[(ty + 1) * bx + tx] = face_flux<R, LIM, SAT>(
                        Tk[oslot], Tk[u], ih1, S[0][oslot], S[0][u], S[2][oslot], S[2][u],
                        Bv[1][oslot], Bv[0][oslot], Bv[2][oslot], Bv[1][u], Bv[0][u], Bv[2][u], fk);
                }
            }
            if (fjob) {
                // direction-generic gather so that the wave runs one face evaluation
                const int t1 = fdir == 0 ? 1 : 0;
                const R f = face_flux<R, LIM, SAT>(
                    Tk[fL], Tk[fR], fdir == 0 ? ih0 : ih1, S[t1][fL], S[t1][fR], S[2][fL], S[2][fR],
                    Bv[fdir][fL], Bv[t1][fL], Bv[2][fL], Bv[fdir][fR], Bv[t1][fR], Bv[2][fR], fk);
                if (fdir == 0) L.FX[fidx] = f; else L.FY[fidx] = f;
            }
        }
        if (do_z && own && k >= z0 - 1) {
            fzn = face_flux<R, LIM, SAT>(L.T[c0][oslot], L.T[c1][oslot], ih2, os00, os10, os01, os11,
                                         ob02, ob00, ob01, ob12, ob10, ob11, fk);
        }
        __syncthreads();

        // ---- D: divergence and the stage update of plane k
        if (k >= z0 && store) {
            const int fx = ty * (bx + 1) + tx;
            R div = (L.FX[fx + 1] - L.FX[fx]) * ih0;
            if (do_y) div += (L.FY[(ty + 1) * bx + tx] - L.FY[ty * bx + tx]) * ih1;
            if (do_z) div += (fzn - fzp) * ih2;
            const size_t o = (size_t)k * plane + oxy;
            const double tl = a.scale * (double)div;
            if (a.kind == 0) {
                a.Yout[o] = tl;
            } else if (a.kind == 1) {
                const R m = R(tl);
                ((R*)a.MY0out)[o] = m;
                a.Yout[o] = yq0 + a.mut * (double)m;
            } else {
                a.Yout[o] = a.mu * yq0 + a.nu * ym2 + a.omn * y0v + a.mut * tl + a.gt * my0;
            }
        }
        fzp = fzn;
        const int t = c0; c0 = c1; c1 = c2; c2 = t;
        const int d = dc; dc = dn; dn = d;
    }
}

}  // namespace rkl
