// rkl_internal.h -- declarations shared by librkl's own translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rkl {

// Device-resident per-grid state, written by the finalize step of every
// super-step / flux_div / dt_par call and read by the stage kernels.
struct GridState {
    double dt_par;   // explicit parabolic step (Eq. dt_exp), +inf if no conduction
    double tau;      // super-step length
    double cdiv;     // tau * (gamma-1)/rho
    double tref;     // reference temperature subtracted before FP32 flux arithmetic
    double tmax, tmin;
    int32_t s;       // RKL2 stage count (0 when not a super-step)
    uint32_t flags;  // RKL_FLAG_* bits
};

// Per-grid constants (host-computed in FP64 from the descriptor).
struct GridConst {
    int n0, n1, n2, ndim;
    double ih0, ih1, ih2;   // 1/h
    double kappa0, kexp, kperp, satq;  // satq = 5 phi rho
    int kmode;              // 0: kappa0, 1: kappa0 T^2.5, 2: kappa0 T^kexp
    int limiter, saturation;
    int scheme;             // 0 RKL2, 1 RKL1
    int bc;                 // bit d set: axis d is outflow or fixed (indices clamp), else periodic
    double fac;             // (gamma-1)/rho
    double cp, ihsum;       // Courant number, sum_d 1/h_d^2 over active axes
    int fixed;              // bit d set: axis d is fixed (Dirichlet ghost layers gh[2d], gh[2d+1])
    const double* gh[6];    // ghost layers (caller's device arrays), low and high edge per axis
};

// kappa_par at a temperature, FP64, with the operation order of the scalar
// definition kappa0 * (T*T*sqrt(T)) so that dt_par is reproducible
__device__ inline double kappa_at(const GridConst& g, double T) {
    const double t = T > 0.0 ? T : 0.0;
    if (g.kmode == 0) return g.kappa0;
    if (g.kmode == 1) return g.kappa0 * (t * t * sqrt(t));
    return g.kappa0 * pow(t, g.kexp);
}

// Turn the temperature maximum/minimum of a grid into its state: dt_par of
// Eq. dt_exp with chi = kappa_par (gamma-1)/rho (kappa_par is non-decreasing
// in T, so its maximum over cells is kappa_par(max T)) and, for a super-step
// (mode 0), the stage count of Eq. RKL-s -- dt_hyp = dt_par (s^2+s-2)/4 for
// RKL2, dt_par (s^2+s)/2 for RKL1 -- with its root rounded up as
// 1 + floor(s).  flag bits as in rkl.h.
__device__ inline GridState finalize_state(const GridConst& g, double mx, double mn, bool bad,
                                           double dt_hyp, int mode, int smax) {
#pragma clang fp contract(off)
    uint32_t flags = 0;
    if (bad) flags |= 2u;          // RKL_FLAG_NONFINITE
    if (mn <= 0.0) flags |= 1u;    // RKL_FLAG_NONPOS
    const double lam = g.fac * kappa_at(g, mx) * g.ihsum;
    const double dtp = lam > 0.0 ? g.cp / lam : INFINITY;
    int32_t s = 0;
    if (mode == 0) {
        const double r = isinf(dtp) ? 0.0 : dt_hyp / dtp;
        const double sr = g.scheme == 1 ? (-1.0 + sqrt(1.0 + 8.0 * r)) / 2.0
                                        : (-1.0 + sqrt(9.0 + 16.0 * r)) / 2.0;
        const double sf = floor(sr);
        s = (sf >= 0.0 && sf < 1e9) ? 1 + (int32_t)sf : 0x7fffffff;
        if (s > smax) flags |= 4u; // RKL_FLAG_STAGES
    }
    GridState o;
    o.dt_par = dtp;
    o.tau = dt_hyp;
    o.cdiv = dt_hyp * g.fac;
    o.tref = 0.5 * (mx + mn);
    if (!isfinite(o.tref)) o.tref = 0.0;
    o.tmax = mx;
    o.tmin = mn;
    o.s = s;
    o.flags = flags;
    return o;
}

// Row j (0 <= j <= s) of the RKL2 coefficient table of an s-stage super-step
// (Appendix A): w1 = 4/(s^2+s-2), b_j = (j^2+j-2)/(2j(j+1)) (b_0 = b_1 =
// b_2 = 1/3), a_j = 1 - b_j; row 1 holds mut_1 = b_1 w1 in r[3]; rows
// j >= 2 hold {mu_j, nu_j, 1 - mu_j - nu_j, mut_j, gt_j} with
// mu_j = (2j-1)/j b_j/b_{j-1}, nu_j = -(j-1)/j b_j/b_{j-2}, mut_j = mu_j w1,
// gt_j = -a_{j-1} mut_j; row 0 is zero.  The host table of a plan and the
// device rows of the allocation-free super-step both come from here
// (IEEE operations, no contraction), so they hold the same bits.
__host__ __device__ inline double rkl2_bj(int j) {
#pragma clang fp contract(off)
    return j <= 2 ? 1.0 / 3.0 : ((double)j * j + j - 2.0) / (2.0 * j * (j + 1.0));
}
__host__ __device__ inline void rkl2_row(int s, int j, double* r) {
#pragma clang fp contract(off)
    for (int i = 0; i < 5; ++i) r[i] = 0.0;
    const double w1 = 4.0 / ((double)s * s + s - 2.0);
    if (j == 1) {
        r[3] = rkl2_bj(1) * w1;
    } else if (j >= 2) {
        const double bj = rkl2_bj(j), bj1 = rkl2_bj(j - 1), bj2 = rkl2_bj(j - 2);
        const double mu = (2.0 * j - 1.0) / j * bj / bj1;
        const double nu = -(j - 1.0) / j * bj / bj2;
        const double mut = mu * w1;
        r[0] = mu;
        r[1] = nu;
        r[2] = 1.0 - mu - nu;
        r[3] = mut;
        r[4] = -(1.0 - bj1) * mut;
    }
}

// Kernel variants of the single-grid stencil: tile shape, z-chunk length and
// stages per launch (1, or 2 for the fused kernel).
struct Variant {
    int bx, by, bz, fuse;
};
int variant_count();
Variant variant_get(int v);

// Launchers (enqueue only; return the HIP error of the launch).
// skip (may be NULL): when *skip is nonzero on the device the launch does
// nothing (the extrema come from the previous super-step's last stage).
hipError_t launch_reduce(const double* T, int64_t N, double* partials, int nblocks, hipStream_t st,
                         const int32_t* skip = nullptr);
int reduce_blocks(int64_t N);
// coef_rows (may be NULL): for a super-step (mode 0, RKL2) whose stage count
// s is in [2, smax], rows 0..s of its coefficient table (rkl2_row, 5 doubles
// each; room for smax + 1 rows) are written there on the device.
// ext_ok (may be NULL): when *ext_ok is nonzero on the device and ext_part
// is given, the extrema are taken from ext_part (ext_nb per-workgroup
// triples written by the last stage of the previous super-step) instead of
// `partials`; *ext_ok is cleared either way.
hipError_t launch_finalize(const double* partials, int nblocks, const GridConst& gc, double dt_hyp,
                           int mode, GridState* state, int32_t* s_out, int smax, hipStream_t st,
                           double* coef_rows = nullptr, const double* ext_part = nullptr, int ext_nb = 0,
                           int32_t* ext_ok = nullptr);
// Device-side routing of an RKL2 stage (for launch sequences that do not
// know s on the host): with s the grid's device-side stage count, stage j
// does nothing when j > s or s is outside [2, s_cap]; otherwise it reads
// Y_{j-1} and Y_{j-2} from, and writes Y_j to, T (Y_0 and Y_s), A (odd j)
// or B (even j).  coef_flat: the coefficient rows of the current s start at
// `coef` (row j at 5 j) instead of the table of all s (row of s at
// 5 s(s+1)/2).
struct Route {
    double* A;
    double* B;
    int s_cap;
    int coef_flat;
};
// Extrema of the last stage (routed sequences, 3-D grids without fixed axes):
// the launch of stage j = s writes, per workgroup, the maximum, the minimum
// and a non-finite flag of the Y_s it stores to part[3 w .. 3 w + 2] (w the
// workgroup index) and sets *ok = 1, for the next super-step's finalize
// (the dt_par bound and T_ref of Sec. 3.1 Eq. dt_exp need only these).
struct ExtOut {
    double* part;
    int32_t* ok;
};
// workgroups of a one-stage launch of variant v on grid gc
int64_t stage_blocks(Variant v, const GridConst& gc);
// kind: 0 flux divergence into Yout, 1 first stage, 2 stage j >= 2,
// 3 explicit sub-step Yout = Yin + tau L(Yin) with sub_scale = -tau (gamma-1)/rho.
// With `route` set (kinds 1 and 2), Yin, Ym2 and Yout are chosen on the
// device as described above and the ones passed are ignored.
hipError_t launch_stage(int precision, Variant v, const GridConst& gc, int kind, int stage,
                        const double* Yin, const double* Ym2, const double* Y0, const void* MY0in,
                        void* MY0out, double* Yout, const void* b, const GridState* state,
                        const double* coef, hipStream_t st, double sub_scale = 0.0,
                        const Route* route = nullptr, const ExtOut* ext = nullptr);
// stages j..j+F-1 (F = v.fuse in 2..4, 2 <= j, j+F-1 < s) in one launch,
// RKL_MIXED and periodic 3-D grids only; Ya receives Y_{j+F-2}, Yb Y_{j+F-1};
// they must alias none of Yin, Ym2, Y0
hipError_t launch_fused(Variant v, const GridConst& gc, int stage, const double* Yin, const double* Ym2,
                        const double* Y0, const void* MY0, double* Ya, double* Yb, const void* b,
                        const GridState* state, const double* coef, hipStream_t st);

}  // namespace rkl
