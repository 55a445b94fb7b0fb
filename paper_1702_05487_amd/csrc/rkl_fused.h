// rkl_fused.h -- two RKL2 stages per launch (temporal fusion) for gfx950.
// Private to librkl; included by the kernel sources only.
//
// Method: Vaidya et al. (2017), arXiv:1702.05487, Appendix A: stages j and
// j+1 (2 <= j, j+1 < s) of
//   Y_j = mu_j Y_{j-1} + nu_j Y_{j-2} + (1-mu_j-nu_j) Y0 + mut_j tau L(Y_{j-1})
//         + gt_j tau M(Y0)
// with L the flux divergence of Sec. 3 (face flux of Sec. 2 and Appendix B,
// face_flux in rkl_tile.h).
//
// Scheme (overlapped tiles, z-march).  The workgroup's BX x BY threads own
// one cell each of a region whose interior (BX-2) x (BY-2) is the output
// tile.
//   Level 1 computes Y_j on the whole region, exactly as run_tile does for
//   one stage: Y_{j-1} with a one-cell ring around the region in a
//   three-plane LDS ring, slopes and b in two-plane rings, every face once.
//   Level 2 computes Y_{j+1} on the interior, three planes behind level 1.
//   Each thread hands its Y_j to level 2's LDS ring and register queue; the
//   region's border cells supply only their slopes along the border and the
//   faces towards the interior.  The pointwise inputs of level 2 (Y_{j-1},
//   Y0, tau M(Y0)) and its unit vectors are the ones level 1 loaded three
//   planes earlier, carried in register delay lines.
// Both levels share the one barrier per plane.  HBM traffic per output cell
// and stage pair: Y_{j-1}, Y_{j-2}, Y0, tau M(Y0) and b read once, Y_j and
// Y_{j+1} written once; the border ring is recomputed by the neighbouring
// tiles.  Tiles overlap, so the outputs go to buffers that the launch does
// not read.
#pragma once
#include "rkl_tile.h"

namespace rkl {

struct FusedArgs {
    const double* Yin;   // Y_{j-1}
    const double* Ym2;   // Y_{j-2}
    const double* Y0;
    const void* MY0;     // tau M(Y0), type R
    const void* b;       // unit vectors, type R, 3 x N
    double* Yj;          // out: Y_j   (aliases no input)
    double* Yj1;         // out: Y_{j+1} (aliases no input)
    int n0, n1, n2, ndim;
    int x0, y0, z0, z1;  // output tile origin and z range [z0, z1)
    double ih0, ih1, ih2;
    double scale;        // -tau (gamma-1)/rho
    double mu1, nu1, omn1, mut1, gt1;   // stage j
    double mu2, nu2, omn2, mut2, gt2;   // stage j+1
};

template <typename R, int BX, int BY>
struct FusedLds {
    static constexpr int PX = BX + 2, PL = (BX + 2) * (BY + 2), RL = BX * BY;
    // level 1: region and the ring around it
    R T1[3][PL];
    R S1[2][3][PL];
    R B1[2][3][PL];
    R FX1[2][(BX + 1) * BY];
    R FY1[2][BX * (BY + 1)];
    // level 2: region
    R T2[3][RL];
    R S2[2][3][RL];
    R B2[2][3][RL];
    R FX2[2][RL];   // face between region cells c and c+1
    R FY2[2][RL];   // face between region cells c and c+BX
};

template <typename R, bool LIM, int SAT, int KM, int BX, int BY>
__device__ __forceinline__ void run_fused2(const FusedArgs& a, const FaceK<R>& fk, double tref,
                                           FusedLds<R, BX, BY>& L) {
    using Lds = FusedLds<R, BX, BY>;
    constexpr int px = Lds::PX;
    const int tid = threadIdx.x;
    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const int plane = n0 * n1;
    const size_t N = (size_t)plane * (size_t)n2;
    const R* b0 = (const R*)a.b;
    const R* b1 = b0 + N;
    const R* b2 = b1 + N;
    const R* M0 = (const R*)a.MY0;
    const R ih0 = R(a.ih0), ih1 = R(a.ih1), ih2 = R(a.ih2);
    const R hih0 = R(0.5 * a.ih0), hih1 = R(0.5 * a.ih1), hih2 = R(0.5 * a.ih2);

    // own cell: region coordinates (tx, ty); the region starts one cell
    // before the output tile along x and y
    const int tx = tid % BX, ty = tid / BX;
    const int rx = a.x0 - 1, ry = a.y0 - 1;
    const int oslot = (ty + 1) * px + tx + 1;   // level-1 slot
    const int rslot = tid;                      // level-2 slot, ty * BX + tx
    const int oxy = wrap(ry + ty, n1) * n0 + wrap(rx + tx, n0);
    const bool inx = tx >= 1 && tx <= BX - 2, iny = ty >= 1 && ty <= BY - 2;
    const bool interior = inx && iny;
    const bool store = interior && (rx + tx < n0) && (ry + ty < n1);

    // level-1 ring cell of this thread (edges, then corners), as in run_tile
    constexpr int ne = 2 * BX + 2 * BY;
    const bool hjob = tid < ne + 4;
    const bool djob = tid < ne;
    bool dxh = false;
    int hslot = 0, hxy = 0;
    if (hjob) {
        int hi, hj;
        if (tid < BX) { hi = tid; hj = -1; }
        else if (tid < 2 * BX) { hi = tid - BX; hj = BY; }
        else if (tid < 2 * BX + BY) { hi = -1; hj = tid - 2 * BX; dxh = true; }
        else if (tid < ne) { hi = BX; hj = tid - 2 * BX - BY; dxh = true; }
        else {
            const int c = tid - ne;
            hi = (c & 1) ? BX : -1;
            hj = (c & 2) ? BY : -1;
        }
        hslot = (hj + 1) * px + hi + 1;
        hxy = wrap(ry + hj, n1) * n0 + wrap(rx + hi, n0);
    }
    // level-1 extra faces (-x face of each region row, -y face of each
    // column), on the last wave(s)
    constexpr int nf = BY + BX;
    constexpr int fbase = (BX * BY - nf) / 64 * 64;
    const int fid = tid - fbase;
    const bool fjob = fid >= 0 && fid < nf;
    int fdir = 0, fL = 0, fR = 0, fidx = 0;
    if (fjob) {
        if (fid < BY) { fdir = 0; fL = (fid + 1) * px; fR = fL + 1; fidx = fid * (BX + 1); }
        else { const int i = fid - BY; fdir = 1; fL = i + 1; fR = px + i + 1; fidx = i; }
    }

    // Level 2 needs Y_j on planes [z0-1, z1] (x/y slopes of the planes next
    // to the output range, for the transverse gradients of its z faces), so
    // level 1 runs planes [l1a, l1b) = [z0-1, z1+1) and reads Y_{j-1} on
    // [z0-3, z1+3).  Iteration K runs level-1 plane K and level-2 plane K-3.
    const int z0 = a.z0, z1 = a.z1;
    const int l1a = z0 - 1, l1b = z1 + 1;
    int pz4 = wrap(l1a + 2, n2);

    // ---- level-1 registers, as in run_tile
    double pTo0 = 0.0, pTo1 = 0.0, pTh0 = 0.0, pTh1 = 0.0;
    R pbo00 = 0, pbo01 = 0, pbo02 = 0, pbo10 = 0, pbo11 = 0, pbo12 = 0;
    R pbd00 = 0, pbd01 = 0, pbd02 = 0, pbd10 = 0, pbd11 = 0, pbd12 = 0;
    double yq0 = 0.0, yq1 = 0.0, yq2 = 0.0;
    R oq0 = 0, oq1 = 0, oq2 = 0, hq0 = 0, hq1 = 0, hq2 = 0;
    R ob00 = 0, ob01 = 0, ob02 = 0, ob10 = 0, ob11 = 0, ob12 = 0;
    R os00 = 0, os01 = 0, os02 = 0, os10 = 0, os11 = 0, os12 = 0;
    R fzp = 0;
    double ym2 = 0.0, y0v = 0.0, q1ym2 = 0.0, q1y0 = 0.0, q2ym2 = 0.0, q2y0 = 0.0;
    R my0 = 0, q1my0 = 0, q2my0 = 0;
    double yj = 0.0;   // Y_j of the last level-1 plane

    // ---- delay lines from level 1 to level 2 (values of planes K-1, K-2, K-3
    // at the start of iteration K)
    double dy1 = 0.0, dy2 = 0.0, dy3 = 0.0;   // Y_{j-1}
    double dz1 = 0.0, dz2 = 0.0, dz3 = 0.0;   // Y0
    R dm1 = 0, dm2 = 0, dm3 = 0;              // tau M(Y0)
    R db10 = 0, db11 = 0, db12 = 0, db20 = 0, db21 = 0, db22 = 0;   // b, planes K-1, K-2

    // ---- level-2 registers
    double uq0 = 0.0, uq1 = 0.0, uq2 = 0.0;   // own Y_j, planes k2, k2+1, k2+2
    R vq0 = 0, vq1 = 0, vq2 = 0;              // same in flux precision
    R ub00 = 0, ub01 = 0, ub02 = 0, ub10 = 0, ub11 = 0, ub12 = 0;   // own b, planes k2, k2+1
    R us00 = 0, us01 = 0, us02 = 0, us10 = 0, us11 = 0, us12 = 0;   // own slopes, k2, k2+1
    R gzp = 0;

    int c0 = 0, c1 = 1, c2 = 2, dc = 1, dn = 0;   // level-1 ring slots
    int e0 = 0, e1 = 1, e2 = 2, ec = 1, en = 0;   // level-2 ring slots
    int fb = 0;

    // level-1 prologue: ring planes l1a-2, l1a-1; prefetch l1a, l1a+1
    {
        const double* p0 = a.Yin + (size_t)wrap(l1a - 2, n2) * plane;
        const double* p1 = a.Yin + (size_t)wrap(l1a - 1, n2) * plane;
        const double* p2 = a.Yin + (size_t)wrap(l1a, n2) * plane;
        const double* p3 = a.Yin + (size_t)wrap(l1a + 1, n2) * plane;
        const size_t pb0 = (size_t)wrap(l1a - 1, n2) * plane;
        const size_t pb1 = (size_t)wrap(l1a, n2) * plane;
        yq1 = p0[oxy];
        yq2 = p1[oxy];
        pTo0 = p2[oxy];
        pTo1 = p3[oxy];
        pbo00 = b0[pb0 + oxy]; pbo01 = b1[pb0 + oxy]; pbo02 = b2[pb0 + oxy];
        pbo10 = b0[pb1 + oxy]; pbo11 = b1[pb1 + oxy]; pbo12 = b2[pb1 + oxy];
        if (hjob) {
            const double h1 = p0[hxy], h2 = p1[hxy];
            pTh0 = p2[hxy];
            pTh1 = p3[hxy];
            hq1 = to_r<R>(h1, tref);
            hq2 = to_r<R>(h2, tref);
            L.T1[0][hslot] = hq1;
            L.T1[1][hslot] = hq2;
        }
        if (djob) {
            pbd00 = b0[pb0 + hxy]; pbd01 = b1[pb0 + hxy]; pbd02 = b2[pb0 + hxy];
            pbd10 = b0[pb1 + hxy]; pbd11 = b1[pb1 + hxy]; pbd12 = b2[pb1 + hxy];
        }
        oq1 = to_r<R>(yq1, tref);
        oq2 = to_r<R>(yq2, tref);
        L.T1[0][oslot] = oq1;
        L.T1[1][oslot] = oq2;
        // the level-2 ring plane below its first one is read (for slopes that
        // are never used) before it is written: give it defined values
        L.T2[0][rslot] = R(0);
        L.T2[1][rslot] = R(0);
        L.T2[2][rslot] = R(0);
    }
    __syncthreads();

    for (int K = l1a - 2; K < z1 + 3; ++K) {
        const int k2 = K - 3;
        const bool l1 = K < l1b;
        const bool l2 = k2 >= z0 - 3;   // level 2 stores Y_j(k2+2) from k2+2 = z0-1 on

        // ============ level 1, A and B: T(K+2), b(K+1) in; slopes of K+1
        if (l1) {
            yq0 = yq1; yq1 = yq2; yq2 = pTo0;
            oq0 = oq1; oq1 = oq2; oq2 = to_r<R>(pTo0, tref);
            L.T1[c2][oslot] = oq2;
            L.B1[dn][0][oslot] = pbo00; L.B1[dn][1][oslot] = pbo01; L.B1[dn][2][oslot] = pbo02;
            ob00 = ob10; ob01 = ob11; ob02 = ob12;
            ob10 = pbo00; ob11 = pbo01; ob12 = pbo02;
            if (hjob) {
                hq0 = hq1; hq1 = hq2; hq2 = to_r<R>(pTh0, tref);
                L.T1[c2][hslot] = hq2;
            }
            if (djob) { L.B1[dn][0][hslot] = pbd00; L.B1[dn][1][hslot] = pbd01; L.B1[dn][2][hslot] = pbd02; }
            pTo0 = pTo1; pTh0 = pTh1;
            pbo00 = pbo10; pbo01 = pbo11; pbo02 = pbo12;
            pbd00 = pbd10; pbd01 = pbd11; pbd02 = pbd12;
            if (K + 2 < l1b) {
                const double* pt = a.Yin + (size_t)pz4 * plane;
                const int pbz = pz4 == 0 ? n2 - 1 : pz4 - 1;
                const size_t pb = (size_t)pbz * plane;
                pTo1 = pt[oxy];
                pbo10 = b0[pb + oxy]; pbo11 = b1[pb + oxy]; pbo12 = b2[pb + oxy];
                if (hjob) pTh1 = pt[hxy];
                if (djob) { pbd10 = b0[pb + hxy]; pbd11 = b1[pb + hxy]; pbd12 = b2[pb + hxy]; }
                pz4 = pz4 + 1 == n2 ? 0 : pz4 + 1;
            }
            ym2 = q1ym2; y0v = q1y0; my0 = q1my0;
            q1ym2 = q2ym2; q1y0 = q2y0; q1my0 = q2my0;
            if (K + 2 >= l1a && K + 2 < l1b) {
                const size_t o = (size_t)wrap(K + 2, n2) * plane + oxy;
                q2ym2 = a.Ym2[o];
                q2y0 = a.Y0[o];
                q2my0 = M0[o];
            }
            const R* T1 = L.T1[c1];
            const R s0 = cell_slope<R, LIM>(T1[oslot - 1], oq1, T1[oslot + 1], hih0);
            const R s1 = cell_slope<R, LIM>(T1[oslot - px], oq1, T1[oslot + px], hih1);
            const R s2 = cell_slope<R, LIM>(oq0, oq1, oq2, hih2);
            L.S1[dn][0][oslot] = s0; L.S1[dn][1][oslot] = s1; L.S1[dn][2][oslot] = s2;
            os00 = os10; os01 = os11; os02 = os12;
            os10 = s0; os11 = s1; os12 = s2;
            if (djob) {
                if (dxh) L.S1[dn][1][hslot] = cell_slope<R, LIM>(T1[hslot - px], hq1, T1[hslot + px], hih1);
                else     L.S1[dn][0][hslot] = cell_slope<R, LIM>(T1[hslot - 1], hq1, T1[hslot + 1], hih0);
                L.S1[dn][2][hslot] = cell_slope<R, LIM>(hq0, hq1, hq2, hih2);
            }
        }

        // ============ level 2, A and B: Y_j(k2+2) = Y_j(K-1), b(k2+1) = b(K-2)
        // in; slopes of k2+1 (along the region border only the slopes
        // parallel to it)
        if (l2) {
            uq0 = uq1; uq1 = uq2; uq2 = yj;
            vq0 = vq1; vq1 = vq2; vq2 = to_r<R>(yj, tref);
            L.T2[e2][rslot] = vq2;
            L.B2[en][0][rslot] = db20; L.B2[en][1][rslot] = db21; L.B2[en][2][rslot] = db22;
            ub00 = ub10; ub01 = ub11; ub02 = ub12;
            ub10 = db20; ub11 = db21; ub12 = db22;
            const R* T2 = L.T2[e1];
            const R s0 = inx ? cell_slope<R, LIM>(T2[rslot - 1], vq1, T2[rslot + 1], hih0) : R(0);
            const R s1 = iny ? cell_slope<R, LIM>(T2[rslot - BX], vq1, T2[rslot + BX], hih1) : R(0);
            const R s2 = cell_slope<R, LIM>(vq0, vq1, vq2, hih2);
            L.S2[en][0][rslot] = s0; L.S2[en][1][rslot] = s1; L.S2[en][2][rslot] = s2;
            us00 = us10; us01 = us11; us02 = us12;
            us10 = s0; us11 = s1; us12 = s2;
        }

        // ============ level 1, C: faces of plane K
        R fzn = 0;
        if (l1 && K >= l1a) {
            const R* Tk = L.T1[c0];
            const R(*S)[Lds::PL] = L.S1[dc];
            const R(*Bv)[Lds::PL] = L.B1[dc];
            R* FX = L.FX1[fb];
            R* FY = L.FY1[fb];
            const int r = oslot + 1;
            FX[ty * (BX + 1) + tx + 1] = face_flux<R, LIM, SAT, KM>(
                oq0, Tk[r], ih0, os01, S[1][r], os02, S[2][r],
                ob00, ob01, ob02, Bv[0][r], Bv[1][r], Bv[2][r], fk);
            const int u = oslot + px;
            FY[(ty + 1) * BX + tx] = face_flux<R, LIM, SAT, KM>(
                oq0, Tk[u], ih1, os00, S[0][u], os02, S[2][u],
                ob01, ob00, ob02, Bv[1][u], Bv[0][u], Bv[2][u], fk);
            if (fjob) {
                const int t1 = fdir == 0 ? 1 : 0;
                const R f = face_flux<R, LIM, SAT, KM>(
                    Tk[fL], Tk[fR], fdir == 0 ? ih0 : ih1, S[t1][fL], S[t1][fR], S[2][fL], S[2][fR],
                    Bv[fdir][fL], Bv[t1][fL], Bv[2][fL], Bv[fdir][fR], Bv[t1][fR], Bv[2][fR], fk);
                if (fdir == 0) FX[fidx] = f; else FY[fidx] = f;
            }
        }
        if (l1 && K >= l1a - 1) {
            fzn = face_flux<R, LIM, SAT, KM>(oq0, oq1, ih2, os00, os10, os01, os11,
                                             ob02, ob00, ob01, ob12, ob10, ob11, fk);
        }

        // ============ level 2, C: faces of plane k2 that touch the interior
        R gzn = 0;
        if (l2 && k2 >= z0) {
            const R* Tk = L.T2[e0];
            const R(*S)[Lds::RL] = L.S2[ec];
            const R(*Bv)[Lds::RL] = L.B2[ec];
            if (iny && tx <= BX - 2) {
                const int r = rslot + 1;
                L.FX2[fb][rslot] = face_flux<R, LIM, SAT, KM>(
                    vq0, Tk[r], ih0, us01, S[1][r], us02, S[2][r],
                    ub00, ub01, ub02, Bv[0][r], Bv[1][r], Bv[2][r], fk);
            }
            if (inx && ty <= BY - 2) {
                const int u = rslot + BX;
                L.FY2[fb][rslot] = face_flux<R, LIM, SAT, KM>(
                    vq0, Tk[u], ih1, us00, S[0][u], us02, S[2][u],
                    ub01, ub00, ub02, Bv[1][u], Bv[0][u], Bv[2][u], fk);
            }
        }
        if (l2 && interior && k2 >= z0 - 1) {
            gzn = face_flux<R, LIM, SAT, KM>(vq0, vq1, ih2, us00, us10, us01, us11,
                                             ub02, ub00, ub01, ub12, ub10, ub11, fk);
        }
        __syncthreads();

        // ============ level 1, D: Y_j of plane K on the whole region
        if (l1 && K >= l1a) {
            const R* FX = L.FX1[fb];
            const R* FY = L.FY1[fb];
            const int fx = ty * (BX + 1) + tx;
            R div = (FX[fx + 1] - FX[fx]) * ih0;
            div = fma(FY[(ty + 1) * BX + tx] - FY[ty * BX + tx], ih1, div);
            div = fma(fzn - fzp, ih2, div);
            const double tl = a.scale * (double)div;
            yj = stage_combine(a.mu1, a.nu1, a.omn1, a.mut1, a.gt1, yq0, ym2, y0v, tl, (double)my0);
            if (store && K >= z0 && K < z1) a.Yj[(size_t)K * plane + oxy] = yj;
        }
        fzp = fzn;

        // ============ level 2, D: Y_{j+1} of plane k2 on the interior
        if (l2 && k2 >= z0 && store) {
            const R* FX = L.FX2[fb];
            const R* FY = L.FY2[fb];
            R div = (FX[rslot] - FX[rslot - 1]) * ih0;
            div = fma(FY[rslot] - FY[rslot - BX], ih1, div);
            div = fma(gzn - gzp, ih2, div);
            const double tl = a.scale * (double)div;
            a.Yj1[(size_t)k2 * plane + oxy] =
                stage_combine(a.mu2, a.nu2, a.omn2, a.mut2, a.gt2, uq0, dy3, dz3, tl, (double)dm3);
        }
        gzp = gzn;

        // delay lines: push plane K
        dy3 = dy2; dy2 = dy1; dy1 = yq0;
        dz3 = dz2; dz2 = dz1; dz1 = y0v;
        dm3 = dm2; dm2 = dm1; dm1 = my0;
        db20 = db10; db21 = db11; db22 = db12;
        db10 = ob00; db11 = ob01; db12 = ob02;

        if (l1) {
            const int t = c0; c0 = c1; c1 = c2; c2 = t;
            const int d = dc; dc = dn; dn = d;
        }
        if (l2) {
            const int t = e0; e0 = e1; e1 = e2; e2 = t;
            const int d = ec; ec = en; en = d;
        }
        fb ^= 1;
    }
}

}  // namespace rkl
