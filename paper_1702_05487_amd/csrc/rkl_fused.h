// rkl_fused.h -- F consecutive RKL2 stages per launch (temporal fusion,
// F = 2, 3 or 4) for gfx950.  Private to librkl; included by the kernel
// sources only.
//
// Method: Vaidya et al. (2017), arXiv:1702.05487, Appendix A: stages
// j, ..., j+F-1 (2 <= j, j+F-1 < s) of
//   Y_m = mu_m Y_{m-1} + nu_m Y_{m-2} + (1-mu_m-nu_m) Y0 + mut_m tau L(Y_{m-1})
//         + gt_m tau M(Y0)
// with L the flux divergence of Sec. 3 (face flux of Sec. 2 and Appendix B,
// face_flux in rkl_tile.h).
//
// Scheme (overlapped tiles, z-march).  The workgroup's BX x BY threads own
// one cell each of a region; a cell's distance from the region border is
// d = min(dx, dy), dx = min(tx, BX-1-tx), dy = min(ty, BY-1-ty).
//   Level 1 computes Y_j on the whole region, exactly as run_tile does for
//   one stage: Y_{j-1} with a one-cell ring around the region in a
//   three-plane LDS ring, slopes and b in two-plane rings, every face once.
//   Level l = 2..F computes Y_{j+l-1} three planes behind level l-1, on the
//   cells with d >= l-1, from level l-1's output (valid on d >= l-2), handed
//   over through LDS and registers.  A cell with d = l-2 supplies only its
//   slope along the border and the faces towards the inside; the output
//   tile is the cells with d >= F-1, of (BX-2(F-1)) x (BY-2(F-1)) cells.
//   The pointwise inputs of level l (Y_{j+l-3}, Y0, tau M(Y0)) and its unit
//   vectors come down from level 1's loads through register delay lines,
//   three planes per level.
// All levels share the one barrier per plane.  HBM traffic per output cell
// and group of F stages: Y_{j-1}, Y_{j-2}, Y0, tau M(Y0) and b read once,
// Y_{j+F-2} and Y_{j+F-1} (what the next launch needs) written once; the
// border rings are recomputed by the neighbouring tiles.  Tiles overlap, so
// the outputs go to buffers that the launch does not read.  Every level
// performs exactly the one-stage kernel's operations, so fused and unfused
// super-steps give the same bits.
#pragma once
#include "rkl_tile.h"

namespace rkl {

constexpr int kMaxFuse = 4;

struct FusedArgs {
    const double* Yin;   // Y_{j-1}
    const double* Ym2;   // Y_{j-2}
    const double* Y0;
    const void* MY0;     // tau M(Y0), type R
    const void* b;       // unit vectors, type R, 3 x N
    double* Ya;          // out: Y_{j+F-2} (aliases no input)
    double* Yb;          // out: Y_{j+F-1} (aliases no input)
    int n0, n1, n2, ndim;
    int x0, y0, z0, z1;  // output tile origin and z range [z0, z1)
    double ih0, ih1, ih2;
    double scale;        // -tau (gamma-1)/rho
    double cf[kMaxFuse][5];   // {mu, nu, 1-mu-nu, mut, gt} of stages j..j+F-1
};

template <typename R, int BX, int BY, int F>
struct FusedLds {
    static constexpr int PX = BX + 2, PL = (BX + 2) * (BY + 2), RL = BX * BY, NL = F - 1;
    // level 1: region and the ring around it
    R T1[3][PL];
    R S1[2][3][PL];
    R B1[2][3][PL];
    R FX1[2][(BX + 1) * BY];
    R FY1[2][BX * (BY + 1)];
    // levels 2..F: region
    R T2[NL][3][RL];
    R S2[NL][2][3][RL];
    R B2[NL][2][3][RL];
    R FX2[NL][2][RL];   // face between region cells c and c+1
    R FY2[NL][2][RL];   // face between region cells c and c+BX
};

template <typename R, bool LIM, int SAT, int KM, int BX, int BY, int F>
__device__ __forceinline__ void run_fused(const FusedArgs& a, const FaceK<R>& fk, double tref,
                                          FusedLds<R, BX, BY, F>& L) {
    using Lds = FusedLds<R, BX, BY, F>;
    constexpr int px = Lds::PX;
    constexpr int NL = F - 1;
    const int tid = threadIdx.x;
    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const int plane = n0 * n1;
    const size_t N = (size_t)plane * (size_t)n2;
    const R* b0 = (const R*)a.b;
    const R* b1 = b0 + N;
    const R* b2 = b1 + N;
    const R* M0 = (const R*)a.MY0;
    const R ih0 = R(a.ih0), ih1 = R(a.ih1), ih2 = R(a.ih2);
    const R hih0 = R(0.25 * a.ih0), hih1 = R(0.25 * a.ih1), hih2 = R(0.25 * a.ih2);   // 1/(4h), see cell_slope

    // own cell: region coordinates (tx, ty); the region starts F-1 cells
    // before the output tile along x and y
    const int tx = tid % BX, ty = tid / BX;
    const int rx = a.x0 - (F - 1), ry = a.y0 - (F - 1);
    const int oslot = (ty + 1) * px + tx + 1;   // level-1 slot
    const int rslot = tid;                      // level-l slot, ty * BX + tx
    const int oxy = wrap(ry + ty, n1) * n0 + wrap(rx + tx, n0);
    const int dx = min(tx, BX - 1 - tx), dy = min(ty, BY - 1 - ty), dd = min(dx, dy);
    const bool store = dd >= F - 1 && (rx + tx < n0) && (ry + ty < n1);

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

    // Level l computes planes [z0-(F-l), z1+(F-l)): each level needs the
    // previous one's output one plane beyond its own range on either side
    // (the x/y slopes of the neighbouring planes, for the transverse
    // gradients of its z faces).  Level 1 therefore runs [l1a, l1b) and
    // reads Y_{j-1} on [l1a-2, l1b+1]; iteration K runs level-1 plane K and
    // level-l plane K - 3(l-1).
    const int z0 = a.z0, z1 = a.z1;
    const int l1a = z0 - (F - 1), l1b = z1 + (F - 1);
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
    double yout0 = 0.0;   // level-1 output Y_j of the last level-1 plane

    // ---- levels 2..F (index m = l - 2)
    double uq[NL][3];     // own input Y_{j+l-2}, planes k, k+1, k+2
    R vq[NL][3];          // same in flux precision
    R ub[NL][2][3];       // own b, planes k, k+1
    R us[NL][2][3];       // own slopes, planes k, k+1
    R gzp[NL];            // +z face flux of plane k-1
    double yout[NL];      // output Y_{j+l-1} of the last plane
    // delay lines into level l (values of the planes 1, 2, 3 iterations back)
    double dY[NL][3];     // Y_{j+l-3}: level l-1's own input (level 1: Y_{j-1})
    double dZ[NL][3];     // Y0
    R dM[NL][3];          // tau M(Y0)
    R dB[NL][2][3];       // b, two planes back
    int e0[NL], e1[NL], e2[NL], ec[NL], en[NL];   // ring slots
#pragma unroll
    for (int m = 0; m < NL; ++m) {
        gzp[m] = 0;
        yout[m] = 0.0;
        e0[m] = 0; e1[m] = 1; e2[m] = 2; ec[m] = 1; en[m] = 0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            uq[m][q] = 0.0; vq[m][q] = 0; dY[m][q] = 0.0; dZ[m][q] = 0.0; dM[m][q] = 0;
            ub[m][0][q] = 0; ub[m][1][q] = 0; us[m][0][q] = 0; us[m][1][q] = 0;
            dB[m][0][q] = 0; dB[m][1][q] = 0;
        }
    }

    int c0 = 0, c1 = 1, c2 = 2, dc = 1, dn = 0;   // level-1 ring slots
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
        // the level-l ring plane below its first one is read (for slopes that
        // are never used) before it is written: give it defined values
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            L.T2[m][0][rslot] = R(0);
            L.T2[m][1][rslot] = R(0);
            L.T2[m][2][rslot] = R(0);
        }
    }
    __syncthreads();

    for (int K = l1a - 2; K < z1 + 3 * (F - 1); ++K) {
        const bool l1 = K < l1b;

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

        // ============ levels 2..F, A and B: Y_{j+l-2}(k+2) (level l-1's last
        // output) and b(k+1) in; slopes of k+1 (where the neighbours have input)
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            const int l = m + 2;
            const int k = K - 3 * (l - 1);
            if (k + 2 < z0 - (F - l + 1)) continue;   // level l-1 has no output yet
            const double yin = m == 0 ? yout0 : yout[m - 1];
            uq[m][0] = uq[m][1]; uq[m][1] = uq[m][2]; uq[m][2] = yin;
            vq[m][0] = vq[m][1]; vq[m][1] = vq[m][2]; vq[m][2] = to_r<R>(yin, tref);
            L.T2[m][e2[m]][rslot] = vq[m][2];
            L.B2[m][en[m]][0][rslot] = dB[m][1][0];
            L.B2[m][en[m]][1][rslot] = dB[m][1][1];
            L.B2[m][en[m]][2][rslot] = dB[m][1][2];
            ub[m][0][0] = ub[m][1][0]; ub[m][0][1] = ub[m][1][1]; ub[m][0][2] = ub[m][1][2];
            ub[m][1][0] = dB[m][1][0]; ub[m][1][1] = dB[m][1][1]; ub[m][1][2] = dB[m][1][2];
            const R* T2 = L.T2[m][e1[m]];
            const R s0 = (dx >= l - 1 && dy >= l - 2) ? cell_slope<R, LIM>(T2[rslot - 1], vq[m][1], T2[rslot + 1], hih0) : R(0);
            const R s1 = (dy >= l - 1 && dx >= l - 2) ? cell_slope<R, LIM>(T2[rslot - BX], vq[m][1], T2[rslot + BX], hih1) : R(0);
            const R s2 = cell_slope<R, LIM>(vq[m][0], vq[m][1], vq[m][2], hih2);
            L.S2[m][en[m]][0][rslot] = s0; L.S2[m][en[m]][1][rslot] = s1; L.S2[m][en[m]][2][rslot] = s2;
            us[m][0][0] = us[m][1][0]; us[m][0][1] = us[m][1][1]; us[m][0][2] = us[m][1][2];
            us[m][1][0] = s0; us[m][1][1] = s1; us[m][1][2] = s2;
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

        // ============ levels 2..F, C: faces of plane k that touch its output cells
        R gzn[NL];
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            const int l = m + 2;
            const int k = K - 3 * (l - 1);
            gzn[m] = 0;
            const int lo = z0 - (F - l), hi = z1 + (F - l);
            if (k + 2 < z0 - (F - l + 1)) continue;
            if (k >= lo && k < hi) {
                const R* Tk = L.T2[m][e0[m]];
                const R(*S)[Lds::RL] = L.S2[m][ec[m]];
                const R(*Bv)[Lds::RL] = L.B2[m][ec[m]];
                if (dy >= l - 1 && tx >= l - 2 && tx <= BX - l) {
                    const int r = rslot + 1;
                    L.FX2[m][fb][rslot] = face_flux<R, LIM, SAT, KM>(
                        vq[m][0], Tk[r], ih0, us[m][0][1], S[1][r], us[m][0][2], S[2][r],
                        ub[m][0][0], ub[m][0][1], ub[m][0][2], Bv[0][r], Bv[1][r], Bv[2][r], fk);
                }
                if (dx >= l - 1 && ty >= l - 2 && ty <= BY - l) {
                    const int u = rslot + BX;
                    L.FY2[m][fb][rslot] = face_flux<R, LIM, SAT, KM>(
                        vq[m][0], Tk[u], ih1, us[m][0][0], S[0][u], us[m][0][2], S[2][u],
                        ub[m][0][1], ub[m][0][0], ub[m][0][2], Bv[1][u], Bv[0][u], Bv[2][u], fk);
                }
            }
            if (dd >= l - 1 && k >= lo - 1 && k < hi) {
                gzn[m] = face_flux<R, LIM, SAT, KM>(vq[m][0], vq[m][1], ih2, us[m][0][0], us[m][1][0], us[m][0][1],
                                                    us[m][1][1], ub[m][0][2], ub[m][0][0], ub[m][0][1], ub[m][1][2],
                                                    ub[m][1][0], ub[m][1][1], fk);
            }
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
            const double* c = a.cf[0];
            yout0 = stage_combine(c[0], c[1], c[2], c[3], c[4], yq0, ym2, y0v, tl, (double)my0);
            if (F == 2 && store && K >= z0 && K < z1) a.Ya[(size_t)K * plane + oxy] = yout0;
        }
        fzp = fzn;

        // ============ levels 2..F, D: Y_{j+l-1} of plane k on the cells with d >= l-1
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            const int l = m + 2;
            const int k = K - 3 * (l - 1);
            const int lo = z0 - (F - l), hi = z1 + (F - l);
            if (k + 2 < z0 - (F - l + 1)) continue;
            if (k >= lo && k < hi && dd >= l - 1) {
                const R* FX = L.FX2[m][fb];
                const R* FY = L.FY2[m][fb];
                R div = (FX[rslot] - FX[rslot - 1]) * ih0;
                div = fma(FY[rslot] - FY[rslot - BX], ih1, div);
                div = fma(gzn[m] - gzp[m], ih2, div);
                const double tl = a.scale * (double)div;
                const double* c = a.cf[l - 1];
                yout[m] = stage_combine(c[0], c[1], c[2], c[3], c[4], uq[m][0], dY[m][2], dZ[m][2], tl,
                                        (double)dM[m][2]);
                if (store && k >= z0 && k < z1) {
                    if (l == F - 1) a.Ya[(size_t)k * plane + oxy] = yout[m];
                    if (l == F) a.Yb[(size_t)k * plane + oxy] = yout[m];
                }
            }
            gzp[m] = gzn[m];
        }

        // delay lines: push this iteration's values, highest level first (a
        // level's source is the line of the level before it)
#pragma unroll
        for (int m = NL - 1; m >= 0; --m) {
            const double srcY = m == 0 ? yq0 : uq[m - 1][0];
            const double srcZ = m == 0 ? y0v : dZ[m - 1][2];
            const R srcM = m == 0 ? my0 : dM[m - 1][2];
            const R sb0 = m == 0 ? ob00 : ub[m - 1][0][0];
            const R sb1 = m == 0 ? ob01 : ub[m - 1][0][1];
            const R sb2 = m == 0 ? ob02 : ub[m - 1][0][2];
            dY[m][2] = dY[m][1]; dY[m][1] = dY[m][0]; dY[m][0] = srcY;
            dZ[m][2] = dZ[m][1]; dZ[m][1] = dZ[m][0]; dZ[m][0] = srcZ;
            dM[m][2] = dM[m][1]; dM[m][1] = dM[m][0]; dM[m][0] = srcM;
            dB[m][1][0] = dB[m][0][0]; dB[m][1][1] = dB[m][0][1]; dB[m][1][2] = dB[m][0][2];
            dB[m][0][0] = sb0; dB[m][0][1] = sb1; dB[m][0][2] = sb2;
        }

        if (l1) {
            const int t = c0; c0 = c1; c1 = c2; c2 = t;
            const int d = dc; dc = dn; dn = d;
        }
#pragma unroll
        for (int m = 0; m < NL; ++m) {
            const int l = m + 2;
            const int k = K - 3 * (l - 1);
            if (k + 2 < z0 - (F - l + 1)) continue;
            const int t = e0[m]; e0[m] = e1[m]; e1[m] = e2[m]; e2[m] = t;
            const int d = ec[m]; ec[m] = en[m]; en[m] = d;
        }
        fb ^= 1;
    }
}

}  // namespace rkl
