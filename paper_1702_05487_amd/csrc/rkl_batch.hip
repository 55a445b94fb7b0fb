// rkl_batch.hip -- one RKL2 super-step of many independent periodic grids
// ("patches") of uneven size, each with its own field, super-step and stage
// count, without host synchronisation (graph-capturable).
//
// Sequence: one reduce/finalize launch (a workgroup per grid computes that
// grid's temperature extrema, dt_par and stage count s_g on the device), then
// one launch per stage j = 1..smax over every tile of every grid; a tile
// whose grid has s_g < j returns at once.  Tile shapes are chosen per grid so
// that a patch narrower than 64 cells is covered by full-width rows (no
// ragged x tiles); every tile runs the same run_tile code as the single-grid
// kernels.
#include <algorithm>
#include <cstring>

#include "rkl_batch.h"
#include "rkl_tile.h"

namespace rkl {

constexpr int kBT = 256;        // threads per batched workgroup
constexpr int kPL = 400;        // LDS plane capacity, (bx+2)(by+2)
constexpr int kFX = 320;        // x-face capacity, (bx+1) by
constexpr int kFY = 320;        // y-face capacity, bx (by+1)

struct BatchGrid {
    GridConst gc;
    int64_t off;
    int bx, by, bz, ntx, nty, nzc;
    int tile0;
};

struct BatchPlan {
    int ngrids = 0, precision = 0, smax = 0, items = 0;
    int limiter = 0, saturation = 0;
    BatchGrid* grids = nullptr;   // device
    int* item_grid = nullptr;     // device, item -> grid
};

__device__ __forceinline__ int xcd_remap_b(int b, int nb) {
    const int q = nb / 8, r = nb % 8;
    const int xcd = b % 8, slot = b / 8;
    return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// one workgroup per grid: extrema of T, then dt_par and s for that grid
__global__ __launch_bounds__(kBT) void batch_reduce_kernel(const BatchGrid* __restrict__ grids,
                                                           const double* __restrict__ T,
                                                           const double* __restrict__ dt_hyp,
                                                           GridState* state, int32_t* s_out, int smax) {
    const int g = blockIdx.x;
    const BatchGrid G = grids[g];
    const int64_t N = (int64_t)G.gc.n0 * G.gc.n1 * G.gc.n2;
    const double* t = T + G.off;
    double mx = -INFINITY, mn = INFINITY, bad = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += kBT) {
        const double v = t[i];
        mx = fmax(mx, v);
        mn = fmin(mn, v);
        bad = isfinite(v) ? bad : 1.0;
    }
    for (int off = 32; off > 0; off >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, off));
        mn = fmin(mn, __shfl_xor(mn, off));
        bad = fmax(bad, __shfl_xor(bad, off));
    }
    __shared__ double sm[3][kBT / 64];
    const int w = threadIdx.x / 64;
    if (threadIdx.x % 64 == 0) { sm[0][w] = mx; sm[1][w] = mn; sm[2][w] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBT / 64; ++i) {
            mx = fmax(mx, sm[0][i]);
            mn = fmin(mn, sm[1][i]);
            bad = fmax(bad, sm[2][i]);
        }
        double dh = dt_hyp[g];
        if (!(dh >= 0.0) || isinf(dh)) dh = NAN;   // rejected below via the stage count
        GridState o = finalize_state(G.gc, mx, mn, bad != 0.0, dh, 0, smax);
        if (isnan(dh)) { o.s = 0x7fffffff; o.flags |= RKL_FLAG_STAGES; }
        state[g] = o;
        if (s_out) s_out[g] = o.s;
    }
}

struct BatchStageArgs {
    const BatchGrid* grids;
    const int* item_grid;
    const GridState* state;
    const double* coef;
    double* T;
    const void* b;
    double* Ya;
    double* Yb;
    void* MY0;
    int stage;
};

template <typename R, bool LIM, bool SAT>
__global__ __launch_bounds__(kBT) void batch_stage_kernel(BatchStageArgs P) {
    __shared__ TileLds<R, kPL, kFX, kFY> L;
    const int item = xcd_remap_b(blockIdx.x, gridDim.x);
    const int g = P.item_grid[item];
    const GridState st = P.state[g];
    const int j = P.stage;
    if (st.s < j || (st.flags & RKL_FLAG_STAGES)) return;   // uniform over the block
    const BatchGrid& G = P.grids[g];
    int t = item - G.tile0;
    const int tile_x = t % G.ntx;
    t /= G.ntx;
    const int tile_y = t % G.nty;
    const int zc = t / G.nty;

    double* Tg = P.T + G.off;
    double* A = P.Ya + G.off;
    double* B = P.Yb + G.off;
    R* M = (R*)P.MY0 + G.off;
    TileArgs a;
    a.b = (const R*)P.b + 3 * G.off;
    a.n0 = G.gc.n0;
    a.n1 = G.gc.n1;
    a.n2 = G.gc.n2;
    a.ndim = G.gc.ndim;
    a.bx = G.bx;
    a.by = G.by;
    a.x0 = tile_x * G.bx;
    a.y0 = tile_y * G.by;
    a.z0 = zc * G.bz;
    a.z1 = min(a.z0 + G.bz, a.n2);
    a.ih0 = G.gc.ih0;
    a.ih1 = G.gc.ih1;
    a.ih2 = G.gc.ih2;
    a.scale = -st.cdiv;
    const double* cf = P.coef + 5 * ((size_t)st.s * (st.s + 1) / 2 + j);
    a.mu = cf[0];
    a.nu = cf[1];
    a.omn = cf[2];
    a.mut = cf[3];
    a.gt = cf[4];
    // stage j writes A for odd j, B for even j, and T for j = s; it reads
    // Y_{j-1} (stencil) and Y_{j-2} (pointwise) from where they were written
    a.Y0 = Tg;
    a.MY0in = M;
    a.MY0out = M;
    if (j == 1) {
        a.kind = 1;
        a.Yin = Tg;
        a.Ym2 = nullptr;
    } else {
        a.kind = 2;
        a.Yin = ((j - 1) & 1) ? A : B;
        a.Ym2 = j == 2 ? Tg : (((j - 2) & 1) ? A : B);
    }
    a.Yout = j == st.s ? Tg : ((j & 1) ? A : B);
    const double tref = sizeof(R) == 4 ? st.tref : 0.0;
    FaceK<R> fk;
    fk.kappa0 = R(G.gc.kappa0);
    fk.kexp = R(G.gc.kexp);
    fk.kperp = R(G.gc.kperp);
    fk.satq = R(G.gc.satq);
    fk.tref = R(tref);
    fk.kmode = G.gc.kmode;
    run_tile<R, LIM, SAT>(a, fk, tref, L);
}

// tile shape for one grid: full-width rows when the grid is at most 64 cells
// wide, as many rows as fit 256 threads (at most 64), the whole z extent up
// to 32 planes per tile
static void choose_tile(const GridConst& g, int& bx, int& by, int& bz) {
    bx = std::min(g.n0, 64);
    by = std::min(std::min(g.n1, kBT / bx), 64);
    bz = std::min(g.n2, 32);
}

rkl_status batch_create(const std::vector<rkl_grid_desc>& desc, const std::vector<GridConst>& gc,
                        const std::vector<int64_t>& off, int precision, int smax, BatchPlan** out,
                        std::string& why) {
    *out = nullptr;
    const int n = (int)desc.size();
    std::vector<BatchGrid> h(n);
    std::vector<int> item_grid;
    for (int g = 0; g < n; ++g) {
        if (desc[g].limiter != desc[0].limiter || desc[g].saturation != desc[0].saturation) {
            why = "batched grids must share the limiter and saturation settings";
            return RKL_EINVAL;
        }
        BatchGrid& B = h[g];
        B.gc = gc[g];
        B.off = off[g];
        choose_tile(gc[g], B.bx, B.by, B.bz);
        if ((B.bx + 2) * (B.by + 2) > kPL || (B.bx + 1) * B.by > kFX || B.bx * (B.by + 1) > kFY ||
            2 * (B.bx + 2) + 2 * B.by > kBT) {
            why = "internal: batched tile shape exceeds the LDS layout";
            return RKL_EINVAL;
        }
        B.ntx = (gc[g].n0 + B.bx - 1) / B.bx;
        B.nty = (gc[g].n1 + B.by - 1) / B.by;
        B.nzc = (gc[g].n2 + B.bz - 1) / B.bz;
        B.tile0 = (int)item_grid.size();
        const int64_t nt = (int64_t)B.ntx * B.nty * B.nzc;
        if (item_grid.size() + nt > (size_t)0x7fffffff) { why = "too many tiles"; return RKL_EINVAL; }
        item_grid.insert(item_grid.end(), (size_t)nt, g);
    }
    BatchPlan* bp = new BatchPlan();
    bp->ngrids = n;
    bp->precision = precision;
    bp->smax = smax;
    bp->items = (int)item_grid.size();
    bp->limiter = desc[0].limiter;
    bp->saturation = desc[0].saturation;
    if (hipMalloc(&bp->grids, sizeof(BatchGrid) * n) != hipSuccess ||
        hipMalloc(&bp->item_grid, sizeof(int) * item_grid.size()) != hipSuccess) {
        hipGetLastError();
        batch_free(bp);
        why = "device allocation failed";
        return RKL_ENOMEM;
    }
    if (hipMemcpy(bp->grids, h.data(), sizeof(BatchGrid) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(bp->item_grid, item_grid.data(), sizeof(int) * item_grid.size(), hipMemcpyHostToDevice) !=
            hipSuccess) {
        hipGetLastError();
        batch_free(bp);
        why = "batched plan upload failed";
        return RKL_EDEVICE;
    }
    *out = bp;
    return RKL_OK;
}

void batch_free(BatchPlan* bp) {
    if (!bp) return;
    hipFree(bp->grids);
    hipFree(bp->item_grid);
    delete bp;
}

template <typename R>
static void launch_stage_b(const BatchPlan* bp, const BatchStageArgs& a, hipStream_t st) {
    const bool lim = bp->limiter != 0, sat = bp->saturation != 0;
    if (lim && sat) batch_stage_kernel<R, true, true><<<bp->items, kBT, 0, st>>>(a);
    else if (lim) batch_stage_kernel<R, true, false><<<bp->items, kBT, 0, st>>>(a);
    else if (sat) batch_stage_kernel<R, false, true><<<bp->items, kBT, 0, st>>>(a);
    else batch_stage_kernel<R, false, false><<<bp->items, kBT, 0, st>>>(a);
}

hipError_t batch_launch(BatchPlan* bp, const BatchBuffers& buf, hipStream_t st) {
    batch_reduce_kernel<<<bp->ngrids, kBT, 0, st>>>(bp->grids, buf.T, buf.dt_hyp, buf.state, buf.s_out,
                                                    bp->smax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    BatchStageArgs a;
    a.grids = bp->grids;
    a.item_grid = bp->item_grid;
    a.state = buf.state;
    a.coef = buf.coef;
    a.T = buf.T;
    a.b = buf.b;
    a.Ya = buf.Ya;
    a.Yb = buf.Yb;
    a.MY0 = buf.MY0;
    for (int j = 1; j <= bp->smax; ++j) {
        a.stage = j;
        if (bp->precision == RKL_MIXED) launch_stage_b<float>(bp, a, st);
        else launch_stage_b<double>(bp, a, st);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rkl
