// rkl_batch.hip -- one RKL2 super-step of many independent grids
// ("patches") of uneven size, each with its own field, super-step and stage
// count, without host synchronisation (graph-capturable).
//
// Launch sequence per super-step: one reduce launch (a workgroup per grid
// computes that grid's temperature extrema, dt_par and stage count s_g on the
// device), then one launch per stage j = 1..smax over every tile of every
// grid; a tile whose grid has s_g < j returns at once.  Stage j of every grid
// therefore starts only after stage j-1 of every grid has finished, with
// kernel boundaries as the only synchronisation between workgroups.  Tiles
// are dispatched largest grid first so that the small tiles fill the tail of
// each launch.
//
// Tile shapes are chosen per grid by a tile policy (z-chunk length; full- or
// half-width rows, so that a patch narrower than 64 cells has no ragged x
// tiles); every tile runs the same run_tile code as the single-grid kernels,
// so the policy never changes the result.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "rkl_batch.h"
#include "rkl_tile.h"

namespace rkl {

constexpr int kBT = 256;        // threads per batched workgroup

// LDS capacities of the batched tile, per element type: a plane (bx+2)(by+2),
// x faces (bx+1) by and y faces bx (by+1) per buffer.  In FP64 the plane
// capacity keeps the tile's 15 planes and 4 face buffers at 51.5 KB, so that
// three workgroups share the 160 KB of a CU, as many as the FP64 kernel's
// registers allow; tiles whose rows are too wide for it get fewer rows.
template <typename R>
struct Cap {
    static constexpr int PL = 400, FX = 320, FY = 320;
};
template <>
struct Cap<double> {
    static constexpr int PL = 344, FX = 320, FY = 320;
};

struct BatchGrid {
    GridConst gc;
    int64_t off;
    int bx, by, bz, ntx, nty, nzc;
    int ntiles;
};

struct BatchPlan {
    int ngrids = 0, precision = 0, smax = 0, items = 0;
    int limiter = 0, saturation = 0, kmode = 0;
    BatchGrid* grids = nullptr;   // device
    int2* items_dev = nullptr;    // device, item -> (grid, tile), largest grids first
};

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

struct BatchBufs {
    const BatchGrid* grids;
    const GridState* state;
    const double* coef;
    double* T;
    const void* b;
    double* Ya;
    double* Yb;
    void* MY0;
};

// stage j of tile t of grid g
template <typename R, bool LIM, int SAT, int KM, typename L_t>
__device__ __forceinline__ void batch_tile(const BatchBufs& P, int g, int j, int t, const GridState& st,
                                           L_t& L) {
    const BatchGrid& G = P.grids[g];
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
    a.bc = G.gc.bc;
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
    const FaceK<R> fk = make_facek<R>(G.gc.kappa0, G.gc.kexp, G.gc.kperp, G.gc.satq, tref);
    run_tile<R, LIM, SAT, KM>(a, fk, tref, L);
}

template <typename R, bool LIM, int SAT, int KM>
__global__ __launch_bounds__(kBT) void batch_stage_kernel(BatchBufs P, const int2* __restrict__ items,
                                                          int stage) {
    __shared__ TileLds<R, Cap<R>::PL, Cap<R>::FX, Cap<R>::FY> L;
    const int2 it = items[xcd_remap(blockIdx.x, gridDim.x)];
    const GridState st = P.state[it.x];
    if (st.s < stage || (st.flags & RKL_FLAG_STAGES)) return;   // uniform over the block
    batch_tile<R, LIM, SAT, KM>(P, it.x, stage, it.y, st, L);
}

// Tile policies of the batched launch: z-chunk length and row width.  Rows
// are the grid's full width (up to 64 cells), or half of it for grids wider
// than 32 cells (twice the tiles, shorter halo rows); by fills the 256
// threads, as far as the plane fits the precision's LDS capacity.
struct BatchPolicy {
    int half_rows;
    int bz;
};
static const BatchPolicy kPolicies[] = {{0, 32}, {0, 16}, {0, 64}, {1, 32}, {1, 16}, {1, 64}};

int batch_policy_count() { return (int)(sizeof(kPolicies) / sizeof(kPolicies[0])); }

void batch_policy_info(int policy, int* half_rows, int* bz) {
    *half_rows = kPolicies[policy].half_rows;
    *bz = kPolicies[policy].bz;
}

static void choose_tile(const GridConst& g, int policy, int plcap, int& bx, int& by, int& bz) {
    const BatchPolicy& P = kPolicies[policy];
    bx = std::min(g.n0, 64);
    if (P.half_rows && g.n0 > 32) bx = std::min((g.n0 + 1) / 2, 32);
    by = std::min(std::min(g.n1, kBT / bx), 64);
    while (by > 1 && (bx + 2) * (by + 2) > plcap) --by;
    bz = std::min(g.n2, P.bz);
}

rkl_status batch_create(const std::vector<rkl_grid_desc>& desc, const std::vector<GridConst>& gc,
                        const std::vector<int64_t>& off, int precision, int smax, int policy,
                        BatchPlan** out, std::string& why) {
    *out = nullptr;
    if (policy < 0 || policy >= batch_policy_count()) {
        why = "batched tile policy out of range";
        return RKL_EINVAL;
    }
    const bool f32 = precision == RKL_MIXED;
    const int plcap = f32 ? Cap<float>::PL : Cap<double>::PL;
    const int fxcap = f32 ? Cap<float>::FX : Cap<double>::FX;
    const int fycap = f32 ? Cap<float>::FY : Cap<double>::FY;
    const int n = (int)desc.size();
    std::vector<BatchGrid> h(n);
    int64_t items = 0;
    for (int g = 0; g < n; ++g) {
        if (desc[g].limiter != desc[0].limiter || desc[g].saturation != desc[0].saturation ||
            gc[g].kmode != gc[0].kmode) {
            why = "batched grids must share the limiter and saturation settings and the kind of "
                  "conductivity law (kappa_exp 0, 2.5 or other)";
            return RKL_EINVAL;
        }
        BatchGrid& B = h[g];
        B.gc = gc[g];
        B.off = off[g];
        choose_tile(gc[g], policy, plcap, B.bx, B.by, B.bz);
        if ((B.bx + 2) * (B.by + 2) > plcap || (B.bx + 1) * B.by > fxcap || B.bx * (B.by + 1) > fycap ||
            2 * B.bx + 2 * B.by + 4 > kBT) {
            why = "internal: batched tile shape exceeds the LDS layout";
            return RKL_EINVAL;
        }
        B.ntx = (gc[g].n0 + B.bx - 1) / B.bx;
        B.nty = (gc[g].n1 + B.by - 1) / B.by;
        B.nzc = (gc[g].n2 + B.bz - 1) / B.bz;
        const int64_t nt = (int64_t)B.ntx * B.nty * B.nzc;
        if (items + nt > (int64_t)0x7fffffff) { why = "too many tiles"; return RKL_EINVAL; }
        B.ntiles = (int)nt;
        items += nt;
    }
    // items ordered by grid size, largest first, so that a launch ends on small tiles
    std::vector<int> by_size(n);
    std::iota(by_size.begin(), by_size.end(), 0);
    std::stable_sort(by_size.begin(), by_size.end(), [&](int a, int b) {
        return (int64_t)gc[a].n0 * gc[a].n1 * gc[a].n2 > (int64_t)gc[b].n0 * gc[b].n1 * gc[b].n2;
    });
    std::vector<int2> item_list;
    item_list.reserve((size_t)items);
    for (int g : by_size)
        for (int t = 0; t < h[g].ntiles; ++t) item_list.push_back(make_int2(g, t));

    BatchPlan* bp = new BatchPlan();
    bp->ngrids = n;
    bp->precision = precision;
    bp->smax = smax;
    bp->items = (int)items;
    bp->limiter = desc[0].limiter;
    bp->saturation = desc[0].saturation;
    bp->kmode = gc[0].kmode;
    if (hipMalloc(&bp->grids, sizeof(BatchGrid) * n) != hipSuccess ||
        hipMalloc(&bp->items_dev, sizeof(int2) * item_list.size()) != hipSuccess) {
        (void)hipGetLastError();
        batch_free(bp);
        why = "device allocation failed";
        return RKL_ENOMEM;
    }
    if (hipMemcpy(bp->grids, h.data(), sizeof(BatchGrid) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(bp->items_dev, item_list.data(), sizeof(int2) * item_list.size(), hipMemcpyHostToDevice) !=
            hipSuccess) {
        (void)hipGetLastError();
        batch_free(bp);
        why = "batched plan upload failed";
        return RKL_EDEVICE;
    }
    *out = bp;
    return RKL_OK;
}

void batch_free(BatchPlan* bp) {
    if (!bp) return;
    (void)hipFree(bp->grids);
    (void)hipFree(bp->items_dev);
    delete bp;
}

template <typename R, bool LIM, int KM>
static void launch_stage_sat(const BatchPlan* bp, const BatchBufs& a, int stage, hipStream_t st) {
    const int2* it = bp->items_dev;
    if (bp->saturation == 2) batch_stage_kernel<R, LIM, 2, KM><<<bp->items, kBT, 0, st>>>(a, it, stage);
    else if (bp->saturation == 1) batch_stage_kernel<R, LIM, 1, KM><<<bp->items, kBT, 0, st>>>(a, it, stage);
    else batch_stage_kernel<R, LIM, 0, KM><<<bp->items, kBT, 0, st>>>(a, it, stage);
}

template <typename R, int KM>
static void launch_stage_km(const BatchPlan* bp, const BatchBufs& a, int stage, hipStream_t st) {
    if (bp->limiter != 0) launch_stage_sat<R, true, KM>(bp, a, stage, st);
    else launch_stage_sat<R, false, KM>(bp, a, stage, st);
}

template <typename R>
static void launch_stage_b(const BatchPlan* bp, const BatchBufs& a, int stage, hipStream_t st) {
    if (bp->kmode == 0) launch_stage_km<R, 0>(bp, a, stage, st);
    else if (bp->kmode == 1) launch_stage_km<R, 1>(bp, a, stage, st);
    else launch_stage_km<R, 2>(bp, a, stage, st);
}

hipError_t batch_launch(BatchPlan* bp, const BatchBuffers& buf, hipStream_t st,
                        std::vector<std::pair<hipEvent_t, hipEvent_t>>* events) {
    batch_reduce_kernel<<<bp->ngrids, kBT, 0, st>>>(bp->grids, buf.T, buf.dt_hyp, buf.state, buf.s_out,
                                                    bp->smax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    BatchBufs a;
    a.grids = bp->grids;
    a.state = buf.state;
    a.coef = buf.coef;
    a.T = buf.T;
    a.b = buf.b;
    a.Ya = buf.Ya;
    a.Yb = buf.Yb;
    a.MY0 = buf.MY0;
    for (int j = 1; j <= bp->smax; ++j) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (events && j >= 2) {
            if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
            if ((e = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return e; }
            events->push_back({e0, e1});
            if ((e = hipEventRecord(e0, st)) != hipSuccess) return e;
        }
        if (bp->precision == RKL_MIXED) launch_stage_b<float>(bp, a, j, st);
        else launch_stage_b<double>(bp, a, j, st);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (e1 && (e = hipEventRecord(e1, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rkl
