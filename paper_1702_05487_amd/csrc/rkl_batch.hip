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
// Persistent mode (rkl_set_batch_mode): three launches per super-step.  The
// reduce launch as above (it also clears each grid's completed-tile
// counter); a schedule launch (one workgroup) that lays out the work items
// -- (stage j, grid, tile) for every tile of every grid whose s reaches j,
// stage-major, so stage j of every grid comes after stage j-1 of every grid
// -- and clears the ticket counter; and one persistent launch whose
// workgroups take items in list order from an atomic ticket counter.  An item of stage j >= 2 of grid g first waits
// until all (j-1) x ntiles(g) tiles of stages 1..j-1 of g are complete
// (g's completed-tile counter, released at agent scope after each tile and
// acquired before the wait ends), then runs the tile and counts it.
// No wait depends on a workgroup that has not started: an item waits only
// for items earlier in the list, and items are handed out in list order, so
// the earliest unfinished item has every item it waits for finished and its
// workgroup (which took it, so is running) proceeds; no assumption about how
// many workgroups are resident at once is needed.  Every wait is bounded:
// after `timeout` wall-clock ticks a waiting workgroup sets the abort word and
// exits, every other workgroup exits at its next item or poll, and the plan
// reports RKL_FLAG_ABORTED.
//
// Tile shapes are chosen per grid by a tile policy (z-chunk length; full- or
// half-width rows, so that a patch narrower than 64 cells has no ragged x
// tiles); every tile runs the same run_tile code as the single-grid kernels,
// so neither the policy nor the mode changes the result.
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

// control words of the persistent launch (device)
struct PersistCtl {
    unsigned long long ticket;   // next item to hand out
    unsigned long long total;    // items of this super-step (schedule launch)
    unsigned int abort;          // set by a workgroup whose wait gave up
    unsigned int pad;
};

constexpr int kPersistSmax = 256;   // stage counts the persistent schedule handles

struct BatchPlan {
    int ngrids = 0, precision = 0, smax = 0, items = 0;
    int limiter = 0, saturation = 0, kmode = 0;
    BatchGrid* grids = nullptr;   // device
    int2* items_dev = nullptr;    // device, item -> (grid, tile), largest grids first
    // persistent mode (allocated on first use)
    int* by_size = nullptr;       // device, grid ids, largest grid first
    int* order = nullptr;         // device, grids by stage count (schedule launch)
    int* tprefix = nullptr;       // device, ngrids + 1 tile prefix sums over `order`
    int2* tiles = nullptr;        // device, items: (grid, tile) in `order`
    unsigned long long* base = nullptr;   // device, smax + 2: first ticket of stage j
    PersistCtl* ctl = nullptr;    // device
    unsigned int* done = nullptr; // device, ngrids completed-tile counters
    int persist_blocks = 0;       // workgroups of the persistent launch
    long long timeout = 0;        // wall-clock ticks a wait may last
    std::vector<int> by_size_host;
};

// one workgroup per grid: extrema of T, then dt_par and s for that grid
__global__ __launch_bounds__(kBT) void batch_reduce_kernel(const BatchGrid* __restrict__ grids,
                                                           const double* __restrict__ T,
                                                           const double* __restrict__ dt_hyp,
                                                           GridState* state, int32_t* s_out, int smax,
                                                           unsigned int* done) {
    const int g = blockIdx.x;
    if (done && threadIdx.x == 0) done[g] = 0u;
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
    a.fixed = 0;         // batched plans take no fixed axes
    a.ext = 0;
    for (int i = 0; i < 6; ++i) a.gh[i] = nullptr;
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

// Schedule of the persistent launch (one workgroup).  The grids are ordered
// by stage count, largest first, stable over the largest-grid-first order
// (a counting sort: histogram, bucket starts, then the grids in chunks of
// kBT, each placed after the grids of its bucket in earlier chunks and in
// the same chunk before it).  cnt(j) counts the grids that reach stage j, so
// stage j's items are the tiles of the first cnt(j) grids of that order --
// a prefix of one list of all tiles in that order -- and the stages are laid
// out one after another from ticket base[j].  Grids flagged at the reduce
// step (s above smax, or a bad dt_hyp) have no items.
__device__ __forceinline__ int stage_bucket(const GridState& st, int smax) {
    return (st.flags & RKL_FLAG_STAGES) || st.s < 2 || st.s > smax ? 0 : st.s;
}

__global__ __launch_bounds__(kBT) void batch_schedule_kernel(const BatchGrid* __restrict__ grids,
                                                             const int* __restrict__ by_size,
                                                             const GridState* __restrict__ state, int ngrids,
                                                             int smax, int* order, int* tprefix, int2* tiles,
                                                             unsigned long long* base, PersistCtl* ctl) {
    __shared__ int cnt[kPersistSmax + 2];        // histogram, then grids with s >= j
    __shared__ int pos[kPersistSmax + 2];        // next free place of each bucket
    __shared__ int key[kBT];                     // buckets of the current chunk
    __shared__ int part[kBT];                    // scan scratch
    __shared__ int carry;
    const int tid = threadIdx.x;
    for (int j = tid; j <= smax + 1; j += kBT) { cnt[j] = 0; pos[j] = 0; }
    __syncthreads();
    for (int g = tid; g < ngrids; g += kBT) atomicAdd(&cnt[stage_bucket(state[g], smax)], 1);
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int v = smax; v >= 0; --v) { pos[v] = acc; acc += cnt[v]; }
        int ge = 0;
        for (int v = smax; v >= 1; --v) { ge += cnt[v]; cnt[v] = ge; }   // grids with s >= v
    }
    __syncthreads();
    // stable scatter in chunks of kBT grids
    for (int c = 0; c < ngrids; c += kBT) {
        const int k = c + tid;
        const int g = k < ngrids ? by_size[k] : -1;
        const int v = g >= 0 ? stage_bucket(state[g], smax) : -1;
        key[tid] = v;
        __syncthreads();
        if (g >= 0) {
            int rank = 0;
            for (int t = 0; t < tid; ++t) rank += key[t] == v;
            order[pos[v] + rank] = g;
        }
        __syncthreads();
        if (tid == 0)
            for (int t = 0; t < kBT; ++t)
                if (key[t] >= 0) pos[key[t]] += 1;
        __syncthreads();
    }
    // tprefix: exclusive scan of the tile counts over the order, in chunks
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int c = 0; c < ngrids; c += kBT) {
        const int k = c + tid;
        const int nt = k < ngrids ? grids[order[k]].ntiles : 0;
        part[tid] = nt;
        __syncthreads();
        for (int off = 1; off < kBT; off <<= 1) {   // inclusive Hillis-Steele scan
            const int add = tid >= off ? part[tid - off] : 0;
            __syncthreads();
            part[tid] += add;
            __syncthreads();
        }
        if (k < ngrids) tprefix[k] = carry + part[tid] - nt;
        __syncthreads();
        if (tid == kBT - 1) carry += part[tid];
        __syncthreads();
    }
    if (tid == 0) {
        tprefix[ngrids] = carry;
        unsigned long long b = 0;
        for (int j = 1; j <= smax; ++j) { base[j] = b; b += (unsigned long long)tprefix[cnt[j]]; }
        base[0] = 0;
        base[smax + 1] = b;
        ctl->ticket = 0ull;
        ctl->total = b;
        ctl->abort = 0u;
    }
    __syncthreads();
    // the tile list: each thread writes the tiles of its grids
    for (int i = tid; i < cnt[1]; i += kBT) {
        const int g = order[i], nt = grids[g].ntiles;
        int2* w = tiles + tprefix[i];
        for (int t = 0; t < nt; ++t) w[t] = make_int2(g, t);
    }
}

template <typename R, bool LIM, int SAT, int KM>
__global__ __launch_bounds__(kBT) void batch_persistent_kernel(BatchBufs P, const int2* __restrict__ tiles,
                                                               const unsigned long long* __restrict__ base,
                                                               int smax, PersistCtl* ctl, unsigned int* done,
                                                               long long timeout) {
    __shared__ TileLds<R, Cap<R>::PL, Cap<R>::FX, Cap<R>::FY> L;
    __shared__ unsigned long long sbase[kPersistSmax + 2];
    __shared__ int3 item;   // (stage, grid, tile)
    __shared__ int ok;
    for (int j = threadIdx.x; j <= smax + 1; j += kBT) sbase[j] = base[j];
    const unsigned long long total = ctl->total;
    int j = 1;   // stage of the last ticket (tickets only grow)
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) {
            int go = 0;
            int3 it = make_int3(0, 0, 0);
            if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
                const unsigned long long t =
                    __hip_atomic_fetch_add(&ctl->ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (t < total) {
                    while (t >= sbase[j + 1]) ++j;
                    const int2 gt = tiles[t - sbase[j]];
                    it = make_int3(j, gt.x, gt.y);
                    go = 1;
                    if (j >= 2) {
                        // stages 1..j-1 of this grid complete: (j-1) x ntiles tiles counted
                        const unsigned int need = (unsigned int)(j - 1) * (unsigned int)P.grids[gt.x].ntiles;
                        const long long t0 = wall_clock64();
                        while (__hip_atomic_load(&done[gt.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                            if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                                go = 0;
                                break;
                            }
                            if (wall_clock64() - t0 > timeout) {
                                __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                go = 0;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(8);
                        }
                        // the other workgroups' stage outputs are visible from here on
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    }
                }
            }
            item = it;
            ok = go;
        }
        __syncthreads();
        if (!ok) break;   // uniform over the workgroup
        const int3 it = item;
        const GridState st = P.state[it.y];
        batch_tile<R, LIM, SAT, KM>(P, it.y, it.x, it.z, st, L);
        __syncthreads();
        // every store of the tile is done; publish it with the count
        if (threadIdx.x == 0) __hip_atomic_fetch_add(&done[it.y], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
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
    bp->by_size_host = by_size;
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
    (void)hipFree(bp->by_size);
    (void)hipFree(bp->order);
    (void)hipFree(bp->tprefix);
    (void)hipFree(bp->tiles);
    (void)hipFree(bp->base);
    (void)hipFree(bp->ctl);
    (void)hipFree(bp->done);
    delete bp;
}

template <typename R, bool LIM, int KM>
static const void* persistent_fn(int sat) {
    if (sat == 2) return (const void*)batch_persistent_kernel<R, LIM, 2, KM>;
    if (sat == 1) return (const void*)batch_persistent_kernel<R, LIM, 1, KM>;
    return (const void*)batch_persistent_kernel<R, LIM, 0, KM>;
}

template <typename R>
static const void* persistent_fn(const BatchPlan* bp) {
    const bool lim = bp->limiter != 0;
    if (bp->kmode == 0) return lim ? persistent_fn<R, true, 0>(bp->saturation) : persistent_fn<R, false, 0>(bp->saturation);
    if (bp->kmode == 1) return lim ? persistent_fn<R, true, 1>(bp->saturation) : persistent_fn<R, false, 1>(bp->saturation);
    return lim ? persistent_fn<R, true, 2>(bp->saturation) : persistent_fn<R, false, 2>(bp->saturation);
}

rkl_status batch_persist_init(BatchPlan* bp, std::string& why) {
    if (bp->ctl) return RKL_OK;
    if (bp->smax > kPersistSmax) {
        why = "the persistent batched launch needs smax <= " + std::to_string(kPersistSmax);
        return RKL_EINVAL;
    }
    const int n = bp->ngrids;
    bool ok = hipMalloc(&bp->by_size, sizeof(int) * n) == hipSuccess &&
              hipMalloc(&bp->order, sizeof(int) * n) == hipSuccess &&
              hipMalloc(&bp->tprefix, sizeof(int) * (n + 1)) == hipSuccess &&
              hipMalloc(&bp->tiles, sizeof(int2) * (size_t)bp->items) == hipSuccess &&
              hipMalloc(&bp->base, sizeof(unsigned long long) * (kPersistSmax + 2)) == hipSuccess &&
              hipMalloc(&bp->ctl, sizeof(PersistCtl)) == hipSuccess &&
              hipMalloc(&bp->done, sizeof(unsigned int) * n) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        why = "device allocation failed (persistent batched launch)";
        return RKL_ENOMEM;
    }
    const PersistCtl zero{0ull, 0ull, 0u, 0u};
    int dev = 0, cus = 0, per_cu = 0, rate_khz = 0;
    hipError_t e = hipMemcpy(bp->by_size, bp->by_size_host.data(), sizeof(int) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bp->ctl, &zero, sizeof zero, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, bp->precision == RKL_MIXED ? persistent_fn<float>(bp) : persistent_fn<double>(bp), kBT, 0);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipGetLastError();
        why = std::string("persistent launch set-up: ") + hipGetErrorString(e);
        return RKL_EDEVICE;
    }
    bp->persist_blocks = std::max(1, per_cu) * std::max(1, cus);
    // a wait longer than 2 s means something is wrong: give up (a whole
    // super-step of the largest workloads takes a few tens of milliseconds)
    if (rate_khz <= 0) rate_khz = 100000;   // the usual 100 MHz counter
    bp->timeout = (long long)rate_khz * 2000ll;
    return RKL_OK;
}

hipError_t batch_aborted(const BatchPlan* bp, bool* aborted) {
    *aborted = false;
    if (!bp || !bp->ctl) return hipSuccess;
    PersistCtl h;
    hipError_t e = hipMemcpy(&h, bp->ctl, sizeof h, hipMemcpyDeviceToHost);
    if (e == hipSuccess) *aborted = h.abort != 0u;
    return e;
}

template <typename R, bool LIM, int KM>
static void launch_persist_sat(const BatchPlan* bp, const BatchBufs& a, hipStream_t st) {
    const int nb = bp->persist_blocks;
    if (bp->saturation == 2)
        batch_persistent_kernel<R, LIM, 2, KM><<<nb, kBT, 0, st>>>(a, bp->tiles, bp->base, bp->smax, bp->ctl,
                                                                   bp->done, bp->timeout);
    else if (bp->saturation == 1)
        batch_persistent_kernel<R, LIM, 1, KM><<<nb, kBT, 0, st>>>(a, bp->tiles, bp->base, bp->smax, bp->ctl,
                                                                   bp->done, bp->timeout);
    else
        batch_persistent_kernel<R, LIM, 0, KM><<<nb, kBT, 0, st>>>(a, bp->tiles, bp->base, bp->smax, bp->ctl,
                                                                   bp->done, bp->timeout);
}

template <typename R>
static void launch_persist(const BatchPlan* bp, const BatchBufs& a, hipStream_t st) {
    const bool lim = bp->limiter != 0;
    if (bp->kmode == 0) { if (lim) launch_persist_sat<R, true, 0>(bp, a, st); else launch_persist_sat<R, false, 0>(bp, a, st); }
    else if (bp->kmode == 1) { if (lim) launch_persist_sat<R, true, 1>(bp, a, st); else launch_persist_sat<R, false, 1>(bp, a, st); }
    else { if (lim) launch_persist_sat<R, true, 2>(bp, a, st); else launch_persist_sat<R, false, 2>(bp, a, st); }
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
                        std::vector<std::pair<hipEvent_t, hipEvent_t>>* events, int mode) {
    const bool persist = mode == 1;
    if (persist && !bp->ctl) return hipErrorNotInitialized;
    batch_reduce_kernel<<<bp->ngrids, kBT, 0, st>>>(bp->grids, buf.T, buf.dt_hyp, buf.state, buf.s_out,
                                                    bp->smax, persist ? bp->done : nullptr);
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
    if (persist) {
        batch_schedule_kernel<<<1, kBT, 0, st>>>(bp->grids, bp->by_size, buf.state, bp->ngrids, bp->smax, bp->order,
                                                 bp->tprefix, bp->tiles, bp->base, bp->ctl);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (events) {
            if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
            if ((e = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return e; }
            events->push_back({e0, e1});
            if ((e = hipEventRecord(e0, st)) != hipSuccess) return e;
        }
        if (bp->precision == RKL_MIXED) launch_persist<float>(bp, a, st);
        else launch_persist<double>(bp, a, st);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (e1 && (e = hipEventRecord(e1, st)) != hipSuccess) return e;
        return hipSuccess;
    }
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
