// rkl_api.hip -- host side of librkl's C ABI (include/rkl.h): descriptor
// validation, plan scratch, the RKL2 coefficient table, and the launch
// sequences of the single-grid entry points.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/rkl.h"
#include "rkl_internal.h"
#include "rkl_batch.h"
#include "rkl_host.h"

using namespace rkl;

static thread_local std::string g_err;

rkl_status rkl::fail(rkl_status st, const std::string& msg) {
    g_err = msg;
    return st;
}
rkl_status rkl::hipfail(hipError_t e, const char* what) {
    return fail(RKL_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCHECK(call, what)                   \
    do {                                       \
        hipError_t e_ = (call);                \
        if (e_ != hipSuccess) return hipfail(e_, what); \
    } while (0)

struct rkl_plan_s {
    int device = 0;
    int ngrids = 0;
    int precision = RKL_FP64;
    int variant = 0;
    int smax = 1024;
    int scheme = RKL_RKL2;
    std::vector<rkl_grid_desc> desc;
    std::vector<GridConst> gc;
    std::vector<int64_t> off;   // packed cell offsets, ngrids + 1 entries
    int64_t total = 0;
    double* Ya = nullptr;       // stage buffers (FP64), packed
    double* Yb = nullptr;
    double* Yc = nullptr;       // two more, allocated once a two-stage variant is selected
    double* Yd = nullptr;
    void* MY0 = nullptr;        // tau M(Y0), FP64 or FP32, packed
    double* coef = nullptr;     // RKL2 table, device
    GridState* state = nullptr; // ngrids entries, device
    double* partials = nullptr; // 3 x 1024 doubles
    double* ext_part = nullptr; // 3 per workgroup of a one-stage launch, the largest over grids and variants
    int32_t* ext_ok = nullptr;  // ngrids flags: ext_part holds the extrema of the grid's T
    int32_t* s_dev = nullptr;   // scratch for the stage-count read-back
    int32_t* s_host = nullptr;  // pinned
    BatchPlan* batch = nullptr; // batched launch data (rkl_batch.hip)
    int batch_policy = 0;       // its tile policy
    int batch_mode = 0;         // 0: one launch per stage; 1: one persistent launch
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    // kernel timing (rkl_profile): one event pair per stencil launch of
    // stage j >= 2, tagged with its stages per launch and cell-stages
    struct ProfRec {
        hipEvent_t a, b;
        int fuse;
        int64_t cells;
    };
    bool prof = false;
    std::vector<ProfRec> prof_recs;
};

static void prof_clear(rkl_plan_s* p) {
    for (auto& r : p->prof_recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    p->prof_recs.clear();
}

// ---------------------------------------------------------------------------
// RKL2 coefficients (Appendix A, rkl2_row in rkl_internal.h): row j of s
// holds {mu_j, nu_j, 1 - mu_j - nu_j, mut_j, gt_j} at 5 (s(s+1)/2 + j).
// RKL1 (Sec. 3.3: P_s(1 + w1 z), w1 = 2/(s^2+s), Legendre recursion): mut_1 =
// w1; mu_j = (2j-1)/j, nu_j = -(j-1)/j, mut_j = mu_j w1, and no Y0 or tau
// M(Y0) term (1 - mu_j - nu_j = 0, gt_j = 0).
static std::vector<double> coefficient_table(int smax, int scheme) {
    const size_t rows = (size_t)(smax + 1) * (smax + 2) / 2;
    std::vector<double> t(rows * 5, 0.0);
    if (scheme == RKL_RKL1) {
        for (int s = 1; s <= smax; ++s) {
            const double w1 = 2.0 / ((double)s * s + s);
            double* row = &t[5 * ((size_t)s * (s + 1) / 2)];
            row[5 * 1 + 3] = w1;
            for (int j = 2; j <= s; ++j) {
                double* r = row + 5 * j;
                r[0] = (2.0 * j - 1.0) / j;
                r[1] = -(j - 1.0) / j;
                r[2] = 0.0;
                r[3] = r[0] * w1;
                r[4] = 0.0;
            }
        }
        return t;
    }
    for (int s = 2; s <= smax; ++s)
        for (int j = 1; j <= s; ++j) rkl2_row(s, j, &t[5 * ((size_t)s * (s + 1) / 2 + j)]);
    return t;
}

bool rkl::validate(const rkl_grid_desc& g, std::string& why) {
    char buf[160];
    if (g.ndim < 1 || g.ndim > 3) { why = "ndim must be 1, 2 or 3"; return false; }
    for (int d = 0; d < 3; ++d) {
        if (g.n[d] < 1) { snprintf(buf, sizeof buf, "n[%d] = %d must be >= 1", d, g.n[d]); why = buf; return false; }
        if (d >= g.ndim && g.n[d] != 1) { snprintf(buf, sizeof buf, "n[%d] must be 1 when ndim = %d", d, g.ndim); why = buf; return false; }
        if (!(g.h[d] > 0.0) || !std::isfinite(g.h[d])) { snprintf(buf, sizeof buf, "h[%d] must be finite and > 0", d); why = buf; return false; }
    }
    if ((int64_t)g.n[0] * g.n[1] > (int64_t)1 << 30 ||
        (int64_t)g.n[0] * g.n[1] * g.n[2] > ((int64_t)1 << 32)) { why = "grid too large"; return false; }
    if (g.limiter != RKL_LIM_NONE && g.limiter != RKL_LIM_MC) { why = "limiter must be RKL_LIM_NONE or RKL_LIM_MC"; return false; }
    if (g.saturation < 0 || g.saturation > 2) { why = "saturation must be 0, 1 or 2"; return false; }
    if (g.saturation && !(g.phi > 0.0 && std::isfinite(g.phi))) { why = "phi must be > 0"; return false; }
    if (!(g.kappa0 >= 0.0) || !std::isfinite(g.kappa0)) { why = "kappa0 must be finite and >= 0"; return false; }
    if (!(g.kappa_exp >= 0.0) || !std::isfinite(g.kappa_exp)) { why = "kappa_exp must be finite and >= 0"; return false; }
    if (!(g.kperp_ratio >= 0.0 && g.kperp_ratio <= 1.0)) { why = "kperp_ratio must be in [0, 1]"; return false; }
    if (!(g.rho > 0.0) || !std::isfinite(g.rho)) { why = "rho must be finite and > 0"; return false; }
    if (!(g.gamma > 1.0) || !std::isfinite(g.gamma)) { why = "gamma must be finite and > 1"; return false; }
    if (!(g.cp > 0.0 && g.cp <= 0.5)) { why = "cp must be in (0, 1/2]"; return false; }
    for (int d = 0; d < 3; ++d) {
        if (g.boundary[d] != RKL_BC_PERIODIC && g.boundary[d] != RKL_BC_OUTFLOW && g.boundary[d] != RKL_BC_FIXED) {
            snprintf(buf, sizeof buf, "boundary[%d] must be RKL_BC_PERIODIC, RKL_BC_OUTFLOW or RKL_BC_FIXED", d);
            why = buf;
            return false;
        }
        if (g.boundary[d] == RKL_BC_FIXED && d >= g.ndim) {
            snprintf(buf, sizeof buf, "boundary[%d] = RKL_BC_FIXED needs ndim > %d", d, d);
            why = buf;
            return false;
        }
    }
    return true;
}

GridConst rkl::make_const(const rkl_grid_desc& g, int scheme) {
    GridConst c;
    c.n0 = g.n[0];
    c.n1 = g.n[1];
    c.n2 = g.n[2];
    c.ndim = g.ndim;
    c.ih0 = 1.0 / g.h[0];
    c.ih1 = 1.0 / g.h[1];
    c.ih2 = 1.0 / g.h[2];
    c.kappa0 = g.kappa0;
    c.kexp = g.kappa_exp;
    c.kperp = g.kperp_ratio;
    c.satq = 5.0 * g.phi * g.rho;
    c.kmode = g.kappa_exp == 0.0 ? 0 : (g.kappa_exp == 2.5 ? 1 : 2);
    c.limiter = g.limiter;
    c.saturation = g.saturation;
    c.scheme = scheme;
    c.bc = (g.boundary[0] ? 1 : 0) | (g.boundary[1] ? 2 : 0) | (g.boundary[2] ? 4 : 0);
    c.fixed = 0;
    for (int d = 0; d < 3; ++d) c.fixed |= g.boundary[d] == RKL_BC_FIXED ? 1 << d : 0;
    for (int i = 0; i < 6; ++i) c.gh[i] = nullptr;
    c.fac = (g.gamma - 1.0) / g.rho;
    c.cp = g.cp;
    double s = 0.0;
    for (int d = 0; d < g.ndim; ++d) s += 1.0 / (g.h[d] * g.h[d]);
    c.ihsum = s;
    return c;
}

static void free_plan(rkl_plan_s* p) {
    if (!p) return;
    prof_clear(p);
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    batch_free(p->batch);
    (void)hipFree(p->Ya);
    (void)hipFree(p->Yb);
    (void)hipFree(p->Yc);
    (void)hipFree(p->Yd);
    (void)hipFree(p->MY0);
    (void)hipFree(p->coef);
    (void)hipFree(p->state);
    (void)hipFree(p->partials);
    (void)hipFree(p->ext_part);
    (void)hipFree(p->ext_ok);
    (void)hipFree(p->s_dev);
    if (p->s_host) (void)hipHostFree(p->s_host);
    delete p;
}

static rkl_status ensure_batch(rkl_plan_s* p) {
    if (!p->batch) {
        // the batched stage routing writes stage j = s into T, which needs s >= 2
        if (p->scheme != RKL_RKL2) return fail(RKL_EINVAL, "the batched super-step implements RKL2 only");
        std::string why;
        rkl_status st = batch_create(p->desc, p->gc, p->off, p->precision, p->smax, p->batch_policy, &p->batch, why);
        if (st != RKL_OK) return fail(st, why);
    }
    if (p->batch_mode == 1) {
        std::string why;
        rkl_status st = batch_persist_init(p->batch, why);
        if (st != RKL_OK) return fail(st, why);
    }
    return RKL_OK;
}

// A plan's buffers live on the device that was current at rkl_plan; its
// launches must go to that device.
static rkl_status check_plan(const rkl_plan_s* p) {
    if (!p) return fail(RKL_EINVAL, "plan is NULL");
    int d = -1;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return hipfail(e, "hipGetDevice");
    if (d != p->device)
        return fail(RKL_EINVAL, "the plan belongs to device " + std::to_string(p->device) + ", device " +
                                    std::to_string(d) + " is current");
    return RKL_OK;
}

static void drop_graph(rkl_plan_s* p) {
    if (p->graph_exec) { (void)hipGraphExecDestroy(p->graph_exec); p->graph_exec = nullptr; }
    if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
}

// Replace the batched launch data by that of `policy`; a captured graph
// refers to the old data, so it is dropped.
static rkl_status select_batch_policy(rkl_plan_s* p, int policy) {
    if (p->batch && policy == p->batch_policy) return RKL_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hipfail(e, "policy sync");
    drop_graph(p);
    batch_free(p->batch);
    p->batch = nullptr;
    p->batch_policy = policy;
    return ensure_batch(p);
}

// Select the batched launch mode; a captured graph holds the old launch
// sequence, so it is dropped.
static rkl_status select_batch_mode(rkl_plan_s* p, int mode) {
    if (mode == p->batch_mode) return ensure_batch(p);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hipfail(e, "mode sync");
    drop_graph(p);
    const int old = p->batch_mode;
    p->batch_mode = mode;
    rkl_status st = ensure_batch(p);
    if (st != RKL_OK) p->batch_mode = old;
    return st;
}

// a stencil call on grid g: every fixed axis needs its ghost layers
static rkl_status check_ghosts(rkl_plan_t p, int32_t g) {
    const GridConst& c = p->gc[g];
    for (int d = 0; d < 3; ++d)
        if ((c.fixed & (1 << d)) && (!c.gh[2 * d] || !c.gh[2 * d + 1]))
            return fail(RKL_EINVAL, "grid " + std::to_string(g) + ": fixed axis " + std::to_string(d) +
                                        " has no ghost layers (rkl_set_ghosts)");
    return RKL_OK;
}

// the batched kernels and the fused variants have no fixed-axis ghosts
static rkl_status check_no_fixed(rkl_plan_t p, const char* what) {
    for (int g = 0; g < p->ngrids; ++g)
        if (p->gc[g].fixed) return fail(RKL_EINVAL, std::string(what) + " does not take RKL_BC_FIXED axes");
    return RKL_OK;
}

extern "C" {

const char* rkl_last_error(void) { return g_err.c_str(); }

int32_t rkl_batch_policy_count(void) { return batch_policy_count(); }

rkl_status rkl_batch_policy_info(int32_t policy, int32_t* half_rows, int32_t* tile_z) {
    if (policy < 0 || policy >= batch_policy_count()) return fail(RKL_EINVAL, "policy out of range");
    int h = 0, z = 0;
    batch_policy_info(policy, &h, &z);
    if (half_rows) *half_rows = h;
    if (tile_z) *tile_z = z;
    return RKL_OK;
}

rkl_status rkl_set_batch_mode(rkl_plan_t p, int32_t mode) {
    if (rkl_status st = check_plan(p)) return st;
    if (mode != 0 && mode != 1) return fail(RKL_EINVAL, "batch mode must be 0 (per-stage launches) or 1 (persistent)");
    return select_batch_mode(p, mode);
}

rkl_status rkl_set_batch_policy(rkl_plan_t p, int32_t policy) {
    if (rkl_status st = check_plan(p)) return st;
    if (policy < 0 || policy >= batch_policy_count()) return fail(RKL_EINVAL, "policy out of range");
    return select_batch_policy(p, policy);
}

rkl_status rkl_autotune_batched(rkl_plan_t p, const double* T, const void* b, const double* dt_hyp,
                                int32_t reps, int32_t* best_policy, double* best_ms, void* stream) {
    if (rkl_status st = check_plan(p)) return st;
    if (rkl_status st = check_no_fixed(p, "the batched path")) return st;
    if (!T || !b || !dt_hyp) return fail(RKL_EINVAL, "NULL pointer");
    if ((const void*)T == b) return fail(RKL_EINVAL, "b must not alias T");
    if (reps < 1 || reps > 1000) return fail(RKL_EINVAL, "reps must be in [1, 1000]");
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = sizeof(double) * (size_t)p->total;
    double* W = nullptr;
    HIPCHECK(hipMalloc(&W, bytes), "autotune scratch");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool saved_prof = p->prof;
    const int saved = p->batch_policy, saved_mode = p->batch_mode;
    p->prof = false;
    int best = -1, best_mode = 0;
    float best_t = 0.f;
    rkl_status res = RKL_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) res = fail(RKL_EDEVICE, "autotune events");
    // every tile policy with per-stage launches, then with the persistent launch
    // (if the plan's smax allows it)
    for (int mode = 0; res == RKL_OK && mode < 2; ++mode) {
        if (mode == 1 && p->smax > 256) break;
        for (int pol = 0; res == RKL_OK && pol < batch_policy_count(); ++pol) {
            res = select_batch_policy(p, pol);
            if (res == RKL_OK) res = select_batch_mode(p, mode);
            if (res != RKL_OK) break;
            BatchBuffers bb{W, b, dt_hyp, nullptr, p->Ya, p->Yb, p->MY0, p->coef, p->state};
            // one untimed super-step from the caller's T, then reps timed ones
            hipError_t e = hipMemcpyAsync(W, T, bytes, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess) e = batch_launch(p->batch, bb, s, nullptr, mode);
            if (e == hipSuccess) e = hipMemcpyAsync(W, T, bytes, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            for (int r = 0; e == hipSuccess && r < reps; ++r) e = batch_launch(p->batch, bb, s, nullptr, mode);
            float t = 0.f;
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) { res = hipfail(e, "batched autotune"); break; }
            bool aborted = false;
            if (mode == 1 && (e = batch_aborted(p->batch, &aborted)) != hipSuccess) { res = hipfail(e, "abort word"); break; }
            if (aborted) continue;   // a persistent launch that gave up is never chosen
            if (best < 0 || t < best_t) { best = pol; best_mode = mode; best_t = t; }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(W);
    p->prof = saved_prof;
    if (res != RKL_OK || best < 0) {
        select_batch_policy(p, saved);
        select_batch_mode(p, saved_mode);
        return res != RKL_OK ? res : fail(RKL_EDEVICE, "batched autotune: no configuration completed");
    }
    res = select_batch_policy(p, best);
    if (res == RKL_OK) res = select_batch_mode(p, best_mode);
    if (res != RKL_OK) return res;
    if (best_policy) *best_policy = best + best_mode * batch_policy_count();
    if (best_ms) *best_ms = best_t / reps;
    return RKL_OK;
}

int32_t rkl_variant_count(void) { return variant_count(); }

rkl_status rkl_variant_info(int32_t v, int32_t* tx, int32_t* ty, int32_t* tz, int32_t* fuse) {
    if (v < 0 || v >= variant_count()) return fail(RKL_EINVAL, "variant out of range");
    const Variant x = variant_get(v);
    if (tx) *tx = x.bx;
    if (ty) *ty = x.by;
    if (tz) *tz = x.bz;
    if (fuse) *fuse = x.fuse;
    return RKL_OK;
}

// A fused variant (2 to 4 stages per launch) needs RKL_MIXED and periodic
// 3-D grids, and two more stage buffers (tiles overlap, so its outputs may
// not overwrite its inputs).
static bool fused_ok(const rkl_plan_s* p) {
    if (p->precision != RKL_MIXED) return false;
    for (const auto& d : p->desc)
        if (d.ndim != 3 || d.boundary[0] || d.boundary[1] || d.boundary[2]) return false;
    return true;
}

static bool variant_ok(const rkl_plan_s* p, const Variant& x) {
    return x.fuse >= 2 ? fused_ok(p) : true;
}

static rkl_status select_variant(rkl_plan_s* p, int v) {
    const Variant x = variant_get(v);
    if (x.fuse >= 2) {
        if (!fused_ok(p)) return fail(RKL_EINVAL, "fused variants need an RKL_MIXED plan of periodic 3-D grids");
        if (!p->Yc) {
            if (hipMalloc(&p->Yc, sizeof(double) * p->total) != hipSuccess ||
                hipMalloc(&p->Yd, sizeof(double) * p->total) != hipSuccess) {
                (void)hipGetLastError();
                (void)hipFree(p->Yc);
                p->Yc = nullptr;
                return fail(RKL_ENOMEM, "stage buffer allocation failed");
            }
        }
    }
    p->variant = v;
    return RKL_OK;
}

rkl_status rkl_plan(const rkl_grid_desc* grids, int32_t ngrids, const rkl_options* opt, rkl_plan_t* out) {
    if (!out) return fail(RKL_EINVAL, "plan_out is NULL");
    *out = nullptr;
    if (!grids || ngrids < 1) return fail(RKL_EINVAL, "need at least one grid descriptor");
    rkl_options o = {RKL_FP64, -1, 0, 0};
    if (opt) o = *opt;
    if (o.precision != RKL_FP64 && o.precision != RKL_MIXED) return fail(RKL_EINVAL, "precision must be RKL_FP64 or RKL_MIXED");
    if (o.smax == 0) o.smax = ngrids > 1 ? 64 : 1024;
    if (o.smax < 2 || o.smax > 4096) return fail(RKL_EINVAL, "smax must be in [2, 4096]");
    if (o.variant < -1 || o.variant >= variant_count()) return fail(RKL_EINVAL, "variant out of range");
    if (o.scheme != RKL_RKL2 && o.scheme != RKL_RKL1) return fail(RKL_EINVAL, "scheme must be RKL_RKL2 or RKL_RKL1");

    rkl_plan_s* p = new rkl_plan_s();
    p->ngrids = ngrids;
    p->precision = o.precision;
    p->variant = 0;
    p->smax = o.smax;
    p->scheme = o.scheme;
    p->off.push_back(0);
    for (int g = 0; g < ngrids; ++g) {
        std::string why;
        if (!validate(grids[g], why)) {
            delete p;
            return fail(RKL_EINVAL, "grid " + std::to_string(g) + ": " + why);
        }
        p->desc.push_back(grids[g]);
        p->gc.push_back(make_const(grids[g], o.scheme));
        const int64_t n = (int64_t)grids[g].n[0] * grids[g].n[1] * grids[g].n[2];
        p->off.push_back(p->off.back() + n);
    }
    p->total = p->off.back();
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { free_plan(p); return hipfail(e, "hipGetDevice"); }

    const size_t rs = o.precision == RKL_MIXED ? sizeof(float) : sizeof(double);
    const std::vector<double> tab = coefficient_table(o.smax, o.scheme);
    int64_t ext_blocks = 1;
    for (int32_t g = 0; g < ngrids; ++g)
        for (int v = 0; v < variant_count(); ++v)
            if (variant_get(v).fuse == 1) ext_blocks = std::max(ext_blocks, stage_blocks(variant_get(v), p->gc[g]));
    bool ok = hipMalloc(&p->Ya, sizeof(double) * p->total) == hipSuccess &&
              hipMalloc(&p->Yb, sizeof(double) * p->total) == hipSuccess &&
              hipMalloc(&p->MY0, rs * p->total) == hipSuccess &&
              hipMalloc(&p->coef, sizeof(double) * tab.size()) == hipSuccess &&
              hipMalloc(&p->state, sizeof(GridState) * ngrids) == hipSuccess &&
              hipMalloc(&p->partials, sizeof(double) * 3 * 1024) == hipSuccess &&
              hipMalloc(&p->ext_part, sizeof(double) * 3 * ext_blocks) == hipSuccess &&
              hipMalloc(&p->ext_ok, sizeof(int32_t) * ngrids) == hipSuccess &&
              hipMalloc(&p->s_dev, sizeof(int32_t)) == hipSuccess &&
              hipHostMalloc((void**)&p->s_host, sizeof(int32_t), hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_plan(p);
        return fail(RKL_ENOMEM, "device allocation failed");
    }
    e = hipMemcpy(p->coef, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(p->state, 0, sizeof(GridState) * ngrids);
    if (e == hipSuccess) e = hipMemset(p->ext_ok, 0, sizeof(int32_t) * ngrids);
    // the set-up above is ordered on the legacy stream; finish it so that the
    // caller's first launch on any stream sees it
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) { free_plan(p); return hipfail(e, "plan upload"); }
    if (ngrids > 1 && o.scheme == RKL_RKL2) {
        std::string why;
        rkl_status st = batch_create(p->desc, p->gc, p->off, p->precision, p->smax, 0, &p->batch, why);
        if (st != RKL_OK) { free_plan(p); return fail(st, why); }
    }
    if (o.variant > 0) {
        rkl_status st = select_variant(p, o.variant);
        if (st != RKL_OK) {
            const std::string why = g_err;
            free_plan(p);
            return fail(st, why);
        }
    }
    *out = p;
    return RKL_OK;
}

rkl_status rkl_destroy(rkl_plan_t p) {
    if (!p) return RKL_OK;
    // free on the plan's device, then restore the caller's
    int cur = -1;
    const bool other = hipGetDevice(&cur) == hipSuccess && cur != p->device && hipSetDevice(p->device) == hipSuccess;
    (void)hipDeviceSynchronize();
    free_plan(p);
    if (other) (void)hipSetDevice(cur);
    return RKL_OK;
}

int64_t rkl_grid_offset(rkl_plan_t p, int32_t g) {
    if (!p || g < 0 || g > p->ngrids) return -1;
    return p->off[g];
}

rkl_status rkl_set_ghosts(rkl_plan_t p, int32_t g, int32_t axis, const double* lo, const double* hi) {
    if (rkl_status st = check_plan(p)) return st;
    if (g < 0 || g >= p->ngrids) return fail(RKL_EINVAL, "grid index out of range");
    if (axis < 0 || axis > 2) return fail(RKL_EINVAL, "axis must be 0, 1 or 2");
    if (!(p->gc[g].fixed & (1 << axis))) return fail(RKL_EINVAL, "axis is not RKL_BC_FIXED");
    if (!lo || !hi) return fail(RKL_EINVAL, "NULL ghost layer");
    p->gc[g].gh[2 * axis] = lo;
    p->gc[g].gh[2 * axis + 1] = hi;
    return RKL_OK;
}

rkl_status rkl_set_variant(rkl_plan_t p, int32_t v) {
    if (rkl_status st = check_plan(p)) return st;
    if (v < 0 || v >= variant_count()) return fail(RKL_EINVAL, "variant out of range");
    return select_variant(p, v);
}

static rkl_status check_grid(rkl_plan_t p, int32_t g) {
    if (rkl_status st = check_plan(p)) return st;
    if (g < 0 || g >= p->ngrids) return fail(RKL_EINVAL, "grid index out of range");
    return RKL_OK;
}

// min/max reduction of T and the finalize step for grid g
static rkl_status reduce_and_finalize(rkl_plan_t p, int32_t g, const double* T, double dt_hyp, int mode,
                                      int32_t* s_dev, hipStream_t st, int smax = 0) {
    const int64_t N = p->off[g + 1] - p->off[g];
    const int nb = reduce_blocks(N);
    HIPCHECK(launch_reduce(T, N, p->partials, nb, st), "reduce launch");
    HIPCHECK(launch_finalize(p->partials, nb, p->gc[g], dt_hyp, mode, p->state + g, s_dev, smax ? smax : p->smax, st),
             "finalize launch");
    return RKL_OK;
}

rkl_status rkl_flux_div(rkl_plan_t p, int32_t g, const double* T, const void* b, double* out, void* stream) {
    rkl_status st = check_grid(p, g);
    if (st != RKL_OK) return st;
    if ((st = check_ghosts(p, g)) != RKL_OK) return st;
    if (!T || !b || !out) return fail(RKL_EINVAL, "NULL field pointer");
    if (out == T || (const void*)out == b) return fail(RKL_EINVAL, "out must not alias T or b");
    hipStream_t s = (hipStream_t)stream;
    st = reduce_and_finalize(p, g, T, 0.0, 1, nullptr, s);
    if (st != RKL_OK) return st;
    HIPCHECK(launch_stage(p->precision, variant_get(p->variant), p->gc[g], 0, 0, T, nullptr, nullptr, nullptr, nullptr,
                          out, b, p->state + g, p->coef, s),
             "flux_div launch");
    return RKL_OK;
}

rkl_status rkl_dt_par(rkl_plan_t p, int32_t g, const double* T, double* dt_par_out, void* stream) {
    rkl_status st = check_grid(p, g);
    if (st != RKL_OK) return st;
    if (!T || !dt_par_out) return fail(RKL_EINVAL, "NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    st = reduce_and_finalize(p, g, T, 0.0, 1, nullptr, s);
    if (st != RKL_OK) return st;
    double v = 0.0;
    HIPCHECK(hipMemcpyAsync(&v, &p->state[g].dt_par, sizeof(double), hipMemcpyDeviceToHost, s), "dt_par copy");
    HIPCHECK(hipStreamSynchronize(s), "dt_par sync");
    *dt_par_out = v;
    return RKL_OK;
}

rkl_status rkl_superstep(rkl_plan_t p, int32_t g, double* T, const void* b, double dt_hyp, int32_t* s_out,
                         void* stream) {
    rkl_status st = check_grid(p, g);
    if (st != RKL_OK) return st;
    if ((st = check_ghosts(p, g)) != RKL_OK) return st;
    if (!T || !b) return fail(RKL_EINVAL, "NULL field pointer");
    if ((const void*)T == b) return fail(RKL_EINVAL, "b must not alias T");
    if (!(dt_hyp >= 0.0) || !std::isfinite(dt_hyp)) return fail(RKL_EINVAL, "dt_hyp must be finite and >= 0");
    hipStream_t s = (hipStream_t)stream;
    st = reduce_and_finalize(p, g, T, dt_hyp, 0, p->s_dev, s);
    if (st != RKL_OK) return st;
    HIPCHECK(hipMemcpyAsync(p->s_host, p->s_dev, sizeof(int32_t), hipMemcpyDeviceToHost, s), "s copy");
    HIPCHECK(hipStreamSynchronize(s), "s sync");
    const int S = *p->s_host;
    if (s_out) *s_out = S;
    const int smin = p->scheme == RKL_RKL1 ? 1 : 2;
    if (S < smin || S > p->smax)
        return fail(RKL_ESTAGES, "stage count " + std::to_string(S) + " outside [" + std::to_string(smin) +
                                     ", smax=" + std::to_string(p->smax) + "]");

    const GridConst& gc = p->gc[g];
    const Variant v = variant_get(p->variant);
    const int64_t n = p->off[g + 1] - p->off[g];
    double* bufs[4] = {p->Ya + p->off[g], p->Yb + p->off[g], p->Yc ? p->Yc + p->off[g] : nullptr,
                       p->Yd ? p->Yd + p->off[g] : nullptr};
    const size_t rs = p->precision == RKL_MIXED ? sizeof(float) : sizeof(double);
    void* M = (char*)p->MY0 + rs * p->off[g];
    const GridState* gs = p->state + g;
    // stage 1: Y1 = Y0 + mut_1 tau M(Y0), tau M(Y0) kept for the later stages
    HIPCHECK(launch_stage(p->precision, v, gc, 1, 1, T, nullptr, nullptr, nullptr, M, bufs[0], b, gs, p->coef, s),
             "stage 1 launch");
    // a stage buffer holding neither Y_{j-1} nor Y_{j-2}
    auto pick = [&](const double* u, const double* w, const double* x) -> double* {
        for (double* c : bufs)
            if (c && c != u && c != w && c != x) return c;
        return nullptr;
    };
    const double* ym1 = bufs[0];
    const double* ym2 = T;
    int j = 2;
    while (j <= S) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        size_t rec = 0;
        if (p->prof) {
            // owned by the plan from here on (prof_clear destroys them)
            HIPCHECK(hipEventCreate(&e0), "event create");
            if (hipEventCreate(&e1) != hipSuccess) {
                (void)hipEventDestroy(e0);
                return fail(RKL_EDEVICE, "event create");
            }
            rec = p->prof_recs.size();
            p->prof_recs.push_back({e0, e1, 0, 0});
            HIPCHECK(hipEventRecord(e0, s), "event record");
        }
        int done;
        if (v.fuse >= 2 && j + v.fuse - 1 < S) {
            // stages j..j+F-1 in one launch, writing Y_{j+F-2} and Y_{j+F-1};
            // the final stage always runs alone (it writes T, which the fused
            // kernel reads around its tiles), and so does a shorter remainder
            double* o1 = pick(ym1, ym2, nullptr);
            double* o2 = pick(ym1, ym2, o1);
            HIPCHECK(launch_fused(v, gc, j, ym1, ym2, T, M, o1, o2, b, gs, p->coef, s), "fused stage launch");
            ym2 = o1;
            ym1 = o2;
            done = v.fuse;
        } else {
            // Y_j overwrites Y_{j-2} cell by cell (never Y0 = T before the last stage)
            double* out = j == S ? T : (ym2 == T ? pick(ym1, T, nullptr) : const_cast<double*>(ym2));
            HIPCHECK(launch_stage(p->precision, v, gc, 2, j, ym1, ym2, T, M, nullptr, out, b, gs, p->coef, s),
                     "stage launch");
            ym2 = ym1;
            ym1 = out;
            done = 1;
        }
        if (p->prof) {
            HIPCHECK(hipEventRecord(e1, s), "event record");
            p->prof_recs[rec].fuse = done;
            p->prof_recs[rec].cells = done * n;
        }
        j += done;
    }
    if (S == 1)   // RKL1 with one stage: Y1 was written next to T (stage 1 reads T around each cell)
        HIPCHECK(hipMemcpyAsync(T, bufs[0], sizeof(double) * n, hipMemcpyDeviceToDevice, s), "result copy");
    return RKL_OK;
}

rkl_status rkl_superstep_async(rkl_plan_t p, int32_t g, double* T, const void* b, double dt_hyp,
                               int32_t s_cap, int32_t* s_out, void* stream) {
    rkl_status st = check_grid(p, g);
    if (st != RKL_OK) return st;
    if ((st = check_ghosts(p, g)) != RKL_OK) return st;
    if (!T || !b) return fail(RKL_EINVAL, "NULL field pointer");
    if ((const void*)T == b) return fail(RKL_EINVAL, "b must not alias T");
    if (!(dt_hyp >= 0.0) || !std::isfinite(dt_hyp)) return fail(RKL_EINVAL, "dt_hyp must be finite and >= 0");
    if (p->scheme != RKL_RKL2) return fail(RKL_EINVAL, "rkl_superstep_async implements RKL2 only");
    if (s_cap < 2 || s_cap > p->smax)
        return fail(RKL_EINVAL, "s_cap must be in [2, smax=" + std::to_string(p->smax) + "]");
    hipStream_t s = (hipStream_t)stream;
    // s on the device; stages beyond it (and every stage, if s > s_cap) return at once
    st = reduce_and_finalize(p, g, T, dt_hyp, 0, s_out, s, s_cap);
    if (st != RKL_OK) return st;
    const GridConst& gc = p->gc[g];
    Variant v = variant_get(p->variant);
    if (v.fuse != 1) v = variant_get(0);   // routed launches are one stage each
    const size_t rs = p->precision == RKL_MIXED ? sizeof(float) : sizeof(double);
    void* M = (char*)p->MY0 + rs * p->off[g];
    const Route r{p->Ya + p->off[g], p->Yb + p->off[g], s_cap, 0};
    for (int j = 1; j <= s_cap; ++j)
        HIPCHECK(launch_stage(p->precision, v, gc, j == 1 ? 1 : 2, j, nullptr, nullptr, nullptr, M, M, T, b,
                              p->state + g, p->coef, s, 0.0, &r),
                 "routed stage launch");
    return RKL_OK;
}

rkl_status rkl_supersteps_async(rkl_plan_t p, int32_t g, double* T, const void* b, double dt_hyp,
                                int32_t nsteps, int32_t s_cap, int32_t* s_out, void* stream) {
    rkl_status st = check_grid(p, g);
    if (st != RKL_OK) return st;
    if ((st = check_ghosts(p, g)) != RKL_OK) return st;
    if (!T || !b) return fail(RKL_EINVAL, "NULL field pointer");
    if ((const void*)T == b) return fail(RKL_EINVAL, "b must not alias T");
    if (!(dt_hyp >= 0.0) || !std::isfinite(dt_hyp)) return fail(RKL_EINVAL, "dt_hyp must be finite and >= 0");
    if (p->scheme != RKL_RKL2) return fail(RKL_EINVAL, "rkl_supersteps_async implements RKL2 only");
    if (s_cap < 2 || s_cap > p->smax)
        return fail(RKL_EINVAL, "s_cap must be in [2, smax=" + std::to_string(p->smax) + "]");
    if (nsteps < 1) return fail(RKL_EINVAL, "nsteps must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    const GridConst& gc = p->gc[g];
    Variant v = variant_get(p->variant);
    if (v.fuse != 1) v = variant_get(0);   // routed launches are one stage each
    // the compile-time-shaped stage kernels keep the last stage's extrema;
    // other grids take the reduction pass before every super-step
    const bool keep = gc.ndim == 3 && !gc.fixed;
    const int64_t N = p->off[g + 1] - p->off[g];
    const int nb = reduce_blocks(N);
    const int64_t nbx = stage_blocks(v, gc);
    const size_t rs = p->precision == RKL_MIXED ? sizeof(float) : sizeof(double);
    void* M = (char*)p->MY0 + rs * p->off[g];
    const Route r{p->Ya + p->off[g], p->Yb + p->off[g], s_cap, 0};
    const ExtOut ext{p->ext_part, p->ext_ok + g};
    for (int32_t i = 0; i < nsteps; ++i) {
        // super-step 0 always reduces (and clears the flag); later ones skip the
        // pass when the previous super-step's last stage left the extrema
        const bool chain = keep && i > 0;
        HIPCHECK(launch_reduce(T, N, p->partials, nb, s, chain ? p->ext_ok + g : nullptr), "reduce launch");
        HIPCHECK(launch_finalize(p->partials, nb, gc, dt_hyp, 0, p->state + g, s_out ? s_out + i : nullptr, s_cap,
                                 s, nullptr, chain ? p->ext_part : nullptr, chain ? (int)nbx : 0,
                                 keep ? p->ext_ok + g : nullptr),
                 "finalize launch");
        for (int j = 1; j <= s_cap; ++j)
            HIPCHECK(launch_stage(p->precision, v, gc, j == 1 ? 1 : 2, j, nullptr, nullptr, nullptr, M, M, T, b,
                                  p->state + g, p->coef, s, 0.0, &r, keep && j >= 2 ? &ext : nullptr),
                     "routed stage launch");
    }
    return RKL_OK;
}

// Forward-Euler sub-steps T <- T + tau_k (gamma-1)/rho (-div F_c(T)), one
// launch each (stage kernel kind 3), ping-ponging between T and the plan's
// first stage buffer; an odd count ends with one copy into T.
static rkl_status euler_substeps(rkl_plan_t p, int32_t g, double* T, const void* b, int64_t count,
                                 const std::function<double(int64_t)>& tau, hipStream_t s) {
    const GridConst& gc = p->gc[g];
    const Variant v = variant_get(p->variant);
    const int64_t n = p->off[g + 1] - p->off[g];
    double* A = p->Ya + p->off[g];
    for (int64_t k = 0; k < count; ++k) {
        const double* in = (k % 2 == 0) ? T : A;
        double* out = (k % 2 == 0) ? A : T;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        size_t rec = 0;
        if (p->prof) {
            HIPCHECK(hipEventCreate(&e0), "event create");
            if (hipEventCreate(&e1) != hipSuccess) {
                (void)hipEventDestroy(e0);
                return fail(RKL_EDEVICE, "event create");
            }
            rec = p->prof_recs.size();
            p->prof_recs.push_back({e0, e1, 0, 0});
            HIPCHECK(hipEventRecord(e0, s), "event record");
        }
        HIPCHECK(launch_stage(p->precision, v, gc, 3, 0, in, nullptr, nullptr, nullptr, nullptr, out, b,
                              p->state + g, p->coef, s, -tau(k) * gc.fac),
                 "sub-step launch");
        if (p->prof) {
            HIPCHECK(hipEventRecord(e1, s), "event record");
            p->prof_recs[rec].fuse = 5;
            p->prof_recs[rec].cells = n;
        }
    }
    if (count % 2 == 1)
        HIPCHECK(hipMemcpyAsync(T, A, sizeof(double) * n, hipMemcpyDeviceToDevice, s), "result copy");
    return RKL_OK;
}

// dt_par of grid g from T (reduction + one read-back)
static rkl_status read_dt_par(rkl_plan_t p, int32_t g, const double* T, double* dtp, hipStream_t s) {
    rkl_status st = reduce_and_finalize(p, g, T, 0.0, 1, nullptr, s);
    if (st != RKL_OK) return st;
    HIPCHECK(hipMemcpyAsync(dtp, &p->state[g].dt_par, sizeof(double), hipMemcpyDeviceToHost, s), "dt_par copy");
    HIPCHECK(hipStreamSynchronize(s), "dt_par sync");
    return RKL_OK;
}

rkl_status rkl_subcycle(rkl_plan_t p, int32_t g, double* T, const void* b, double dt_hyp, int64_t max_sub,
                        int64_t* nsub_out, void* stream) {
    rkl_status st = check_grid(p, g);
    if (st != RKL_OK) return st;
    if ((st = check_ghosts(p, g)) != RKL_OK) return st;
    if (nsub_out) *nsub_out = 0;
    if (!T || !b) return fail(RKL_EINVAL, "NULL field pointer");
    if ((const void*)T == b) return fail(RKL_EINVAL, "b must not alias T");
    if (!(dt_hyp >= 0.0) || !std::isfinite(dt_hyp)) return fail(RKL_EINVAL, "dt_hyp must be finite and >= 0");
    if (max_sub < 1) return fail(RKL_EINVAL, "max_sub must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    double dtp = 0.0;
    st = read_dt_par(p, g, T, &dtp, s);
    if (st != RKL_OK) return st;
    if (dt_hyp == 0.0 || std::isinf(dtp)) return RKL_OK;   // nothing to do
    // N_sub = ceil(dt_hyp / dt_par) forward-Euler sub-steps of dt_hyp / N_sub
    const double q = std::ceil(dt_hyp / dtp);
    if (!(q <= (double)max_sub))
        return fail(RKL_ESTAGES, "sub-step count above max_sub (T unchanged)");
    const int64_t nsub = (int64_t)q;
    const double tau = dt_hyp / (double)nsub;
    st = euler_substeps(p, g, T, b, nsub, [tau](int64_t) { return tau; }, s);
    if (st != RKL_OK) return st;
    if (nsub_out) *nsub_out = nsub;
    return RKL_OK;
}

// AAG gain (the sum of the sub-steps over dt_par) of s stages, Eq. AAG-STS.
// Where (1+sqrt(nu))^{2s} is beyond the double range, the bracket
// (a-c)/(a+c) is 1 to double precision (c <= 1).
static double aag_gain(int s, double nu) {
    const double q = std::sqrt(nu);
    const double a = std::pow(1.0 + q, 2.0 * s), c = std::pow(1.0 - q, 2.0 * s);
    if (std::isinf(a)) return s / (2.0 * q);
    return s / (2.0 * q) * ((a - c) / (a + c));
}

rkl_status rkl_aag(rkl_plan_t p, int32_t g, double* T, const void* b, double dt_hyp, double nu, int32_t max_s,
                   int32_t* s_out, void* stream) {
    rkl_status st = check_grid(p, g);
    if (st != RKL_OK) return st;
    if ((st = check_ghosts(p, g)) != RKL_OK) return st;
    if (s_out) *s_out = 0;
    if (!T || !b) return fail(RKL_EINVAL, "NULL field pointer");
    if ((const void*)T == b) return fail(RKL_EINVAL, "b must not alias T");
    if (!(dt_hyp >= 0.0) || !std::isfinite(dt_hyp)) return fail(RKL_EINVAL, "dt_hyp must be finite and >= 0");
    if (!(nu > 0.0 && nu < 1.0)) return fail(RKL_EINVAL, "nu must be in (0, 1)");
    if (max_s < 1) return fail(RKL_EINVAL, "max_s must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    double dtp = 0.0;
    st = read_dt_par(p, g, T, &dtp, s);
    if (st != RKL_OK) return st;
    if (dt_hyp == 0.0 || std::isinf(dtp)) return RKL_OK;
    const double r = dt_hyp / dtp;
    int S = -1;
    for (int k = 1; k <= max_s; ++k)
        if (aag_gain(k, nu) >= r) { S = k; break; }
    if (S < 0) return fail(RKL_ESTAGES, "AAG stage count above max_s (T unchanged)");
    // tau_j = dt_p / ((nu-1) cos(pi (2j-1)/(2S)) + 1 + nu), scaled to sum to dt_hyp
    std::vector<double> taus(S);
    double sum = 0.0;
    for (int j = 1; j <= S; ++j) {
        taus[j - 1] = 1.0 / ((nu - 1.0) * std::cos(M_PI * (2.0 * j - 1.0) / (2.0 * S)) + 1.0 + nu);
        sum += taus[j - 1];
    }
    for (double& t : taus) t *= dt_hyp / sum;
    st = euler_substeps(p, g, T, b, S, [&taus](int64_t k) { return taus[k]; }, s);
    if (st != RKL_OK) return st;
    if (s_out) *s_out = S;
    return RKL_OK;
}

rkl_status rkl_autotune(rkl_plan_t p, int32_t g, const double* T, const void* b, double dt_hyp, int32_t reps,
                        int32_t* best_variant, double* best_ms, void* stream) {
    rkl_status st = check_grid(p, g);
    if (st != RKL_OK) return st;
    if ((st = check_ghosts(p, g)) != RKL_OK) return st;
    if (!T || !b) return fail(RKL_EINVAL, "NULL field pointer");
    if ((const void*)T == b) return fail(RKL_EINVAL, "b must not alias T");
    if (reps < 1 || reps > 1000) return fail(RKL_EINVAL, "reps must be in [1, 1000]");
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = sizeof(double) * (size_t)(p->off[g + 1] - p->off[g]);
    double* W = nullptr;
    HIPCHECK(hipMalloc(&W, bytes), "autotune scratch");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int best = -1;
    float best_t = 0.f;
    const int saved = p->variant;
    const bool saved_prof = p->prof;
    p->prof = false;
    rkl_status res = RKL_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        res = fail(RKL_EDEVICE, "autotune events");
    }
    for (int v = 0; res == RKL_OK && v < variant_count(); ++v) {
        if (!variant_ok(p, variant_get(v))) continue;
        res = select_variant(p, v);
        if (res != RKL_OK) break;
        // one untimed super-step from the caller's T, then reps timed ones
        if (hipMemcpyAsync(W, T, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) { res = fail(RKL_EDEVICE, "autotune copy"); break; }
        res = rkl_superstep(p, g, W, b, dt_hyp, nullptr, stream);
        if (res != RKL_OK) break;
        if (hipMemcpyAsync(W, T, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipEventRecord(e0, s) != hipSuccess) { res = fail(RKL_EDEVICE, "autotune copy"); break; }
        for (int r = 0; r < reps && res == RKL_OK; ++r) res = rkl_superstep(p, g, W, b, dt_hyp, nullptr, stream);
        if (res != RKL_OK) break;
        float t = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess) { res = fail(RKL_EDEVICE, "autotune timing"); break; }
        if (best < 0 || t < best_t) { best = v; best_t = t; }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(W);
    p->prof = saved_prof;
    if (res != RKL_OK) {
        p->variant = saved;
        return res;
    }
    p->variant = best;
    if (best_variant) *best_variant = best;
    if (best_ms) *best_ms = best_t / reps;
    return RKL_OK;
}

rkl_status rkl_profile(rkl_plan_t p, int32_t enable) {
    if (rkl_status st = check_plan(p)) return st;
    HIPCHECK(hipDeviceSynchronize(), "profile sync");
    prof_clear(p);
    p->prof = enable != 0;
    return RKL_OK;
}

rkl_status rkl_profile_read(rkl_plan_t p, int32_t fuse, double* ms, int64_t* launches, int64_t* cells) {
    if (rkl_status st = check_plan(p)) return st;
    if (fuse < 1 || fuse > 6) return fail(RKL_EINVAL, "kind must be 1 to 6");
    double tot = 0.0;
    int64_t nl = 0, nc = 0;
    for (const auto& r : p->prof_recs) {
        if (r.fuse != fuse) continue;
        HIPCHECK(hipEventSynchronize(r.b), "event sync");
        float t = 0.f;
        HIPCHECK(hipEventElapsedTime(&t, r.a, r.b), "event elapsed");
        tot += t;
        nl += 1;
        nc += r.cells;
    }
    if (ms) *ms = tot;
    if (launches) *launches = nl;
    if (cells) *cells = nc;
    return RKL_OK;
}

rkl_status rkl_query(rkl_plan_t p, int32_t g, int32_t* last_s, double* last_dt_par, uint32_t* flags) {
    rkl_status st = check_grid(p, g);
    if (st != RKL_OK) return st;
    GridState h;
    HIPCHECK(hipDeviceSynchronize(), "query sync");
    HIPCHECK(hipMemcpy(&h, p->state + g, sizeof h, hipMemcpyDeviceToHost), "query copy");
    bool aborted = false;
    if (p->batch_mode == 1) HIPCHECK(batch_aborted(p->batch, &aborted), "abort word");
    if (last_s) *last_s = h.s;
    if (last_dt_par) *last_dt_par = h.dt_par;
    if (flags) *flags = h.flags | (aborted ? (uint32_t)RKL_FLAG_ABORTED : 0u);
    return RKL_OK;
}

rkl_status rkl_superstep_batched(rkl_plan_t p, double* T, const void* b, const double* dt_hyp, int32_t* s_out,
                                 void* stream) {
    if (rkl_status st = check_plan(p)) return st;
    if (rkl_status st = check_no_fixed(p, "the batched path")) return st;
    if (!T || !b || !dt_hyp) return fail(RKL_EINVAL, "NULL pointer");
    if ((const void*)T == b) return fail(RKL_EINVAL, "b must not alias T");
    rkl_status st = ensure_batch(p);
    if (st != RKL_OK) return st;
    BatchBuffers bb{T, b, dt_hyp, s_out, p->Ya, p->Yb, p->MY0, p->coef, p->state};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    hipError_t e = batch_launch(p->batch, bb, (hipStream_t)stream, p->prof ? &ev : nullptr, p->batch_mode);
    // cell-stages of a batched launch depend on the device-side stage counts:
    // recorded as 0 (the caller knows them from s_out); the persistent launch
    // is recorded as kind 6
    for (auto& x : ev) p->prof_recs.push_back({x.first, x.second, p->batch_mode == 1 ? 6 : 1, 0});
    if (e != hipSuccess) return hipfail(e, "batched launch");
    return RKL_OK;
}

rkl_status rkl_graph_capture(rkl_plan_t p, double* T, const void* b, const double* dt_hyp, int32_t* s_out,
                             void* stream) {
    if (rkl_status st = check_plan(p)) return st;
    if (rkl_status st = check_no_fixed(p, "the batched path")) return st;
    if (!T || !b || !dt_hyp) return fail(RKL_EINVAL, "NULL pointer");
    if ((const void*)T == b) return fail(RKL_EINVAL, "b must not alias T");
    rkl_status st = ensure_batch(p);
    if (st != RKL_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipStream_t cap;
    HIPCHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "capture stream");
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { (void)hipStreamDestroy(cap); return hipfail(e, "begin capture"); }
    BatchBuffers bb{T, b, dt_hyp, s_out, p->Ya, p->Yb, p->MY0, p->coef, p->state};
    hipError_t le = batch_launch(p->batch, bb, cap, nullptr, p->batch_mode);
    hipGraph_t gr = nullptr;
    e = hipStreamEndCapture(cap, &gr);
    (void)hipStreamDestroy(cap);
    if (le != hipSuccess) { if (gr) (void)hipGraphDestroy(gr); return hipfail(le, "batched launch under capture"); }
    if (e != hipSuccess) return hipfail(e, "end capture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(gr); return hipfail(e, "graph instantiate"); }
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph = gr;
    p->graph_exec = ex;
    (void)s;
    return RKL_OK;
}

rkl_status rkl_graph_launch(rkl_plan_t p, void* stream) {
    if (rkl_status st = check_plan(p)) return st;
    if (!p->graph_exec) return fail(RKL_ESTATE, "no graph captured");
    HIPCHECK(hipGraphLaunch(p->graph_exec, (hipStream_t)stream), "graph launch");
    return RKL_OK;
}

}  // extern "C"
