// rkl_noalloc.hip -- the RKL2 super-step for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc): no plan, no allocation, no host synchronisation.
//
// Its scratch (two FP64 stage buffers, the tau M(Y0) buffer, the coefficient
// rows of the current stage count, the grid state and the reduction
// partials) is one file-scope device array, `scratch`.  Each GPU the library
// runs on holds its own copy of the array until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in symbol): the array's device address is looked up once per device
// with hipGetSymbolAddress, with that device current, and only that address
// is used.  Every call on one GPU shares that GPU's array; calls that
// overlap on one GPU race.  Nothing in the array needs to start at zero:
// each call writes every part before it reads it.
#include <cmath>
#include <mutex>
#include <string>

#include "../../include/rkl.h"
#include "rkl_host.h"
#include "rkl_internal.h"

namespace rkl {
namespace {

constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }

constexpr int64_t kCells = RKL_NOALLOC_MAX_CELLS;
constexpr int kSmax = RKL_NOALLOC_MAX_STAGES;
constexpr int kPartials = 1024;    // reduce_blocks() never uses more
constexpr size_t kOffA = 0;
constexpr size_t kOffB = kOffA + align256(sizeof(double) * kCells);
constexpr size_t kOffM = kOffB + align256(sizeof(double) * kCells);
constexpr size_t kOffCoef = kOffM + align256(sizeof(double) * kCells);
constexpr size_t kOffState = kOffCoef + align256(sizeof(double) * 5 * (kSmax + 1));
constexpr size_t kOffPart = kOffState + align256(sizeof(GridState));
constexpr size_t kBytes = kOffPart + align256(sizeof(double) * 3 * kPartials);

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_base[kMaxDevices] = {};   // device address of `scratch`, per device

}  // namespace
}  // namespace rkl

static __device__ __align__(256) unsigned char scratch[rkl::kBytes];

using namespace rkl;

// the device address of `scratch` on the current device (looked up once)
static rkl_status scratch_base(unsigned char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hipfail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(RKL_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_base[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hipfail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(RKL_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_base[dev] = (unsigned char*)p;
    }
    *out = g_base[dev];
    return RKL_OK;
}

extern "C" rkl_status rkl_superstep_noalloc(const rkl_grid_desc* grid, int32_t precision, double* T,
                                            const void* b, double dt_hyp, int32_t s_cap, int32_t* s_out,
                                            void* stream) {
    if (!grid) return fail(RKL_EINVAL, "grid descriptor is NULL");
    std::string why;
    if (!validate(*grid, why)) return fail(RKL_EINVAL, why);
    for (int d = 0; d < 3; ++d)
        if (grid->boundary[d] == RKL_BC_FIXED) return fail(RKL_EINVAL, "rkl_superstep_noalloc does not take RKL_BC_FIXED axes");
    if (precision != RKL_FP64 && precision != RKL_MIXED) return fail(RKL_EINVAL, "precision must be RKL_FP64 or RKL_MIXED");
    const int64_t N = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
    if (N > kCells)
        return fail(RKL_EINVAL, "rkl_superstep_noalloc: the grid has " + std::to_string(N) +
                                    " cells, above the static scratch limit RKL_NOALLOC_MAX_CELLS = " +
                                    std::to_string(kCells));
    if (s_cap < 2 || s_cap > kSmax)
        return fail(RKL_EINVAL, "s_cap must be in [2, RKL_NOALLOC_MAX_STAGES = " + std::to_string(kSmax) + "]");
    if (!T || !b) return fail(RKL_EINVAL, "NULL field pointer");
    if ((const void*)T == b) return fail(RKL_EINVAL, "b must not alias T");
    if (!(dt_hyp >= 0.0) || !std::isfinite(dt_hyp)) return fail(RKL_EINVAL, "dt_hyp must be finite and >= 0");

    unsigned char* base = nullptr;
    if (rkl_status st = scratch_base(&base)) return st;
    double* A = (double*)(base + kOffA);
    double* B = (double*)(base + kOffB);
    void* M = base + kOffM;
    double* coef = (double*)(base + kOffCoef);
    GridState* state = (GridState*)(base + kOffState);
    double* part = (double*)(base + kOffPart);

    hipStream_t s = (hipStream_t)stream;
    const GridConst gc = make_const(*grid, RKL_RKL2);
    const int nb = reduce_blocks(N);
    hipError_t e = launch_reduce(T, N, part, nb, s);
    if (e != hipSuccess) return hipfail(e, "reduce launch");
    // dt_par, s and the coefficient rows of s on the device; s > s_cap flags
    // the grid and every stage below returns at once
    e = launch_finalize(part, nb, gc, dt_hyp, 0, state, s_out, s_cap, s, coef);
    if (e != hipSuccess) return hipfail(e, "finalize launch");
    const Route r{A, B, s_cap, 1};
    for (int j = 1; j <= s_cap; ++j) {
        e = launch_stage(precision, variant_get(0), gc, j == 1 ? 1 : 2, j, nullptr, nullptr, nullptr, M, M, T, b,
                         state, coef, s, 0.0, &r);
        if (e != hipSuccess) return hipfail(e, "routed stage launch");
    }
    return RKL_OK;
}
