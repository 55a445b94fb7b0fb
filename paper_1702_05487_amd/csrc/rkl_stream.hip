// rkl_stream.hip -- a streaming probe of the HBM path for the measurements
// that put the stencil against its memory roofline: a coalesced copy (or a
// read-only sweep) with the stencil's own per-lane access widths, so that
// its bandwidth is what such loads can reach on this device, and its HBM
// counters calibrate the counters read on the stencil kernels.
#include "../../include/rkl.h"
#include "rkl_host.h"

namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 4;   // elements per thread, kThreads apart (each wave reads whole lines)

template <typename V>
__global__ __launch_bounds__(kThreads) void copy_kernel(const V* __restrict__ src, V* __restrict__ dst,
                                                         int64_t n) {
    const int64_t base = (int64_t)blockIdx.x * kThreads * kUnroll + threadIdx.x;
    V v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const int64_t i = base + (int64_t)u * kThreads;
        if (i < n) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const int64_t i = base + (int64_t)u * kThreads;
        if (i < n) dst[i] = v[u];
    }
}

// read-only sweep: each block stores one sum (so the loads cannot be dropped)
__global__ __launch_bounds__(kThreads) void read_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                         int64_t n) {
    const int64_t base = (int64_t)blockIdx.x * kThreads * kUnroll + threadIdx.x;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const int64_t i = base + (int64_t)u * kThreads;
        if (i < n) acc += src[i];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    __shared__ double sm[kThreads / 64];
    if (threadIdx.x % 64 == 0) sm[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0) dst[blockIdx.x] = sm[0] + sm[1] + sm[2] + sm[3];
}

}  // namespace

using namespace rkl;

extern "C" rkl_status rkl_stream(const void* src, void* dst, int64_t bytes, int32_t mode, void* stream) {
    if (!src || !dst) return fail(RKL_EINVAL, "NULL pointer");
    if (mode < 0 || mode > 3) return fail(RKL_EINVAL, "mode must be 0, 1, 2 or 3");
    const int64_t width = mode == 1 ? 16 : (mode == 3 ? 4 : 8);
    if (bytes <= 0 || bytes % 16 != 0) return fail(RKL_EINVAL, "bytes must be a positive multiple of 16");
    if ((uintptr_t)src % 16 || (uintptr_t)dst % 16) return fail(RKL_EINVAL, "pointers must be 16-byte aligned");
    const int64_t n = bytes / width;
    const int64_t blocks = (n + kThreads * kUnroll - 1) / (kThreads * kUnroll);
    if (blocks > 0x7fffffff) return fail(RKL_EINVAL, "too large");
    hipStream_t s = (hipStream_t)stream;
    if (mode == 0) copy_kernel<double><<<(int)blocks, kThreads, 0, s>>>((const double*)src, (double*)dst, n);
    else if (mode == 1) copy_kernel<double2><<<(int)blocks, kThreads, 0, s>>>((const double2*)src, (double2*)dst, n);
    else if (mode == 3) copy_kernel<float><<<(int)blocks, kThreads, 0, s>>>((const float*)src, (float*)dst, n);
    else read_kernel<<<(int)blocks, kThreads, 0, s>>>((const double*)src, (double*)dst, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipfail(e, "stream launch");
    return RKL_OK;
}
