// k_assign.hip -- nearest-mode labelling ("cluster x by the distance to
// modes", Algorithm 2, final loop) and the input finiteness scan, for gfx950.
//
// One lane per point: the point row stays in registers, the modes stream
// through LDS tiles shared by the workgroup, and the lane keeps the two
// smallest squared distances.  Distances are FP32 direct differences (the
// expanded |x|^2 + |m|^2 - 2 x.m form cancels badly at large coordinates).
// Modes are scanned in increasing index with a strict '<', so ties go to
// the lowest index, as the oracle's argmin does.

#include "fms_internal.h"

namespace fms {

namespace {

constexpr int kT = 256;

template <int D>
__global__ __launch_bounds__(kT) void assign_kernel(const float* __restrict__ X, int n, int d,
                                                    const float* __restrict__ modes, int k,
                                                    int32_t* __restrict__ labels,
                                                    float* __restrict__ margin) {
    constexpr int TM = (D <= 4) ? 1024 : (4096 / D);   // modes per LDS tile (16 KB)
    __shared__ float tile[TM * D];
    const int i = blockIdx.x * kT + threadIdx.x;
    float x[D];
    const bool live = i < n;
#pragma unroll
    for (int q = 0; q < D; ++q) x[q] = (live && q < d) ? X[(long long)i * d + q] : 0.0f;
    float best = __builtin_inff(), second = __builtin_inff();
    int arg = 0;
    for (int base = 0; base < k; base += TM) {
        const int cnt = min(TM, k - base);
        __syncthreads();
        for (int e = threadIdx.x; e < cnt * D; e += kT) {
            const int j = e / D, q = e % D;
            tile[e] = (q < d) ? modes[(long long)(base + j) * d + q] : 0.0f;
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            float dd = 0.0f;
#pragma unroll
            for (int q = 0; q < D; ++q) {
                const float t = x[q] - tile[j * D + q];
                dd = fmaf(t, t, dd);
            }
            if (dd < best) {
                second = best;
                best = dd;
                arg = base + j;
            } else if (dd < second) {
                second = dd;
            }
        }
    }
    if (live) {
        labels[i] = arg;
        if (margin) margin[i] = (k > 1) ? sqrtf(second) - sqrtf(best) : __builtin_inff();
    }
}

__global__ void check_finite_kernel(const float* __restrict__ X, long long count,
                                    int32_t* flag) {
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    bool bad = false;
    for (; e < count; e += stride) bad = bad || !isfinite(X[e]);
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

}  // namespace

hipError_t launch_assign(const float* X, int n, int d, const float* modes, int k,
                         int32_t* labels, float* margin, hipStream_t s) {
    const int blocks = (n + kT - 1) / kT;
    switch (step_shape(d).D) {
#define FMS_CASE(DD)                                                                       \
    case DD:                                                                               \
        hipLaunchKernelGGL(assign_kernel<DD>, dim3(blocks), dim3(kT), 0, s, X, n, d, modes, \
                           k, labels, margin);                                             \
        break;
        FMS_CASE(1)
        FMS_CASE(2)
        FMS_CASE(3)
        FMS_CASE(4)
        FMS_CASE(8)
        FMS_CASE(16)
        FMS_CASE(32)
        FMS_CASE(64)
        FMS_CASE(128)
        FMS_CASE(256)
#undef FMS_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_check_finite(const float* X, long long count, int32_t* flag, hipStream_t s) {
    long long blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, count,
                       flag);
    return hipGetLastError();
}

}  // namespace fms
