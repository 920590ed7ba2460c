// k_adjoint.hip -- the differentiable Gaussian update and its hand-written
// adjoint, for gfx950, in FP32 or FP64.
//
// Forward (the batched update of Section II-B for every seed, no stopping):
//     w_ij = exp(-|s_j - x_i|^2 / (2 h^2)),  W_j = sum_i w_ij,
//     s'_j = s_j + delta_j,  delta_j = sum_i w_ij (x_i - s_j) / W_j .
// Reverse, for an upstream gradient g_j = dL/ds'_j (derived from the
// forward: ds'_j/dw_ij = (x_i - s'_j)/W_j, dw_ij/ds_j = w_ij (x_i - s_j)/h^2,
// and the direct path ds'_j/dx_i = (w_ij/W_j) I):
//     beta_ij = w_ij * g_j.(x_i - s'_j) / (h^2 W_j)
//     dL/ds_j += sum_i beta_ij (x_i - s_j)
//     dL/dx_i += sum_j (w_ij / W_j) g_j + beta_ij (s_j - x_i)
// Three passes over the pairs recompute the weights each time; no m x n
// weight matrix is ever stored.  Each pass splits its inner sum into kP
// chunks (one partial per chunk) that a reduction kernel adds in chunk
// order, so results are bitwise reproducible.  The inner loop of every pass
// streams the other set's rows through wave-uniform (scalar) loads.

#include "fms_internal.h"

namespace fms {

namespace {

constexpr int kT = 256;
constexpr int kP = 8;   // inner-sum chunks per pass

template <typename T>
__device__ __forceinline__ T expw(T q, T c);   // exp(c q), c = -1/(2h^2)
template <>
__device__ __forceinline__ float expw<float>(float q, float c) {
    return __builtin_amdgcn_exp2f(q * c);       // c pre-multiplied by log2(e)
}
template <>
__device__ __forceinline__ double expw<double>(double q, double c) {
    return exp(q * c);
}

// Per-pass per-row state loaded once per lane.
template <typename T, int D>
struct Row {
    T v[D];
};

// Row `row` of a d-column array, zero-padded to D.  EXACT (d == D) loads
// with compile-time offsets, which lets wave-uniform rows become wide scalar
// loads; otherwise each column is guarded.
template <typename T, int D, bool EXACT>
__device__ __forceinline__ void load_row(const T* __restrict__ A, long long row, int d, T* out) {
    if constexpr (EXACT) {
#pragma unroll
        for (int k = 0; k < D; ++k) out[k] = A[row * D + k];
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) out[k] = (k < d) ? A[row * d + k] : T(0);
    }
}

// Forward partials: lane = seed j, chunk of points.  part[(b*kP + c)*(D+1) + k][m]
template <typename T, int D, bool EXACT>
__global__ __launch_bounds__(kT) void fwd_partial_kernel(const T* __restrict__ X, int n,
                                                         const T* __restrict__ S, int m, int d,
                                                         T c, T* __restrict__ part) {
    const int b = blockIdx.z, chunk = blockIdx.y;
    const int j = blockIdx.x * kT + threadIdx.x;
    const T* Xb = X + (long long)b * n * d;
    T s[D], acc[D + 1];
    load_row<T, D, EXACT>(S + (long long)b * m * d, j < m ? j : 0, d, s);
#pragma unroll
    for (int k = 0; k <= D; ++k) acc[k] = T(0);
    const int p0 = (int)((long long)n * chunk / kP), p1 = (int)((long long)n * (chunk + 1) / kP);
    for (int i = p0; i < p1; ++i) {
        T x[D];
        load_row<T, D, EXACT>(Xb, i, d, x);
        T dx[D], q = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            dx[k] = x[k] - s[k];
            q = fma(dx[k], dx[k], q);
        }
        const T w = expw<T>(q, c);
        acc[D] += w;
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = fma(w, dx[k], acc[k]);
    }
    if (j < m) {
        T* out = part + (long long)(b * kP + chunk) * (D + 1) * m + j;
#pragma unroll
        for (int k = 0; k <= D; ++k) out[(long long)k * m] = acc[k];
    }
}

// Reduce forward partials: S_out = s + delta; keeps delta and 1/W per seed.
template <typename T, int D>
__global__ void fwd_reduce_kernel(const T* __restrict__ part, const T* __restrict__ S, int m,
                                  int d, T* S_out, T* delta, T* invW) {
    const int b = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    T a[D + 1];
#pragma unroll
    for (int k = 0; k <= D; ++k) a[k] = T(0);
    for (int c = 0; c < kP; ++c) {
        const T* p = part + (long long)(b * kP + c) * (D + 1) * m + j;
#pragma unroll
        for (int k = 0; k <= D; ++k) a[k] += p[(long long)k * m];
    }
    const T iw = T(1) / a[D];
    const long long row = (long long)b * m + j;
    if (invW) invW[row] = iw;
#pragma unroll
    for (int k = 0; k < D; ++k) {   // constant indices keep a[] in registers
        if (k < d) {
            const T dk = a[k] * iw;
            if (delta) delta[row * d + k] = dk;
            if (S_out) S_out[row * d + k] = S[row * d + k] + dk;
        }
    }
}

// dS partials: lane = seed j, chunk of points.
template <typename T, int D, bool EXACT>
__global__ __launch_bounds__(kT) void ds_partial_kernel(const T* __restrict__ X, int n,
                                                        const T* __restrict__ S, int m, int d,
                                                        T c, T inv_h2, const T* __restrict__ G,
                                                        const T* __restrict__ delta,
                                                        const T* __restrict__ invW,
                                                        T* __restrict__ gdel_out,
                                                        T* __restrict__ part) {
    const int b = blockIdx.z, chunk = blockIdx.y;
    const int j = blockIdx.x * kT + threadIdx.x;
    const int jj = j < m ? j : 0;
    const long long row = (long long)b * m + jj;
    const T* Xb = X + (long long)b * n * d;
    T s[D], g[D], acc[D];
    load_row<T, D, EXACT>(S + (long long)b * m * d, jj, d, s);
    load_row<T, D, EXACT>(G + (long long)b * m * d, jj, d, g);
    T gdel = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k)
        if (k < d) gdel = fma(g[k], delta[row * d + k], gdel);
    if (chunk == 0 && j < m) gdel_out[row] = gdel;   // g_j . delta_j, read by the dX pass
    const T coef = inv_h2 * invW[row];
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] = T(0);
    const int p0 = (int)((long long)n * chunk / kP), p1 = (int)((long long)n * (chunk + 1) / kP);
    for (int i = p0; i < p1; ++i) {
        T x[D];
        load_row<T, D, EXACT>(Xb, i, d, x);
        T dx[D], q = T(0), gdx = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            dx[k] = x[k] - s[k];
            q = fma(dx[k], dx[k], q);
            gdx = fma(g[k], dx[k], gdx);
        }
        // g.(x - s') = g.(x - s) - g.delta
        const T beta = expw<T>(q, c) * (gdx - gdel) * coef;
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = fma(beta, dx[k], acc[k]);
    }
    if (j < m) {
        T* out = part + (long long)(b * kP + chunk) * D * m + j;
#pragma unroll
        for (int k = 0; k < D; ++k) out[(long long)k * m] = acc[k];
    }
}

// dX partials: lane = point i, chunk of seeds.
template <typename T, int D, bool EXACT>
__global__ __launch_bounds__(kT) void dx_partial_kernel(const T* __restrict__ X, int n,
                                                        const T* __restrict__ S, int m, int d,
                                                        T c, T inv_h2, const T* __restrict__ G,
                                                        const T* __restrict__ gdel,
                                                        const T* __restrict__ invW,
                                                        T* __restrict__ part) {
    const int b = blockIdx.z, chunk = blockIdx.y;
    const int i = blockIdx.x * kT + threadIdx.x;
    const T* Sb = S + (long long)b * m * d;
    const T* Gb = G + (long long)b * m * d;
    const T* Eb = gdel + (long long)b * m;
    const T* Wb = invW + (long long)b * m;
    T x[D], acc[D];
    load_row<T, D, EXACT>(X + (long long)b * n * d, i < n ? i : 0, d, x);
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] = T(0);
    const int j0 = (int)((long long)m * chunk / kP), j1 = (int)((long long)m * (chunk + 1) / kP);
    for (int j = j0; j < j1; ++j) {
        T s[D], g[D];
        load_row<T, D, EXACT>(Sb, j, d, s);
        load_row<T, D, EXACT>(Gb, j, d, g);
        const T iw = Wb[j];
        const T gd = Eb[j];
        T dx[D], q = T(0), gdx = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            dx[k] = x[k] - s[k];
            q = fma(dx[k], dx[k], q);
            gdx = fma(g[k], dx[k], gdx);
        }
        const T w = expw<T>(q, c);
        const T a = w * iw;                              // w_ij / W_j
        const T beta = a * (gdx - gd) * inv_h2;          // beta_ij
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = fma(a, g[k], fma(-beta, dx[k], acc[k]));
    }
    if (i < n) {
        T* out = part + (long long)(b * kP + chunk) * D * n + i;
#pragma unroll
        for (int k = 0; k < D; ++k) out[(long long)k * n] = acc[k];
    }
}

// out[row, k] += sum over chunks of part (chunk order).
template <typename T, int D>
__global__ void add_reduce_kernel(const T* __restrict__ part, int rows, int d, T* out) {
    const int b = blockIdx.y;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    for (int k = 0; k < d; ++k) {
        T a = T(0);
        for (int c = 0; c < kP; ++c) a += part[((long long)(b * kP + c) * D + k) * rows + r];
        out[((long long)b * rows + r) * d + k] += a;
    }
}

template <typename T>
T weight_coef(double h) {
    return sizeof(T) == 4 ? T(-1.4426950408889634 / (2.0 * h * h)) : T(-1.0 / (2.0 * h * h));
}

template <typename T, int D>
hipError_t fwd_t(const T* X, int nb, int n, const T* S, int m, int d, double h, T* S_out,
                 T* delta, T* invW, T* part, hipStream_t s) {
    dim3 g1((m + kT - 1) / kT, kP, nb);
    if (d == D)
        hipLaunchKernelGGL((fwd_partial_kernel<T, D, true>), g1, dim3(kT), 0, s, X, n, S, m, d,
                           weight_coef<T>(h), part);
    else
        hipLaunchKernelGGL((fwd_partial_kernel<T, D, false>), g1, dim3(kT), 0, s, X, n, S, m, d,
                           weight_coef<T>(h), part);
    dim3 g2((m + 255) / 256, nb);
    hipLaunchKernelGGL((fwd_reduce_kernel<T, D>), g2, dim3(256), 0, s, part, S, m, d, S_out,
                       delta, invW);
    return hipGetLastError();
}

template <typename T, int D, bool EXACT>
void adj_passes(const T* X, int nb, int n, const T* S, int m, int d, T c, T ih2, const T* G,
                const T* delta, const T* invW, T* gdel, T* part, T* dS, T* dX, hipStream_t s) {
    hipLaunchKernelGGL((ds_partial_kernel<T, D, EXACT>), dim3((m + kT - 1) / kT, kP, nb), dim3(kT), 0,
                       s, X, n, S, m, d, c, ih2, G, delta, invW, gdel, part);
    hipLaunchKernelGGL((add_reduce_kernel<T, D>), dim3((m + 255) / 256, nb), dim3(256), 0, s,
                       part, m, d, dS);
    hipLaunchKernelGGL((dx_partial_kernel<T, D, EXACT>), dim3((n + kT - 1) / kT, kP, nb), dim3(kT), 0,
                       s, X, n, S, m, d, c, ih2, G, gdel, invW, part);
    hipLaunchKernelGGL((add_reduce_kernel<T, D>), dim3((n + 255) / 256, nb), dim3(256), 0, s,
                       part, n, d, dX);
}

template <typename T, int D>
hipError_t adj_t(const T* X, int nb, int n, const T* S, int m, int d, double h, const T* G,
                 T* dS, T* dX, T* delta, T* invW, T* gdel, T* part, hipStream_t s) {
    hipError_t e = fwd_t<T, D>(X, nb, n, S, m, d, h, nullptr, delta, invW, part, s);
    if (e != hipSuccess) return e;
    const T c = weight_coef<T>(h);
    const T ih2 = T(1.0 / (h * h));
    if (d == D) adj_passes<T, D, true>(X, nb, n, S, m, d, c, ih2, G, delta, invW, gdel, part, dS, dX, s);
    else adj_passes<T, D, false>(X, nb, n, S, m, d, c, ih2, G, delta, invW, gdel, part, dS, dX, s);
    return hipGetLastError();
}

struct Ws {
    char* base;
    size_t part, delta, invw, gdel;
};

Ws carve(void* ws, int nb, int n, int m, int d, int bytes) {
    const int D = step_shape(d).D;
    const long long rows = n > m ? n : m;
    Ws w;
    w.base = (char*)ws;
    w.part = 0;
    size_t off = (size_t)nb * kP * (D + 1) * rows * bytes;
    off = (off + 255) & ~(size_t)255;
    w.delta = off;
    off += (size_t)nb * m * d * bytes;
    off = (off + 255) & ~(size_t)255;
    w.invw = off;
    off += (size_t)nb * m * bytes;
    off = (off + 255) & ~(size_t)255;
    w.gdel = off;
    return w;
}

#define FMS_ADJ_DSWITCH(D_, CALL)                           \
    switch (D_) {                                           \
        case 1: { constexpr int DD = 1; return CALL; }      \
        case 2: { constexpr int DD = 2; return CALL; }      \
        case 3: { constexpr int DD = 3; return CALL; }      \
        case 4: { constexpr int DD = 4; return CALL; }      \
        case 8: { constexpr int DD = 8; return CALL; }      \
        case 16: { constexpr int DD = 16; return CALL; }    \
        case 32: { constexpr int DD = 32; return CALL; }    \
        case 64: { constexpr int DD = 64; return CALL; }    \
        default: return hipErrorInvalidValue;               \
    }

}  // namespace

size_t adjoint_workspace_bytes(int nb, int n, int m, int d, int bytes) {
    Ws w = carve(nullptr, nb, n, m, d, bytes);
    return w.gdel + (size_t)nb * m * bytes + 256;
}

hipError_t launch_forward_update(const void* X, int nb, int n, const void* S, int m, int d,
                                 double h, void* S_out, int bytes, void* ws, hipStream_t s) {
    Ws w = carve(ws, nb, n, m, d, bytes);
    const int D = step_shape(d).D;
    if (bytes == 4) {
        FMS_ADJ_DSWITCH(D, (fwd_t<float, DD>((const float*)X, nb, n, (const float*)S, m, d, h,
                                             (float*)S_out, nullptr, nullptr,
                                             (float*)(w.base + w.part), s)));
    }
    FMS_ADJ_DSWITCH(D, (fwd_t<double, DD>((const double*)X, nb, n, (const double*)S, m, d, h,
                                          (double*)S_out, nullptr, nullptr,
                                          (double*)(w.base + w.part), s)));
}

hipError_t launch_step_adjoint(const void* X, int nb, int n, const void* S, int m, int d,
                               double h, const void* G, void* dS, void* dX, int bytes, void* ws,
                               hipStream_t s) {
    Ws w = carve(ws, nb, n, m, d, bytes);
    const int D = step_shape(d).D;
    if (bytes == 4) {
        FMS_ADJ_DSWITCH(D, (adj_t<float, DD>((const float*)X, nb, n, (const float*)S, m, d, h,
                                             (const float*)G, (float*)dS, (float*)dX,
                                             (float*)(w.base + w.delta),
                                             (float*)(w.base + w.invw),
                                             (float*)(w.base + w.gdel),
                                             (float*)(w.base + w.part), s)));
    }
    FMS_ADJ_DSWITCH(D, (adj_t<double, DD>((const double*)X, nb, n, (const double*)S, m, d, h,
                                          (const double*)G, (double*)dS, (double*)dX,
                                          (double*)(w.base + w.delta),
                                          (double*)(w.base + w.invw),
                                          (double*)(w.base + w.gdel),
                                          (double*)(w.base + w.part), s)));
}

}  // namespace fms
