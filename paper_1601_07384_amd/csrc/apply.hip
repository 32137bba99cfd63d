// Matrix-free pressure Schur operator y = S x (eq. CS_19, negated; Sec. 2.4).
//
// S = dt^2 S^sp (x) C: for element i with neighbours k_f across its local
// faces f,
//   Y_i = sum_{k in {i, k_0..k_3}} B_{c(i),k} X_k C^T
// where X_k is the N x G coefficient matrix of element k ([G][N] in memory),
// B_{c,0..4} the class-deduplicated dt^2-scaled spatial blocks and C the G x G
// time factor.  One thread produces one spatial row n of one element for all
// G time nodes; neighbour coefficients are gathered through the neighbour
// table (elements are numbered along a Hilbert curve, so the four neighbours
// of a tile are mostly inside or next to it).
#include "internal.hpp"
#include "kernels.hpp"

namespace stdg {

template <int G, typename T>
__global__ void __launch_bounds__(256) schur_apply_rows(
    const T* __restrict__ B, const int32_t* __restrict__ cls, const int32_t* __restrict__ nbr,
    const T* __restrict__ C, const T* __restrict__ x, T* __restrict__ y, int64_t E, int N) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = gid / N;
    const int n = (int)(gid - i * N);
    if (i >= E) return;
    const T* Bc = B + (int64_t)cls[i] * 5 * N * N;
    T acc[G];
#pragma unroll
    for (int b = 0; b < G; ++b) acc[b] = T(0);
    for (int k = 0; k < 5; ++k) {
        const int64_t t = (k == 0) ? i : (int64_t)nbr[4 * i + (k - 1)];
        if (t < 0) continue;
        const T* Br = Bc + ((int64_t)k * N + n) * N;
        const T* xt = x + t * G * N;
        for (int m = 0; m < N; ++m) {
            const T bv = Br[m];
#pragma unroll
            for (int b = 0; b < G; ++b) acc[b] += bv * xt[b * N + m];
        }
    }
    T* yi = y + i * G * N;
#pragma unroll
    for (int a = 0; a < G; ++a) {
        T s = T(0);
#pragma unroll
        for (int b = 0; b < G; ++b) s += C[a * G + b] * acc[b];
        yi[a * N + n] = s;
    }
}

template <typename T>
static hipError_t launch_rows(const stdg_mesh* m, const T* B, const T* C, const T* x, T* y,
                              hipStream_t s) {
    const int64_t work = m->E * m->N;
    const int threads = 256;
    const int64_t blocks = (work + threads - 1) / threads;
    switch (m->G) {
#define STDG_G(g)                                                                              \
    case g:                                                                                    \
        hipLaunchKernelGGL((schur_apply_rows<g, T>), dim3(blocks), dim3(threads), 0, s, B,    \
                           m->d.cls, m->d.nbr, C, x, y, m->E, m->N);                          \
        break;
        STDG_G(1) STDG_G(2) STDG_G(3) STDG_G(4) STDG_G(5) STDG_G(6) STDG_G(7)
#undef STDG_G
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_apply_f64(const stdg_mesh* m, const double* x, double* y, hipStream_t s) {
    return launch_rows<double>(m, m->d.blocks, m->d.C, x, y, s);
}

hipError_t launch_apply_f32(const stdg_mesh* m, const float* x, float* y, hipStream_t s) {
    return launch_rows<float>(m, m->d.blocks32, m->d.C32, x, y, s);
}

// FP32 blocks with FP64 input/output: convert through a scratch vector.
__global__ void cvt_d2f(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}
__global__ void cvt_f2d(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}

hipError_t convert_d2f(const double* a, float* b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(cvt_d2f, dim3((n + 255) / 256), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}
hipError_t convert_f2d(const float* a, double* b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(cvt_f2d, dim3((n + 255) / 256), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}

}  // namespace stdg
