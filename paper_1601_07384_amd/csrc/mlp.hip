// Learned Krylov initial guess: a three-layer perceptron acting element by
// element on the history of the first Picard pressure p^{n+1,1} and on the
// right-hand side of the first pressure-correction solve of a time step
// (Sec. 2.6, step 5 with the zero pressure guess of step 0), which yields
// that pressure.  Training and inference run entirely in the
// kernels of this file: a feature gather, one MFMA-tiled GEMM with fused
// bias/activation epilogues (FP64 v_mfma_f64_16x16x4 or FP32
// v_mfma_f32_16x16x4), deterministic split-K reductions for the weight
// gradients, the mean-squared loss and Adam.
//
// With P = p^{n,1} and Pm = p^{n-1,1}, the features of element i
// (11 N_st + 4 values) are: P of i and of its neighbours across local faces
// 0..3 divided by the RMS of P; P - Pm of the same five elements divided by
// its RMS s_D; b_i divided by the RMS of b; four neighbour-present flags.
// The network corrects the linear extrapolation 2P - Pm: its target is
// (x* - 2P + Pm) / s_D with x* = p^{n+1,1}, and the guess is
// x0 = 2P - Pm + s_D * output.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

struct stdg_model {
    int nin = 0, hid = 0, nout = 0, nst = 0;
    int64_t E = 0;
    stdg_model_config cfg{};
    int64_t np = 0;             // parameter count
    int64_t oW1, ob1, oW2, ob2, oW3, ob3;
    int64_t t_adam = 0;
    void* theta = nullptr;      // parameters, gradient, Adam moments (model precision)
    void* grad = nullptr;
    void* mom1 = nullptr;
    void* mom2 = nullptr;
    void* one = nullptr;        // a single 1 (ones row for bias gradients)
    void* F = nullptr;          // [batch][nin]
    void* Z1 = nullptr;         // [batch][hid]
    void* H1 = nullptr;
    void* Z2 = nullptr;
    void* H2 = nullptr;
    void* Y = nullptr;          // [batch][nout]
    void* dY = nullptr;
    void* dZ2 = nullptr;        // [batch][hid]
    void* dZ1 = nullptr;
    void* part = nullptr;       // split-K partials [KSPLIT][max block]
    double* lpart = nullptr;    // loss partials
    double* lbatch = nullptr;   // per-batch loss
    int64_t lbatch_n = 0;
    double* scales = nullptr;   // per step: s_P, s_D, s_B
    int64_t scales_n = 0;
    double* spart = nullptr;
    int64_t* idx = nullptr;
    int64_t idx_n = 0;
    double* hbuf = nullptr;     // pinned host scratch
    double* ve = nullptr;       // residual objective: guess error, S e, S^T S e  [E][G][N]
    double* vR = nullptr;
    double* vG = nullptr;
    double* CT = nullptr;       // transposed time factor (S^T = B (x) C^T)
};

namespace stdg {
namespace {

constexpr int KSPLIT = 64;      // split-K slices for the weight gradients
constexpr int RB = 256;         // reduction block
constexpr int NRB = 512;        // reduction blocks

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct MF;
// row of result register r in lane l (the column is l % 16)
template <> struct MF<double> {
    using V = d4;
    __device__ static V op(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct MF<float> {
    using V = f4;
    __device__ static V op(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

__device__ inline double sig(double z) { return 1.0 / (1.0 + exp(-z)); }
__device__ inline float sig(float z) { return 1.0f / (1.0f + expf(-z)); }

enum { EPI_STORE = 0, EPI_BIAS_ACT = 1, EPI_BIAS = 2, EPI_DACT = 3 };

// C = op(A) op(B) over the k-slice blockIdx.z, A(m,k) = A[m*sam + k*sak],
// B(k,n) = B[k*sbk + n*sbn].  64x64 tile per 256-thread block, each wave a
// 32x32 quarter as 2x2 MFMA 16x16x4 tiles; k staged 16 at a time in LDS.
// MFMA 16x16x4 operand layout: lane l holds A[l%16][l/16] and B[l/16][l%16];
// result register r of lane l is D[MF<T>::row(l, r)][l%16] (the FP64 and
// FP32 instructions interleave the rows differently).
// Epilogues: STORE (slice z written at C + z*M*ldc), BIAS_ACT (Zout = acc +
// bias, C = silu), BIAS (C = acc + bias), DACT (C = acc * silu'(Zin)).
template <typename T, int EPI>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, int kchunk, const T* __restrict__ A, int64_t sam,
                                              int64_t sak, const T* __restrict__ B, int64_t sbk, int64_t sbn,
                                              T* __restrict__ C, int64_t ldc, const T* __restrict__ bias,
                                              T* __restrict__ Zout, const T* __restrict__ Zin) {
    __shared__ T As[16][65];
    __shared__ T Bs[16][65];
    using V = typename MF<T>::V;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
    const int kb = blockIdx.z * kchunk;
    const int ke = min(K, kb + kchunk);
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    V acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = V{0, 0, 0, 0};
    for (int k0 = kb; k0 < ke; k0 += 16) {
        for (int e = tid; e < 1024; e += 256) {
            int mm, kk;
            if (sak == 1) { kk = e & 15; mm = e >> 4; } else { mm = e & 63; kk = e >> 6; }
            const int gm = m0 + mm, gk = k0 + kk;
            As[kk][mm] = (gm < M && gk < ke) ? A[(int64_t)gm * sam + (int64_t)gk * sak] : T(0);
        }
        for (int e = tid; e < 1024; e += 256) {
            int nn, kk;
            if (sbn == 1) { nn = e & 63; kk = e >> 6; } else { kk = e & 15; nn = e >> 4; }
            const int gn = n0 + nn, gk = k0 + kk;
            Bs[kk][nn] = (gn < N && gk < ke) ? B[(int64_t)gk * sbk + (int64_t)gn * sbn] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            T a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[kk + (lane >> 4)][wm + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[kk + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = MF<T>::op(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
    T* Cz = C + (int64_t)blockIdx.z * M * ldc;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + i * 16 + MF<T>::row(lane, r);
                const int gn = n0 + wn + j * 16 + (lane & 15);
                if (gm < M && gn < N) {
                    T v = acc[i][j][r];
                    const int64_t o = (int64_t)gm * ldc + gn;
                    if (EPI == EPI_BIAS_ACT) {
                        const T z = v + bias[gn];
                        Zout[o] = z;
                        v = z * sig(z);
                    } else if (EPI == EPI_BIAS) {
                        v += bias[gn];
                    } else if (EPI == EPI_DACT) {
                        const T z = Zin[o];
                        const T s = sig(z);
                        v *= s * (T(1) + z * (T(1) - s));
                    }
                    Cz[o] = v;
                }
            }
}

// out[t] = sum_z part[z * count + t], z in order (deterministic).
template <typename T>
__global__ void k_sum_slices(const T* __restrict__ part, int nz, int64_t count, T* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    T s = 0;
    for (int z = 0; z < nz; ++z) s += part[(int64_t)z * count + t];
    out[t] = s;
}

// Feature rows.  Row r is sample q = idx[r] (or r + row0 without idx): step
// s = q / E, element i = q % E.  scales[3 s + {0,1,2}] = s_P, s_D, s_B.
template <typename T>
__global__ void k_features(const double* __restrict__ P, const double* __restrict__ Pm,
                           const double* __restrict__ Bv, const int32_t* __restrict__ nbr,
                           const int64_t* __restrict__ idx, int64_t row0, int64_t n, int64_t E, int nst,
                           const double* __restrict__ scales, T* __restrict__ F) {
    const int nin = 11 * nst + 4;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nin) return;
    const int64_t row = t / nin;
    const int f = (int)(t % nin);
    const int64_t q = idx ? idx[row] : row + row0;
    const int64_t s = q / E, i = q % E;
    const int64_t base = s * E * nst;
    double v;
    if (f < 10 * nst) {
        const int slot = (f / nst) % 5, c = f % nst;
        const int64_t k = slot == 0 ? i : (int64_t)nbr[4 * i + slot - 1];
        if (k < 0) {
            v = 0.0;
        } else if (f < 5 * nst) {
            v = P[base + k * nst + c] / scales[3 * s];
        } else {
            v = (P[base + k * nst + c] - Pm[base + k * nst + c]) / scales[3 * s + 1];
        }
    } else if (f < 11 * nst) {
        v = Bv[base + i * nst + (f - 10 * nst)] / scales[3 * s + 2];
    } else {
        v = nbr[4 * i + (f - 11 * nst)] >= 0 ? 1.0 : 0.0;
    }
    F[t] = (T)v;
}

// Block partial sums of squares of P, P - Pm and B over one step's vector.
__global__ void k_sumsq3(const double* __restrict__ P, const double* __restrict__ Pm, const double* __restrict__ B,
                         int64_t n, double* __restrict__ part) {
    __shared__ double sh[3][RB];
    double a = 0, b = 0, c = 0;
    for (int64_t t = (int64_t)blockIdx.x * RB + threadIdx.x; t < n; t += (int64_t)gridDim.x * RB) {
        const double p = P[t], d = p - Pm[t], r = B[t];
        a += p * p; b += d * d; c += r * r;
    }
    sh[0][threadIdx.x] = a; sh[1][threadIdx.x] = b; sh[2][threadIdx.x] = c;
    __syncthreads();
    for (int w = RB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) part[3 * blockIdx.x + k] = sh[k][0];
}

// scales[0..2] = RMS values (1 when zero) from the block partials.
__global__ void k_scales(const double* __restrict__ part, int nb, int64_t n, double* __restrict__ scales) {
    __shared__ double sh[3][RB];
    double a = 0, b = 0, c = 0;
    for (int k = threadIdx.x; k < nb; k += RB) { a += part[3 * k]; b += part[3 * k + 1]; c += part[3 * k + 2]; }
    sh[0][threadIdx.x] = a; sh[1][threadIdx.x] = b; sh[2][threadIdx.x] = c;
    __syncthreads();
    for (int w = RB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        const double r = sqrt(sh[threadIdx.x][0] / (double)n);
        scales[threadIdx.x] = r > 0.0 ? r : 1.0;
    }
}

// dY = 2 (Y - target) / (n nout) and block partials of the squared error.
// target = tgt[row][c] if given, else (X - 2P + Pm)/s_D of the row's sample.
template <typename T>
__global__ void k_mse(const T* __restrict__ Y, const double* __restrict__ tgt, const double* __restrict__ X,
                      const double* __restrict__ P, const double* __restrict__ Pm, const double* __restrict__ scales,
                      const int64_t* __restrict__ idx, int64_t row0, int64_t E, int64_t n, int nout,
                      T* __restrict__ dY, double* __restrict__ part) {
    __shared__ double sh[RB];
    const int64_t total = n * nout;
    const double inv = 2.0 / (double)total;
    double acc = 0;
    for (int64_t t = (int64_t)blockIdx.x * RB + threadIdx.x; t < total; t += (int64_t)gridDim.x * RB) {
        const int64_t row = t / nout;
        const int c = (int)(t % nout);
        double target;
        if (tgt) {
            target = tgt[t];
        } else {
            const int64_t q = idx ? idx[row] : row + row0;
            const int64_t s = q / E, i = q % E;
            const int64_t o = s * E * nout + i * nout + c;
            target = (X[o] - 2.0 * P[o] + Pm[o]) / scales[3 * s + 1];
        }
        const double r = (double)Y[t] - target;
        acc += r * r;
        dY[t] = (T)(inv * r);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = RB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// out[slot] = sum(part[0..nb)) * scale
__global__ void k_sum_scalar(const double* __restrict__ part, int nb, double scale, double* __restrict__ out) {
    __shared__ double sh[RB];
    double a = 0;
    for (int k = threadIdx.x; k < nb; k += RB) a += part[k];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = RB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0] * scale;
}

template <typename T>
__global__ void k_adam(T* __restrict__ th, const T* __restrict__ g, T* __restrict__ m, T* __restrict__ v, int64_t n,
                       double lr, double b1, double b2, double eps, double c1, double c2) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double gg = (double)g[t];
    const double mm = b1 * (double)m[t] + (1.0 - b1) * gg;
    const double vv = b2 * (double)v[t] + (1.0 - b2) * gg * gg;
    m[t] = (T)mm;
    v[t] = (T)vv;
    th[t] = (T)((double)th[t] - lr * (mm / c1) / (sqrt(vv / c2) + eps));
}

// e = 2P - Pm - X (+ s_D Y) over all rows of one step
template <typename T>
__global__ void k_guess_err(const double* __restrict__ P, const double* __restrict__ Pm,
                            const double* __restrict__ X, const T* __restrict__ Y, const double* __restrict__ scales,
                            int64_t n, int with_y, double* __restrict__ e) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double v = (2.0 * P[t] - Pm[t]) - X[t];
    if (with_y) v += scales[1] * (double)Y[t];
    e[t] = v;
}

// dY = 2 s_D (S^T S e) / den
template <typename T>
__global__ void k_resid_dy(const double* __restrict__ g, const double* __restrict__ scales, double inv_den, int64_t n,
                           T* __restrict__ dY) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    dY[t] = (T)(2.0 * scales[1] * inv_den * g[t]);
}

// x0 = 2 P - Pm + s_D * Y (or the correction s_D * Y alone) for rows
// row0 .. row0 + n of one step
template <typename T>
__global__ void k_guess(const double* __restrict__ P, const double* __restrict__ Pm, const T* __restrict__ Y,
                        const double* __restrict__ scales, int64_t off, int64_t count, int correction_only,
                        double* __restrict__ x0) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const double d = scales[1] * (double)Y[t];
    x0[off + t] = correction_only ? d : (2.0 * P[off + t] - Pm[off + t]) + d;
}

template <typename T>
__global__ void k_cvt(const double* __restrict__ a, T* __restrict__ b, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = (T)a[t];
}
template <typename T>
__global__ void k_cvt_back(const T* __restrict__ a, double* __restrict__ b, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = (double)a[t];
}

inline unsigned nb256(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

#define MCK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { set_error(std::string(#x) + ": " + hipGetErrorString(e_)); return STDG_ERR_DEVICE; } } while (0)

template <typename T, int EPI>
hipError_t gemm(hipStream_t s, int M, int N, int K, int nz, const T* A, int64_t sam, int64_t sak, const T* B,
                int64_t sbk, int64_t sbn, T* C, int64_t ldc, const T* bias = nullptr, T* Zout = nullptr,
                const T* Zin = nullptr) {
    int kchunk = (K + nz - 1) / nz;
    kchunk = (kchunk + 15) / 16 * 16;
    nz = (K + kchunk - 1) / kchunk;
    if (nz < 1) nz = 1;
    dim3 grid((M + 63) / 64, (N + 63) / 64, nz);
    hipLaunchKernelGGL((k_gemm<T, EPI>), grid, dim3(256), 0, s, M, N, K, kchunk, A, sam, sak, B, sbk, sbn, C, ldc,
                       bias, Zout, Zin);
    return hipGetLastError();
}

// weight gradient G[M][N] = A^T B over the batch (K rows), split-K + ordered sum
template <typename T>
hipError_t grad_gemm(stdg_model* md, hipStream_t s, int M, int N, int K, const T* A, int64_t sam, int64_t sak,
                     const T* B, int64_t sbk, int64_t sbn, T* G) {
    int nz = std::max(1, std::min(KSPLIT, K / 256));
    int kchunk = ((K + nz - 1) / nz + 15) / 16 * 16;
    nz = std::max(1, (K + kchunk - 1) / kchunk);
    T* part = (T*)md->part;
    dim3 grid((M + 63) / 64, (N + 63) / 64, nz);
    hipLaunchKernelGGL((k_gemm<T, EPI_STORE>), grid, dim3(256), 0, s, M, N, K, kchunk, A, sam, sak, B, sbk, sbn,
                       part, (int64_t)N, (const T*)nullptr, (T*)nullptr, (const T*)nullptr);
    const int64_t count = (int64_t)M * N;
    hipLaunchKernelGGL(k_sum_slices<T>, dim3(nb256(count)), dim3(256), 0, s, part, nz, count, G);
    return hipGetLastError();
}

template <typename T>
int forward_t(stdg_model* md, int64_t n, hipStream_t s) {
    const T* th = (const T*)md->theta;
    const int nin = md->nin, H = md->hid, no = md->nout;
    MCK((gemm<T, EPI_BIAS_ACT>(s, (int)n, H, nin, 1, (const T*)md->F, nin, 1, th + md->oW1, H, 1, (T*)md->H1, H,
                               th + md->ob1, (T*)md->Z1)));
    MCK((gemm<T, EPI_BIAS_ACT>(s, (int)n, H, H, 1, (const T*)md->H1, H, 1, th + md->oW2, H, 1, (T*)md->H2, H,
                               th + md->ob2, (T*)md->Z2)));
    MCK((gemm<T, EPI_BIAS>(s, (int)n, no, H, 1, (const T*)md->H2, H, 1, th + md->oW3, no, 1, (T*)md->Y, no,
                           th + md->ob3)));
    return STDG_OK;
}

// gradient of the loss of the rows in md->F (forward already run, dY set)
template <typename T>
int backward_t(stdg_model* md, int64_t n, hipStream_t s) {
    const T* th = (const T*)md->theta;
    T* g = (T*)md->grad;
    const int nin = md->nin, H = md->hid, no = md->nout;
    const int K = (int)n;
    const T* one = (const T*)md->one;
    // output layer
    MCK(grad_gemm<T>(md, s, H, no, K, (const T*)md->H2, 1, H, (const T*)md->dY, no, 1, g + md->oW3));
    MCK(grad_gemm<T>(md, s, 1, no, K, one, 0, 0, (const T*)md->dY, no, 1, g + md->ob3));
    MCK((gemm<T, EPI_DACT>(s, K, H, no, 1, (const T*)md->dY, no, 1, th + md->oW3, 1, no, (T*)md->dZ2, H, nullptr,
                           nullptr, (const T*)md->Z2)));
    // second layer
    MCK(grad_gemm<T>(md, s, H, H, K, (const T*)md->H1, 1, H, (const T*)md->dZ2, H, 1, g + md->oW2));
    MCK(grad_gemm<T>(md, s, 1, H, K, one, 0, 0, (const T*)md->dZ2, H, 1, g + md->ob2));
    MCK((gemm<T, EPI_DACT>(s, K, H, H, 1, (const T*)md->dZ2, H, 1, th + md->oW2, 1, H, (T*)md->dZ1, H, nullptr,
                           nullptr, (const T*)md->Z1)));
    // first layer
    MCK(grad_gemm<T>(md, s, nin, H, K, (const T*)md->F, 1, nin, (const T*)md->dZ1, H, 1, g + md->oW1));
    MCK(grad_gemm<T>(md, s, 1, H, K, one, 0, 0, (const T*)md->dZ1, H, 1, g + md->ob1));
    return STDG_OK;
}

template <typename T>
int mse_t(stdg_model* md, int64_t n, const double* tgt, const double* X, const double* P, const double* Pm,
          const int64_t* idx, int64_t row0, double* loss_slot, hipStream_t s) {
    const int64_t total = n * md->nout;
    const int nb = (int)std::min<int64_t>(NRB, std::max<int64_t>(1, (total + RB - 1) / RB));
    hipLaunchKernelGGL(k_mse<T>, dim3(nb), dim3(RB), 0, s, (const T*)md->Y, tgt, X, P, Pm, md->scales, idx, row0,
                       md->E, n, md->nout, (T*)md->dY, md->lpart);
    hipLaunchKernelGGL(k_sum_scalar, dim3(1), dim3(RB), 0, s, md->lpart, nb, 1.0 / (double)total, loss_slot);
    MCK(hipGetLastError());
    return STDG_OK;
}

template <typename T>
int adam_t(stdg_model* md, hipStream_t s) {
    md->t_adam++;
    const double c1 = 1.0 - std::pow(md->cfg.beta1, (double)md->t_adam);
    const double c2 = 1.0 - std::pow(md->cfg.beta2, (double)md->t_adam);
    hipLaunchKernelGGL(k_adam<T>, dim3(nb256(md->np)), dim3(256), 0, s, (T*)md->theta, (const T*)md->grad,
                       (T*)md->mom1, (T*)md->mom2, md->np, md->cfg.lr, md->cfg.beta1, md->cfg.beta2, md->cfg.eps, c1,
                       c2);
    MCK(hipGetLastError());
    return STDG_OK;
}

template <typename T>
int features_t(stdg_model* md, const stdg_mesh* m, const double* P, const double* Pm, const double* B,
               const int64_t* idx, int64_t row0, int64_t n, T* F, hipStream_t s) {
    hipLaunchKernelGGL(k_features<T>, dim3(nb256(n * md->nin)), dim3(256), 0, s, P, Pm, B, m->d.nbr, idx, row0, n,
                       md->E, md->nst, md->scales, F);
    MCK(hipGetLastError());
    return STDG_OK;
}

int ensure_scales(stdg_model* md, int64_t steps) {
    if (md->scales_n < steps) {
        if (md->scales) STDG_HIP(hipFree(md->scales));
        md->scales = nullptr;
        STDG_HIP(hipMalloc(&md->scales, sizeof(double) * 3 * steps));
        md->scales_n = steps;
    }
    return STDG_OK;
}

// per-step RMS scales of (P, P - Pm, B), steps of E*nst values each
int compute_scales(stdg_model* md, const double* P, const double* Pm, const double* B, int64_t steps, hipStream_t s) {
    if (int e = ensure_scales(md, steps)) return e;
    const int64_t cnt = md->E * md->nst;
    for (int64_t k = 0; k < steps; ++k) {
        hipLaunchKernelGGL(k_sumsq3, dim3(NRB), dim3(RB), 0, s, P + k * cnt, Pm + k * cnt, B + k * cnt, cnt,
                           md->spart);
        hipLaunchKernelGGL(k_scales, dim3(1), dim3(RB), 0, s, md->spart, NRB, cnt, md->scales + 3 * k);
    }
    MCK(hipGetLastError());
    return STDG_OK;
}

bool is64(const stdg_model* md) { return md->cfg.precision == STDG_FP64; }

int check_model(const stdg_model* md, const stdg_mesh* m) {
    if (!md) { set_error("null model"); return STDG_ERR_ARG; }
    if (m && (m->E != md->E || m->Nst != md->nst)) {
        set_error("model was created for a different mesh shape");
        return STDG_ERR_ARG;
    }
    if (m && !m->d.blocks) { set_error("mesh was built host-only"); return STDG_ERR_ARG; }
    return STDG_OK;
}

int ensure_resid_buffers(stdg_model* md, const stdg_mesh* m) {
    const size_t n = (size_t)md->E * md->nst;
    if (!md->ve) {
        STDG_HIP(hipMalloc(&md->ve, n * sizeof(double)));
        STDG_HIP(hipMalloc(&md->vR, n * sizeof(double)));
        STDG_HIP(hipMalloc(&md->vG, n * sizeof(double)));
        const int G = m->G;
        std::vector<double> ct((size_t)G * G);
        for (int a = 0; a < G; ++a)
            for (int b = 0; b < G; ++b) ct[(size_t)a * G + b] = m->Ctime[(size_t)b * G + a];
        STDG_HIP(hipMalloc(&md->CT, ct.size() * sizeof(double)));
        STDG_HIP(hipMemcpy(md->CT, ct.data(), ct.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    return STDG_OK;
}

// |S (2P - Pm - X)|^2 of step k (scales already computed)
int resid_den(stdg_model* md, stdg_mesh* m, const double* P, const double* Pm, const double* X, int64_t k,
              double& den, hipStream_t s) {
    const int64_t n = md->E * md->nst;
    hipLaunchKernelGGL(k_guess_err<float>, dim3(nb256(n)), dim3(256), 0, s, P + k * n, Pm + k * n, X + k * n,
                       (const float*)nullptr, md->scales + 3 * k, n, 0, md->ve);
    MCK(hipGetLastError());
    MCK(launch_apply_f64(m, md->ve, md->vR, s));
    const double* a[1] = {md->vR};
    return device_dots(m, 1, a, a, n, s, &den);
}

// residual objective of step k and its gradient; scales of step k computed
template <typename T>
int resid_step_t(stdg_model* md, stdg_mesh* m, const double* P, const double* Pm, const double* B, const double* X,
                 int64_t k, double den, double& loss, hipStream_t s) {
    const int64_t E = md->E, n = E * md->nst;
    if (int e = features_t<T>(md, m, P, Pm, B, nullptr, k * E, E, (T*)md->F, s)) return e;
    if (int e = forward_t<T>(md, E, s)) return e;
    hipLaunchKernelGGL(k_guess_err<T>, dim3(nb256(n)), dim3(256), 0, s, P + k * n, Pm + k * n, X + k * n,
                       (const T*)md->Y, md->scales + 3 * k, n, 1, md->ve);
    MCK(hipGetLastError());
    MCK(launch_apply_f64(m, md->ve, md->vR, s));
    double num = 0.0;
    const double* a[1] = {md->vR};
    if (int e = device_dots(m, 1, a, a, n, s, &num)) return e;
    MCK(launch_apply_f64_c(m, md->CT, md->vR, md->vG, s));
    const double inv = den > 0.0 ? 1.0 / den : 0.0;
    hipLaunchKernelGGL(k_resid_dy<T>, dim3(nb256(n)), dim3(256), 0, s, md->vG, md->scales + 3 * k, inv, n,
                       (T*)md->dY);
    MCK(hipGetLastError());
    if (int e = backward_t<T>(md, E, s)) return e;
    loss = num * inv;
    return STDG_OK;
}

}  // namespace

// x0 = 2P - Pm + s_D MLP(features(P, Pm, B)) over all elements (used by the Picard
// step's learned guess).  Asynchronous.
int model_predict(stdg_model* md, const stdg_mesh* m, const double* P, const double* Pm, const double* B,
                  double* x0, hipStream_t s, bool correction_only) {
    if (int e = check_model(md, m)) return e;
    if (int e = compute_scales(md, P, Pm, B, 1, s)) return e;
    const int64_t bs = md->cfg.batch;
    for (int64_t r0 = 0; r0 < md->E; r0 += bs) {
        const int64_t n = std::min(bs, md->E - r0);
        int e;
        if (is64(md)) {
            if ((e = features_t<double>(md, m, P, Pm, B, nullptr, r0, n, (double*)md->F, s))) return e;
            if ((e = forward_t<double>(md, n, s))) return e;
            hipLaunchKernelGGL(k_guess<double>, dim3(nb256(n * md->nst)), dim3(256), 0, s, P, Pm,
                               (const double*)md->Y, md->scales, r0 * md->nst, n * md->nst, (int)correction_only,
                               x0);
        } else {
            if ((e = features_t<float>(md, m, P, Pm, B, nullptr, r0, n, (float*)md->F, s))) return e;
            if ((e = forward_t<float>(md, n, s))) return e;
            hipLaunchKernelGGL(k_guess<float>, dim3(nb256(n * md->nst)), dim3(256), 0, s, P, Pm, (const float*)md->Y,
                               md->scales, r0 * md->nst, n * md->nst, (int)correction_only, x0);
        }
        MCK(hipGetLastError());
    }
    return STDG_OK;
}

}  // namespace stdg

using namespace stdg;

extern "C" void stdg_model_config_default(stdg_model_config* c) {
    if (!c) return;
    c->hidden = 128;
    c->precision = STDG_FP32;
    c->batch = 16384;
    c->seed = 1601;
    c->lr = 1e-3;
    c->beta1 = 0.9;
    c->beta2 = 0.999;
    c->eps = 1e-8;
    c->init_scale_out = 0.0;
    c->loss = STDG_LOSS_RESIDUAL;
}

extern "C" int stdg_model_create(const stdg_mesh* m, const stdg_model_config* cfg, stdg_model** out) {
    if (!m || !cfg || !out) { set_error("null argument"); return STDG_ERR_ARG; }
    *out = nullptr;
    if (!m->d.blocks) { set_error("mesh was built host-only"); return STDG_ERR_ARG; }
    if (cfg->hidden < 1 || cfg->hidden > 1024 || cfg->batch < 1 || cfg->batch > (1 << 22)) {
        set_error("hidden must be in 1..1024 and batch in 1..4194304");
        return STDG_ERR_ARG;
    }
    if (cfg->loss != STDG_LOSS_MSE && cfg->loss != STDG_LOSS_RESIDUAL) {
        set_error("unknown training loss");
        return STDG_ERR_ARG;
    }
    if (cfg->precision != STDG_FP64 && cfg->precision != STDG_FP32) {
        set_error("model precision must be STDG_FP64 or STDG_FP32");
        return STDG_ERR_ARG;
    }
    if (!(cfg->lr > 0) || !(cfg->beta1 >= 0 && cfg->beta1 < 1) || !(cfg->beta2 >= 0 && cfg->beta2 < 1) ||
        !(cfg->eps > 0)) {
        set_error("invalid Adam parameters");
        return STDG_ERR_ARG;
    }
    stdg_model* md = new stdg_model();
    md->cfg = *cfg;
    md->nst = m->Nst;
    md->E = m->E;
    md->nin = 11 * m->Nst + 4;
    md->hid = cfg->hidden;
    md->nout = m->Nst;
    const int64_t nin = md->nin, H = md->hid, no = md->nout;
    md->oW1 = 0;
    md->ob1 = nin * H;
    md->oW2 = md->ob1 + H;
    md->ob2 = md->oW2 + H * H;
    md->oW3 = md->ob2 + H;
    md->ob3 = md->oW3 + H * no;
    md->np = md->ob3 + no;
    const size_t ts = cfg->precision == STDG_FP64 ? 8 : 4;
    const int64_t bs = cfg->batch;
    auto fail = [&](hipError_t e) {
        set_error(std::string("model allocation: ") + hipGetErrorString(e));
        stdg_model_free(md);
        return STDG_ERR_NOMEM;
    };
    hipError_t e;
    const int64_t part_n = (int64_t)KSPLIT * std::max<int64_t>({nin * H, H * H, H * no});
    struct { void** p; size_t bytes; } al[] = {
        {&md->theta, ts * md->np}, {&md->grad, ts * md->np}, {&md->mom1, ts * md->np}, {&md->mom2, ts * md->np},
        {&md->one, ts}, {&md->F, ts * bs * nin}, {&md->Z1, ts * bs * H}, {&md->H1, ts * bs * H},
        {&md->Z2, ts * bs * H}, {&md->H2, ts * bs * H}, {&md->Y, ts * bs * no}, {&md->dY, ts * bs * no},
        {&md->dZ2, ts * bs * H}, {&md->dZ1, ts * bs * H}, {&md->part, ts * part_n},
        {(void**)&md->lpart, sizeof(double) * NRB}, {(void**)&md->spart, sizeof(double) * 3 * NRB}};
    for (auto& a : al)
        if ((e = hipMalloc(a.p, a.bytes)) != hipSuccess) return fail(e);
    if ((e = hipHostMalloc((void**)&md->hbuf, sizeof(double) * 4)) != hipSuccess) return fail(e);
    // seeded initialisation (uniform Glorot for the hidden layers, scaled for the output layer, zero biases)
    std::vector<double> th(md->np, 0.0);
    std::mt19937_64 rng(cfg->seed);
    auto uni = [&](double a) { return a * (2.0 * ((rng() >> 11) * 0x1.0p-53) - 1.0); };
    const double a1 = std::sqrt(6.0 / (double)(nin + H)), a2 = std::sqrt(6.0 / (double)(2 * H)),
                 a3 = cfg->init_scale_out * std::sqrt(6.0 / (double)(H + no));
    for (int64_t k = 0; k < nin * H; ++k) th[md->oW1 + k] = uni(a1);
    for (int64_t k = 0; k < H * H; ++k) th[md->oW2 + k] = uni(a2);
    for (int64_t k = 0; k < H * no; ++k) th[md->oW3 + k] = uni(a3);
    if (int st = stdg_model_set_params(md, th.data())) { stdg_model_free(md); return st; }
    *out = md;
    return STDG_OK;
}

extern "C" int stdg_model_free(stdg_model* md) {
    if (!md) return STDG_OK;
    for (void* p : {md->theta, md->grad, md->mom1, md->mom2, md->one, md->F, md->Z1, md->H1, md->Z2, md->H2, md->Y,
                    md->dY, md->dZ2, md->dZ1, md->part, (void*)md->lpart, (void*)md->lbatch, (void*)md->scales,
                    (void*)md->spart, (void*)md->idx, (void*)md->ve, (void*)md->vR, (void*)md->vG,
                    (void*)md->CT})
        if (p) (void)hipFree(p);
    if (md->hbuf) (void)hipHostFree(md->hbuf);
    delete md;
    return STDG_OK;
}

extern "C" int stdg_model_info(const stdg_model* md, int64_t* n_params, int32_t* n_in, int32_t* n_out) {
    if (!md) { set_error("null model"); return STDG_ERR_ARG; }
    if (n_params) *n_params = md->np;
    if (n_in) *n_in = md->nin;
    if (n_out) *n_out = md->nout;
    return STDG_OK;
}

namespace {
int copy_params(stdg_model* md, void* dev, const double* host, double* host_out) {
    const int64_t n = md->np;
    if (is64(md)) {
        if (host) STDG_HIP(hipMemcpy(dev, host, sizeof(double) * n, hipMemcpyHostToDevice));
        else STDG_HIP(hipMemcpy(host_out, dev, sizeof(double) * n, hipMemcpyDeviceToHost));
        return STDG_OK;
    }
    std::vector<float> f(n);
    if (host) {
        for (int64_t k = 0; k < n; ++k) f[k] = (float)host[k];
        STDG_HIP(hipMemcpy(dev, f.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    } else {
        STDG_HIP(hipMemcpy(f.data(), dev, sizeof(float) * n, hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < n; ++k) host_out[k] = f[k];
    }
    return STDG_OK;
}
}  // namespace

extern "C" int stdg_model_set_params(stdg_model* md, const double* host) {
    if (!md || !host) { set_error("null argument"); return STDG_ERR_ARG; }
    if (int e = copy_params(md, md->theta, host, nullptr)) return e;
    const size_t ts = is64(md) ? 8 : 4;
    STDG_HIP(hipMemset(md->mom1, 0, ts * md->np));
    STDG_HIP(hipMemset(md->mom2, 0, ts * md->np));
    STDG_HIP(hipMemset(md->grad, 0, ts * md->np));
    if (is64(md)) { const double one = 1.0; STDG_HIP(hipMemcpy(md->one, &one, 8, hipMemcpyHostToDevice)); }
    else { const float one = 1.0f; STDG_HIP(hipMemcpy(md->one, &one, 4, hipMemcpyHostToDevice)); }
    md->t_adam = 0;
    return STDG_OK;
}

extern "C" int stdg_model_get_params(const stdg_model* md, double* host) {
    if (!md || !host) { set_error("null argument"); return STDG_ERR_ARG; }
    return copy_params(const_cast<stdg_model*>(md), md->theta, nullptr, host);
}

extern "C" int stdg_model_get_grads(const stdg_model* md, double* host) {
    if (!md || !host) { set_error("null argument"); return STDG_ERR_ARG; }
    return copy_params(const_cast<stdg_model*>(md), md->grad, nullptr, host);
}

extern "C" int stdg_model_features(stdg_model* md, const stdg_mesh* m, const double* P, const double* Pm,
                                   const double* B, double* F, void* stream) {
    if (int e = check_model(md, m)) return e;
    if (!P || !Pm || !B || !F) { set_error("null vector"); return STDG_ERR_ARG; }
    hipStream_t s = (hipStream_t)stream;
    if (int e = compute_scales(md, P, Pm, B, 1, s)) return e;
    return features_t<double>(md, m, P, Pm, B, nullptr, 0, md->E, F, s);
}

extern "C" int stdg_model_forward(stdg_model* md, const double* F, int64_t n, double* Y, void* stream) {
    if (int e = check_model(md, nullptr)) return e;
    if (!F || !Y || n < 1 || n > md->cfg.batch) { set_error("need 1 <= n <= batch rows and non-null buffers"); return STDG_ERR_ARG; }
    hipStream_t s = (hipStream_t)stream;
    if (is64(md)) {
        STDG_HIP(hipMemcpyAsync(md->F, F, sizeof(double) * n * md->nin, hipMemcpyDeviceToDevice, s));
        if (int e = forward_t<double>(md, n, s)) return e;
        STDG_HIP(hipMemcpyAsync(Y, md->Y, sizeof(double) * n * md->nout, hipMemcpyDeviceToDevice, s));
    } else {
        hipLaunchKernelGGL(k_cvt<float>, dim3(nb256(n * md->nin)), dim3(256), 0, s, F, (float*)md->F, n * md->nin);
        if (int e = forward_t<float>(md, n, s)) return e;
        hipLaunchKernelGGL(k_cvt_back<float>, dim3(nb256(n * md->nout)), dim3(256), 0, s, (const float*)md->Y, Y,
                           n * md->nout);
    }
    MCK(hipGetLastError());
    return STDG_OK;
}

namespace {
int ensure_lbatch(stdg_model* md, int64_t n) {
    if (md->lbatch_n < n) {
        if (md->lbatch) STDG_HIP(hipFree(md->lbatch));
        md->lbatch = nullptr;
        STDG_HIP(hipMalloc(&md->lbatch, sizeof(double) * n));
        md->lbatch_n = n;
    }
    return STDG_OK;
}
}  // namespace

extern "C" int stdg_model_loss_grad(stdg_model* md, const double* F, const double* target, int64_t n, double* loss,
                                    void* stream) {
    if (int e = check_model(md, nullptr)) return e;
    if (!F || !target || n < 1 || n > md->cfg.batch) {
        set_error("need 1 <= n <= batch rows and non-null buffers");
        return STDG_ERR_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    if (int e = ensure_lbatch(md, 1)) return e;
    int e;
    if (is64(md)) {
        STDG_HIP(hipMemcpyAsync(md->F, F, sizeof(double) * n * md->nin, hipMemcpyDeviceToDevice, s));
        if ((e = forward_t<double>(md, n, s)) || (e = mse_t<double>(md, n, target, nullptr, nullptr, nullptr, nullptr, 0,
                                                                    md->lbatch, s)) ||
            (e = backward_t<double>(md, n, s)))
            return e;
    } else {
        hipLaunchKernelGGL(k_cvt<float>, dim3(nb256(n * md->nin)), dim3(256), 0, s, F, (float*)md->F, n * md->nin);
        if ((e = forward_t<float>(md, n, s)) || (e = mse_t<float>(md, n, target, nullptr, nullptr, nullptr, nullptr, 0,
                                                                  md->lbatch, s)) ||
            (e = backward_t<float>(md, n, s)))
            return e;
    }
    STDG_HIP(hipMemcpyAsync(md->hbuf, md->lbatch, sizeof(double), hipMemcpyDeviceToHost, s));
    STDG_HIP(hipStreamSynchronize(s));
    if (loss) *loss = md->hbuf[0];
    return STDG_OK;
}

extern "C" int stdg_model_residual_loss_grad(stdg_model* md, const stdg_mesh* cm, const double* P, const double* Pm,
                                             const double* B, const double* X, double* loss, void* stream) {
    if (int e = check_model(md, cm)) return e;
    if (!P || !Pm || !B || !X) { set_error("null vector"); return STDG_ERR_ARG; }
    if (md->cfg.batch < md->E) { set_error("the residual objective needs batch >= number of elements"); return STDG_ERR_ARG; }
    stdg_mesh* m = const_cast<stdg_mesh*>(cm);
    hipStream_t s = (hipStream_t)stream;
    if (int e = ensure_resid_buffers(md, m)) return e;
    if (int e = compute_scales(md, P, Pm, B, 1, s)) return e;
    double den = 0.0, l = 0.0;
    if (int e = resid_den(md, m, P, Pm, X, 0, den, s)) return e;
    const int e = is64(md) ? resid_step_t<double>(md, m, P, Pm, B, X, 0, den, l, s)
                           : resid_step_t<float>(md, m, P, Pm, B, X, 0, den, l, s);
    if (e) return e;
    STDG_HIP(hipStreamSynchronize(s));
    if (loss) *loss = l;
    return STDG_OK;
}

extern "C" int stdg_model_adam_step(stdg_model* md, void* stream) {
    if (int e = check_model(md, nullptr)) return e;
    return is64(md) ? adam_t<double>(md, (hipStream_t)stream) : adam_t<float>(md, (hipStream_t)stream);
}

extern "C" int stdg_model_predict(stdg_model* md, const stdg_mesh* m, const double* P, const double* Pm,
                                  const double* B, double* x0, void* stream) {
    if (!P || !Pm || !B || !x0) { set_error("null vector"); return STDG_ERR_ARG; }
    return model_predict(md, m, P, Pm, B, x0, (hipStream_t)stream, false);
}

extern "C" int stdg_model_train(stdg_model* md, const stdg_mesh* m, int32_t n_steps, const double* P,
                                const double* Pm, const double* B, const double* X, int32_t epochs,
                                stdg_train_report* rep, void* stream) {
    if (int e = check_model(md, m)) return e;
    if (!P || !Pm || !B || !X || n_steps < 1 || epochs < 1) {
        set_error("need n_steps >= 1, epochs >= 1 and non-null data");
        return STDG_ERR_ARG;
    }
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    if (md->cfg.loss == STDG_LOSS_RESIDUAL) {
        if (md->cfg.batch < md->E) { set_error("the residual objective needs batch >= number of elements"); return STDG_ERR_ARG; }
        stdg_mesh* mm = const_cast<stdg_mesh*>(m);
        if (int e = ensure_resid_buffers(md, mm)) return e;
        if (int e = compute_scales(md, P, Pm, B, n_steps, s)) return e;
        std::vector<double> den(n_steps);
        for (int k = 0; k < n_steps; ++k)
            if (int e = resid_den(md, mm, P, Pm, X, k, den[k], s)) return e;
        std::vector<int> order(n_steps);
        std::iota(order.begin(), order.end(), 0);
        std::mt19937_64 rng(md->cfg.seed ^ 0x5DEECE66DULL);
        double first = 0.0, last = 0.0;
        for (int ep = 0; ep < epochs; ++ep) {
            for (int k = n_steps - 1; k > 0; --k) std::swap(order[k], order[rng() % (uint64_t)(k + 1)]);
            double acc = 0.0;
            for (int k : order) {
                double l = 0.0;
                const int e = is64(md) ? resid_step_t<double>(md, mm, P, Pm, B, X, k, den[k], l, s)
                                       : resid_step_t<float>(md, mm, P, Pm, B, X, k, den[k], l, s);
                if (e) return e;
                if (int e2 = is64(md) ? adam_t<double>(md, s) : adam_t<float>(md, s)) return e2;
                acc += l;
            }
            last = acc / n_steps;
            if (!std::isfinite(last)) { set_error("non-finite training loss"); return STDG_ERR_NUMERIC; }
            if (ep == 0) first = last;
        }
        STDG_HIP(hipStreamSynchronize(s));
        if (rep) {
            rep->epochs = epochs;
            rep->samples = (int64_t)n_steps * md->E;
            rep->first_loss = first;
            rep->last_loss = last;
            rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        return STDG_OK;
    }
    const int64_t total = (int64_t)n_steps * md->E;
    const int64_t bs = md->cfg.batch;
    const int64_t nbatch = (total + bs - 1) / bs;
    if (int e = compute_scales(md, P, Pm, B, n_steps, s)) return e;
    if (int e = ensure_lbatch(md, nbatch)) return e;
    if (md->idx_n < total) {
        if (md->idx) STDG_HIP(hipFree(md->idx));
        md->idx = nullptr;
        STDG_HIP(hipMalloc(&md->idx, sizeof(int64_t) * total));
        md->idx_n = total;
    }
    std::vector<int64_t> order(total);
    std::iota(order.begin(), order.end(), (int64_t)0);
    std::mt19937_64 rng(md->cfg.seed ^ 0x5DEECE66DULL);
    std::vector<double> lb(nbatch);
    double first = 0.0, last = 0.0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int64_t k = total - 1; k > 0; --k) std::swap(order[k], order[rng() % (uint64_t)(k + 1)]);
        STDG_HIP(hipMemcpyAsync(md->idx, order.data(), sizeof(int64_t) * total, hipMemcpyHostToDevice, s));
        for (int64_t b = 0; b < nbatch; ++b) {
            const int64_t r0 = b * bs, n = std::min(bs, total - r0);
            const int64_t* id = md->idx + r0;
            int e;
            if (is64(md)) {
                if ((e = features_t<double>(md, m, P, Pm, B, id, 0, n, (double*)md->F, s)) ||
                    (e = forward_t<double>(md, n, s)) ||
                    (e = mse_t<double>(md, n, nullptr, X, P, Pm, id, 0, md->lbatch + b, s)) ||
                    (e = backward_t<double>(md, n, s)) || (e = adam_t<double>(md, s)))
                    return e;
            } else {
                if ((e = features_t<float>(md, m, P, Pm, B, id, 0, n, (float*)md->F, s)) ||
                    (e = forward_t<float>(md, n, s)) ||
                    (e = mse_t<float>(md, n, nullptr, X, P, Pm, id, 0, md->lbatch + b, s)) ||
                    (e = backward_t<float>(md, n, s)) || (e = adam_t<float>(md, s)))
                    return e;
            }
        }
        STDG_HIP(hipMemcpyAsync(lb.data(), md->lbatch, sizeof(double) * nbatch, hipMemcpyDeviceToHost, s));
        STDG_HIP(hipStreamSynchronize(s));
        double acc = 0.0;
        for (int64_t b = 0; b < nbatch; ++b) acc += lb[b] * (double)std::min(bs, total - b * bs);
        last = acc / (double)total;
        if (!std::isfinite(last)) { set_error("non-finite training loss"); return STDG_ERR_NUMERIC; }
        if (ep == 0) first = last;
    }
    if (rep) {
        rep->epochs = epochs;
        rep->samples = total;
        rep->first_loss = first;
        rep->last_loss = last;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return STDG_OK;
}
