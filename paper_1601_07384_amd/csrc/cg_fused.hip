// Fused conjugate-gradient iteration for the FP32 inner solves of the
// pressure system (eq. CS_19) when the operator is B (x) I: the spatial
// Schur operator B = dt^2 S^sp on every time node (the time-decoupled form of
// S = B (x) C, or p_gamma = 0 where C is the scalar 1).
//
// Iteration i is two kernels:
//   k_cg_spmv : rr_i = sum of the previous update's partials, beta_i =
//               rr_i / rr_{i-1}, p_i = r_i + beta_i p_{i-1} (formed while the
//               operand panels are staged), q_i = B p_i on MFMA, per-block
//               partials of p_i . q_i;
//   k_cg_upd  : alpha_i = rr_i / (p_i . q_i) from those partials,
//               x += alpha_i p_i, r -= alpha_i q_i, per-block partials of r.r.
// Every block re-adds the previous kernel's partials in the same fixed order,
// so all blocks hold bitwise-identical scalars without any cross-block
// synchronisation inside a kernel, and results are deterministic.  rr_i is
// kept in slot s_rr + (i & 1) (written by block 0 of k_cg_spmv); the other
// slot still holds rr_{i-1} for the blocks that are reading it.
//
// k_cg_spmv: four wavefronts per block, one wavefront per (16-element tile,
// time node).  Elements are stored class-chunked, so a tile shares one
// geometry class: the five N x N blocks of the class are the A operands of
// v_mfma_f32_16x16x4f32 and the 16 elements are its 16 columns.  All five
// operand panels (own rows and the neighbours across the four faces) are
// gathered in one batch of vector loads into the wavefront's LDS, so a
// wavefront waits for memory once.  Tiles that mix classes (the tail of a
// mesh with many classes) run one MFMA pass per class present, with the other
// classes' columns masked.

#include "internal.hpp"
#include "kernels.hpp"

namespace stdg {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline double wave_add(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Ordered sum of part[0 .. n) by a 256-thread block; every thread gets it.
__device__ double block_total(const double* __restrict__ part, int64_t n, double* sh) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += part[i];
    s = wave_add(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    const double t = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return t;
}

// LDS written by some lanes of a wavefront and read by others: wait for the
// wavefront's LDS operations and keep the compiler from moving accesses.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <int N> struct RowVec;     // widest aligned vector load of a row of N floats
template <> struct RowVec<4> { typedef float4 T; static constexpr int W = 4; };
template <> struct RowVec<10> { typedef float2 T; static constexpr int W = 2; };
template <> struct RowVec<20> { typedef float4 T; static constexpr int W = 4; };

__device__ inline float4 vfma(float4 r, float b, float4 p) {
    return float4(r.x + b * p.x, r.y + b * p.y, r.z + b * p.z, r.w + b * p.w);
}
__device__ inline float2 vfma(float2 r, float b, float2 p) { return float2(r.x + b * p.x, r.y + b * p.y); }
__device__ inline void vput(float* d, const float4& v) { d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w; }
__device__ inline void vput(float* d, const float2& v) { d[0] = v.x; d[1] = v.y; }

template <int N>
__global__ void __launch_bounds__(256) k_cg_spmv(const float* __restrict__ BT, const int32_t* __restrict__ cls,
                                                 const int32_t* __restrict__ nbr, const float* __restrict__ r,
                                                 const float* __restrict__ pold, float* __restrict__ pnew,
                                                 float* __restrict__ q, double* __restrict__ scal, int s_rr,
                                                 int iter, float cscale, int64_t E, int G,
                                                 const double* __restrict__ upart, int64_t n_upart,
                                                 double* __restrict__ spart) {
    constexpr int MT = (N + 15) / 16, KS = (N + 3) / 4, LD = N + 1;
    typedef typename RowVec<N>::T V;
    constexpr int W = RowVec<N>::W, CPR = N / W;          // vectors per row
    constexpr int NVEC = 5 * 16 * CPR;                     // vectors of the five panels
    __shared__ float pan[4][5 * 16 * LD];
    __shared__ int32_t rows[4][5 * 16];
    __shared__ double sh[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float* P = pan[wave];
    // rr_i and beta_i (identical in every block)
    const double rr = block_total(upart, n_upart, sh);
    const double rr_prev = scal[s_rr + ((iter + 1) & 1)];
    const float beta = (iter == 0 || !(rr_prev > 0.0)) ? 0.0f : (float)(rr / rr_prev);
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[s_rr + (iter & 1)] = rr;
    // wavefront = 16 elements (the 16 MFMA columns) at time node a.  The
    // hardware deals consecutive workgroups round-robin to the 8 XCDs (each
    // with its own L2); give XCD x the contiguous range of tiles x * per ..,
    // so neighbouring elements are gathered through the same L2.
    const int64_t per = gridDim.x / 8;
    const int64_t lblock = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    const int64_t ntile = (E + 15) / 16;
    const int64_t wid = lblock * 4 + wave;
    const bool active = wid < ntile * G;
    const int a = active ? (int)(wid % G) : 0;
    const int64_t e0 = active ? (wid / G) * 16 : 0;
    const int col = lane & 15;
    const bool vcol = active && e0 + col < E;
    const int c = vcol ? cls[e0 + col] : -1;
    const int c0 = __builtin_amdgcn_readfirstlane(c);
    const bool uniform = __all(!vcol || c == c0);
    // element of each panel row: slot k (own element, then the neighbours
    // across local faces 0..3), row = column; -1 for none
    for (int t = lane; t < 80; t += 64) {
        const int k = t >> 4, rw = t & 15;
        const int64_t er = e0 + rw;
        int32_t v = -1;
        if (active && er < E) v = k == 0 ? (int32_t)er : nbr[4 * er + k - 1];
        rows[wave][t] = v;
    }
    // A operands of a single-class tile, loaded while the panels stream in
    // (lane l supplies row l % 16 of A, whatever the validity of column l % 16)
    float aop[5][MT][KS];
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) aop[k][mt][ks] = 0.0f;
    if (uniform && active) {
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const int row = mt * 16 + (lane & 15), m = ks * 4 + (lane >> 4);
                    aop[k][mt][ks] = (row < N && m < N) ? BT[((int64_t)c0 * 5 + k) * N * N + m * N + row] : 0.0f;
                }
    }
    wave_lds_sync();
    // stage the five panels: p = r + beta p_old of every row (own rows also
    // written to p_new)
#pragma unroll
    for (int f0 = 0; f0 < NVEC; f0 += 64) {
        const int f = f0 + lane;
        if (f < NVEC) {
            const int k = f / (16 * CPR), rem = f % (16 * CPR);
            const int rw = rem / CPR, j = rem % CPR;
            const int32_t t = rows[wave][k * 16 + rw];
            V v;
            if (t >= 0) {
                const int64_t o = ((int64_t)t * G + a) * N + j * W;
                v = vfma(*(const V*)(r + o), beta, *(const V*)(pold + o));
                if (k == 0) *(V*)(pnew + o) = v;
            } else {
                v = V(0.0f);
            }
            vput(P + (k * 16 + rw) * LD + j * W, v);
        }
    }
    wave_lds_sync();
    f4 acc[MT];
#pragma unroll
    for (int i = 0; i < MT; ++i) acc[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    if (uniform) {
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int m = ks * 4 + (lane >> 4);
                const float bop = m < N ? P[(k * 16 + col) * LD + m] : 0.0f;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[k][mt][ks], bop, acc[mt], 0, 0, 0);
            }
    } else {
        // one MFMA pass per class present; other classes' columns masked
        uint64_t todo = __ballot(vcol && lane < 16);
        while (todo) {
            const int lead = __builtin_ctzll(todo);
            const int cur = __builtin_amdgcn_readlane(c, lead);
            const bool mine = vcol && c == cur;
            todo &= ~__ballot(mine && lane < 16);
            for (int k = 0; k < 5; ++k) {
                const float* Bk = BT + ((int64_t)cur * 5 + k) * N * N;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const int m = ks * 4 + (lane >> 4);
                    const float bop = (m < N && mine) ? P[(k * 16 + col) * LD + m] : 0.0f;
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        const int row = mt * 16 + (lane & 15);
                        const float av = (row < N && m < N) ? Bk[m * N + row] : 0.0f;
                        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bop, acc[mt], 0, 0, 0);
                    }
                }
            }
        }
    }
    // q and the partial p . q; result register j of lane l holds row
    // 4 (l / 16) + j of column l % 16
    double dot = 0.0;
    if (vcol) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = mt * 16 + 4 * (lane >> 4) + j;
                if (row < N) {
                    const float qv = cscale * acc[mt][j];
                    q[((e0 + col) * G + a) * N + row] = qv;
                    dot += (double)P[col * LD + row] * (double)qv;
                }
            }
    }
    dot = wave_add(dot);
    if (lane == 0) sh[wave] = dot;
    __syncthreads();
    if (threadIdx.x == 0) spart[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// alpha = rr_i / (p.q); x += alpha p, r -= alpha q; per-block partials of r.r
__global__ void __launch_bounds__(256) k_cg_upd(float* __restrict__ x, float* __restrict__ r,
                                                const float* __restrict__ p, const float* __restrict__ q,
                                                const double* __restrict__ scal, int s_rr, int iter, int64_t n,
                                                const double* __restrict__ spart, int64_t n_spart,
                                                double* __restrict__ upart) {
    __shared__ double sh[4];
    const double pq = block_total(spart, n_spart, sh);
    const double rr = scal[s_rr + (iter & 1)];
    const float alpha = (pq > 0.0 && rr > 0.0) ? (float)(rr / pq) : 0.0f;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        x[i] += alpha * p[i];
        const float ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += (double)ri * (double)ri;
    }
    acc = wave_add(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) upart[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

template <int N>
hipError_t spmv_n(const stdg_mesh* m, const float* r, const float* pold, float* pnew, float* q, double* scal,
                  int s_rr, int iter, float cscale, const double* upart, int64_t n_upart, double* spart,
                  hipStream_t s) {
    hipLaunchKernelGGL((k_cg_spmv<N>), dim3((unsigned)cg_spmv_blocks(m)), dim3(256), 0, s, m->d.blocks32, m->d.cls,
                       m->d.nbr, r, pold, pnew, q, scal, s_rr, iter, cscale, m->E, m->G, upart, n_upart, spart);
    return hipGetLastError();
}

}  // namespace

bool cg_fused_supported(const stdg_mesh* m) {
    return m->N == 4 || m->N == 10 || m->N == 20;
}

int64_t cg_spmv_blocks(const stdg_mesh* m) {
    const int64_t waves = (m->E + 15) / 16 * m->G;
    return ((waves + 3) / 4 + 7) / 8 * 8;       // a multiple of the 8 XCDs
}

hipError_t launch_cg_spmv_f32(const stdg_mesh* m, const float* r, const float* pold, float* pnew, float* q,
                              double* scal, int s_rr, int iter, float cscale, const double* upart,
                              int64_t n_upart, double* spart, hipStream_t s) {
    switch (m->N) {
        case 4: return spmv_n<4>(m, r, pold, pnew, q, scal, s_rr, iter, cscale, upart, n_upart, spart, s);
        case 10: return spmv_n<10>(m, r, pold, pnew, q, scal, s_rr, iter, cscale, upart, n_upart, spart, s);
        case 20: return spmv_n<20>(m, r, pold, pnew, q, scal, s_rr, iter, cscale, upart, n_upart, spart, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cg_upd_f32(float* x, float* r, const float* p, const float* q, const double* scal, int s_rr,
                             int iter, int64_t n, const double* spart, int64_t n_spart, double* upart,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_cg_upd, dim3(CG_UPD_BLOCKS), dim3(256), 0, s, x, r, p, q, scal, s_rr, iter, n, spart,
                       n_spart, upart);
    return hipGetLastError();
}

}  // namespace stdg
