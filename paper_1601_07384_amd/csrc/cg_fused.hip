// Fused conjugate-gradient iteration for the FP32 inner solves of the
// pressure system (eq. CS_19) when the operator is B (x) I: the spatial
// Schur operator B = dt^2 S^sp on every time node (the time-decoupled form of
// S = B (x) C, or p_gamma = 0 where C is the scalar 1).
//
// One CG iteration is one operator kernel, k_cg_op<N, ITER>, after a
// one-block kernel k_cg_red that adds up the previous launch's per-block
// partials in a fixed order (deterministic).  The dot products of an
// iteration ((p.q), (r.q), (q.q) and (r.r)) are all reduced at its end, and
// the next iteration takes alpha_{i-1} = (r.r)_{i-1} / (p.q)_{i-1} and, from
// the expansion of |r_{i-1} - alpha q_{i-1}|^2,
//   rr_i = (r.r)_{i-1} - 2 alpha (r.q)_{i-1} + alpha^2 (q.q)_{i-1},
// beta_i = rr_i / (r.r)_{i-1} (the single-reduction form of Chronopoulos &
// Gear, with the recurrence restarted every iteration from the reduced r.r).
// Iteration i forms, for every row it touches (its own 16 elements and their
// face neighbours),
//   r_i = r_{i-1} - alpha_{i-1} q_{i-1},  p_i = r_i + beta_i p_{i-1},
// applies q_i = B p_i on MFMA, writes r_i, p_i, q_i of its own rows to the
// other buffer of each pair (neighbour rows are still being read from the
// current one) and adds alpha_{i-1} p_{i-1} to x.  After the last iteration
// k_cg_tail adds alpha_i p_i to x.
//
// Four wavefronts per block, one wavefront per (16-element tile, time node).
// Elements are stored class-chunked, so a tile shares one geometry class:
// the five N x N blocks of the class are the A operands of
// v_mfma_f32_16x16x4f32 and the 16 elements are its 16 columns.  All five
// operand panels (own rows and the neighbours across the four faces) are
// gathered in one batch of vector loads into the wavefront's LDS, so a
// wavefront waits for memory once.  Tiles that mix classes (the tail of a
// mesh with many classes) run one MFMA pass per class present, with the other
// classes' columns masked.  With ITER = false the kernel is the plain
// operator y = B x (no CG state).

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

// Ordered sums of the 4-vectors part[4 b + c], b < n, by a 256-thread block;
// every thread gets all four.
__device__ void block_total4(const double* __restrict__ part, int64_t n, double (&out)[4], double* sh) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < n; i += 256)
#pragma unroll
        for (int c = 0; c < 4; ++c) s[c] += part[4 * i + c];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double v = wave_add(s[c]);
        if ((threadIdx.x & 63) == 0) sh[4 * (threadIdx.x >> 6) + c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; ++c) out[c] = ((sh[c] + sh[4 + c]) + sh[8 + c]) + sh[12 + c];
    __syncthreads();
}

// CG scalars of iteration `iter` from the partials of the previous one:
// alpha_{i-1} = (r.r)_{i-1} / (p.q)_{i-1} with the true (r.r)_{i-1}, and
// rr_i by one step of the recurrence from it (restarting the recurrence from
// the reduced r.r every iteration keeps its rounding from accumulating).
struct CgScalars {
    double alpha;    // alpha_{i-1}
    double beta;     // beta_i
};

__device__ CgScalars cg_scalars(int iter, const double* __restrict__ part, int64_t n_part, double* sh) {
    CgScalars c{0.0, 0.0};
    if (iter == 0) return c;
    double t[4];
    block_total4(part, n_part, t, sh);
    const double pq = t[0], rq = t[1], qq = t[2], rr_prev = t[3];
    c.alpha = (pq > 0.0 && rr_prev > 0.0) ? rr_prev / pq : 0.0;
    const double rr = fmax(rr_prev - 2.0 * c.alpha * rq + c.alpha * c.alpha * qq, 0.0);
    c.beta = rr_prev > 0.0 ? rr / rr_prev : 0.0;
    return c;
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

__device__ inline float4 vaxpy(float4 y, float a, float4 x) {
    return float4(y.x + a * x.x, y.y + a * x.y, y.z + a * x.z, y.w + a * x.w);
}
__device__ inline float2 vaxpy(float2 y, float a, float2 x) { return float2(y.x + a * x.x, y.y + a * x.y); }
__device__ inline void vput(float* d, const float4& v) { d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w; }
__device__ inline void vput(float* d, const float2& v) { d[0] = v.x; d[1] = v.y; }

template <int N, bool ITER>
__global__ void __launch_bounds__(256) k_cg_op(const float* __restrict__ BT, const int32_t* __restrict__ cls,
                                               const int32_t* __restrict__ nbr, float* __restrict__ x,
                                               const float* __restrict__ r_in, const float* __restrict__ p_in,
                                               const float* __restrict__ q_in, float* __restrict__ r_out,
                                               float* __restrict__ p_out, float* __restrict__ q_out,
                                               const double* __restrict__ ab, float cscale,
                                               int64_t E, int G, double* __restrict__ part_out) {
    constexpr int MT = (N + 15) / 16, KS = (N + 3) / 4, LD = N + 1;
    typedef typename RowVec<N>::T V;
    constexpr int W = RowVec<N>::W, CPR = N / W;          // vectors per row
    constexpr int NVEC = 5 * 16 * CPR;                     // vectors of the five panels
    __shared__ float pan[4][5 * 16 * LD];
    __shared__ float rown[4][16 * LD];                     // own r_i rows (for r.q, r.r)
    __shared__ int32_t rows[4][5 * 16];
    __shared__ double sh[16];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float* P = pan[wave];
    float* R = rown[wave];
    float alpha = 0.0f, beta = 0.0f;
    if (ITER) {
        alpha = (float)ab[0];
        beta = (float)ab[1];
    }
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
    // stage the five panels (CG: r_i = r - alpha q, p_i = r_i + beta p; own
    // rows also written out, and x += alpha p_{i-1})
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
                if (ITER) {
                    const V pv = *(const V*)(p_in + o);
                    const V rv = vaxpy(*(const V*)(r_in + o), -alpha, *(const V*)(q_in + o));
                    v = vaxpy(rv, beta, pv);
                    if (k == 0) {
                        *(V*)(r_out + o) = rv;
                        *(V*)(p_out + o) = v;
                        *(V*)(x + o) = vaxpy(*(const V*)(x + o), alpha, pv);
                        vput(R + rw * LD + j * W, rv);
                    }
                } else {
                    v = *(const V*)(r_in + o);
                }
            } else {
                v = V(0.0f);
                if (ITER && k == 0) vput(R + rw * LD + j * W, v);
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
    // q of the own rows and the partial dot products; result register j of
    // lane l holds row 4 (l / 16) + j of column l % 16
    double d[4] = {0.0, 0.0, 0.0, 0.0};
    if (vcol) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = mt * 16 + 4 * (lane >> 4) + j;
                if (row < N) {
                    const float qv = cscale * acc[mt][j];
                    q_out[((e0 + col) * G + a) * N + row] = qv;
                    if (ITER) {
                        const double pv = P[col * LD + row], rv = R[col * LD + row];
                        d[0] += pv * (double)qv;
                        d[1] += rv * (double)qv;
                        d[2] += (double)qv * (double)qv;
                        d[3] += rv * rv;
                    }
                }
            }
    }
    if (ITER) {
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const double v = wave_add(d[cc]);
            if (lane == 0) sh[4 * wave + cc] = v;
        }
        __syncthreads();
        if (threadIdx.x < 4) {
            const int cc = threadIdx.x;
            part_out[4 * blockIdx.x + cc] = ((sh[cc] + sh[4 + cc]) + sh[8 + cc]) + sh[12 + cc];
        }
    }
}

// ab[0..1] = (alpha_{i-1}, beta_i) from the previous iteration's partials (one block)
__global__ void __launch_bounds__(256) k_cg_red(const double* __restrict__ part, int64_t n_part, int iter,
                                                double* __restrict__ ab) {
    __shared__ double sh[16];
    const CgScalars c = cg_scalars(iter, part, n_part, sh);
    if (threadIdx.x == 0) {
        ab[0] = c.alpha;
        ab[1] = c.beta;
    }
}

// x += alpha_i p_i after the last iteration i (alpha_i from its partials)
__global__ void __launch_bounds__(256) k_cg_tail(float* __restrict__ x, const float* __restrict__ p, int64_t n,
                                                 const double* __restrict__ part, int64_t n_part) {
    __shared__ double sh[16];
    double t[4];
    block_total4(part, n_part, t, sh);
    const float alpha = (t[0] > 0.0 && t[3] > 0.0) ? (float)(t[3] / t[0]) : 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        x[i] += alpha * p[i];
}

// scal[slot] = sum_b part[4 b + comp] (one block)
__global__ void __launch_bounds__(256) k_fin4(const double* __restrict__ part, int64_t n, int comp,
                                              double* __restrict__ scal, int slot) {
    __shared__ double sh[4];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += part[4 * i + comp];
    s = wave_add(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) scal[slot] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

template <int N, bool ITER>
hipError_t op_n(const stdg_mesh* m, float* x, const float* r_in, const float* p_in, const float* q_in, float* r_out,
                float* p_out, float* q_out, const double* ab, float cscale, double* part_out, hipStream_t s) {
    hipLaunchKernelGGL((k_cg_op<N, ITER>), dim3((unsigned)cg_op_blocks(m)), dim3(256), 0, s, m->d.blocks32, m->d.cls,
                       m->d.nbr, x, r_in, p_in, q_in, r_out, p_out, q_out, ab, cscale, m->E, m->G, part_out);
    return hipGetLastError();
}

}  // namespace

bool cg_fused_supported(const stdg_mesh* m) {
    return m->N == 4 || m->N == 10 || m->N == 20;
}

int64_t cg_op_blocks(const stdg_mesh* m) {
    const int64_t waves = (m->E + 15) / 16 * m->G;
    return ((waves + 3) / 4 + 7) / 8 * 8;       // a multiple of the 8 XCDs
}

hipError_t launch_cg_iter_f32(const stdg_mesh* m, float* x, const float* r_in, const float* p_in, const float* q_in,
                              float* r_out, float* p_out, float* q_out, int iter, float cscale,
                              const double* part_in, int64_t n_in, double* part_out, double* ab, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_red, dim3(1), dim3(256), 0, s, part_in, n_in, iter, ab);
#define STDG_OPN(n) \
    case n: return op_n<n, true>(m, x, r_in, p_in, q_in, r_out, p_out, q_out, ab, cscale, part_out, s);
    switch (m->N) {
        STDG_OPN(4) STDG_OPN(10) STDG_OPN(20)
        default: return hipErrorInvalidValue;
    }
#undef STDG_OPN
}

hipError_t launch_cg_apply_f32(const stdg_mesh* m, const float* x, float* y, float cscale, hipStream_t s) {
#define STDG_OPN(n)                                                                                             \
    case n: return op_n<n, false>(m, nullptr, x, nullptr, nullptr, nullptr, nullptr, y, nullptr, cscale, nullptr, s);
    switch (m->N) {
        STDG_OPN(4) STDG_OPN(10) STDG_OPN(20)
        default: return hipErrorInvalidValue;
    }
#undef STDG_OPN
}

hipError_t launch_cg_tail_f32(float* x, const float* p, int64_t n, const double* part, int64_t n_part,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_cg_tail, dim3(CG_UPD_BLOCKS), dim3(256), 0, s, x, p, n, part, n_part);
    return hipGetLastError();
}

hipError_t launch_cg_check_f32(const double* part, int64_t n_part, double* scal, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_fin4, dim3(1), dim3(256), 0, s, part, n_part, 3, scal, slot);
    return hipGetLastError();
}

}  // namespace stdg
