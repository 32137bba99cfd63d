// Fused (block-Jacobi preconditioned) conjugate-gradient iteration for the
// FP32 inner solves of the pressure system (eq. CS_19) when the operator is
// A = c B (x) I: the spatial Schur operator B = dt^2 S^sp on every time node
// (the time-decoupled form of S = B (x) C, or p_gamma = 0 where C is the
// scalar c).  The preconditioner is M = c diag(B_e): each element's own
// diagonal block of its class (SPD as a principal block of B), inverted once
// per class on the host.
//
// The iteration carries z = M^-1 r and w = M^-1 q instead of r and q, so a
// neighbour row of p_i needs the same three vectors as unpreconditioned CG:
//   z_i = z_{i-1} - alpha_{i-1} w_{i-1},  p_i = z_i + beta_i p_{i-1},
// and x_i = x_{i-1} + alpha_{i-1} p_{i-1}; the own rows then give
// q_i = A p_i (MFMA over the five class blocks), w_i = M^-1 q_i and
// r_i = M z_i (one extra MFMA set each, on the own block), and the partial
// dot products (p.q), (q.z), (q.w), (r.z) and (r.r).  One CG iteration is
// one such kernel, k_cg_op<N, ITER>, after a one-block kernel k_cg_red that
// adds up the previous launch's per-block partials in a fixed order
// (deterministic) and takes alpha_{i-1} = (r.z)_{i-1} / (p.q)_{i-1} and,
// from the expansion of (r - alpha q) . M^-1 (r - alpha q),
//   rz_i = (r.z)_{i-1} - 2 alpha (q.z)_{i-1} + alpha^2 (q.w)_{i-1},
// beta_i = rz_i / (r.z)_{i-1} (the single-reduction form of Chronopoulos &
// Gear, with the recurrence restarted every iteration from the reduced r.z).
// Without the preconditioner (M = I) the same kernel is plain CG: z = r,
// w = q.  Every launch writes its own rows of z_i, p_i, w_i to the other
// buffer of each pair (neighbour rows are still being read from the current
// one).  After the last iteration k_cg_tail adds alpha_i p_i to x.
//
// One wavefront per (16-element tile, time node), registers only.  Lane l
// serves element column l % 16 of the tile and holds a fixed slice of KS of
// the element's N values (slice_dof below): W consecutive values from
// W * (l / 16), then value 4 W + l / 16.  The slice is at once the lane's B
// operand of v_mfma_f32_16x16x4f32 (the contraction index of K step ks is
// slice position ks of lane group l / 16) and the lane's share of the result
// (the rows of the class blocks are permuted at upload so that the result
// registers of lane l are its own slice), so gathering a neighbour row, the
// CG update of it, the products and the dot products need no lane exchange.
// The class blocks are stored in MFMA operand order (upload_cg_operands):
// float4 i of lane l at [class][i][l]; a workgroup copies the operands of its
// class into LDS once and its wavefronts read them from there.  All
// global loads of a wavefront are issued before the first is used; rows that
// do not exist (boundary faces, the ragged end of the last tile) read through
// a buffer resource at an offset past its end, which returns zeros, and
// their stores are dropped the same way.  Elements are stored class-chunked,
// so a tile shares one geometry class; a tile that mixes classes (the tail of
// a mesh with many classes) runs one MFMA pass per class present, with the
// other classes' columns masked.  With ITER = false the kernel is the plain
// operator y = A x (no CG state).

#include <algorithm>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

namespace stdg {

// Lane slice of an element row of N values: width of the aligned vector part
// and the number of lane groups holding one extra value.
template <int N> struct Slice;
template <> struct Slice<4> { static constexpr int W = 1, REM = 0; };
template <> struct Slice<10> { static constexpr int W = 2, REM = 2; };
template <> struct Slice<20> { static constexpr int W = 4, REM = 4; };

template <int N> struct SliceShape {
    static constexpr int W = Slice<N>::W, REM = Slice<N>::REM;
    static constexpr int KS = W + (REM > 0 ? 1 : 0);     // values per lane = MFMA K steps
    static constexpr int MT = (KS + 3) / 4;              // 16-row MFMA tiles of the result
    static constexpr int NB = MT * KS;                   // operands per lane of one block
    static constexpr int NA = (5 * NB + 3) / 4 * 4;      // the five blocks, padded to float4
    static constexpr int NI = (NB + 3) / 4 * 4;          // the own block's inverse, padded
    static constexpr int NT = NA + NI;                   // operands per lane and class
};

// Row value held at slice position s by lane group kk, or -1 (padding).
__host__ __device__ constexpr int slice_dof(int W, int REM, int s, int kk) {
    return s < W ? W * kk + s : (s == W && kk < REM ? 4 * W + kk : -1);
}

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef __amdgpu_buffer_rsrc_t Rsrc;

constexpr uint32_t OOB = 0x80000000u;   // byte offset past every buffer: loads give 0, stores are dropped
constexpr int RED_T = 1024;             // threads of the one-block reductions
constexpr int WPB = 4;                  // wavefronts per workgroup of the operator kernel (8 measured slower)
constexpr int NPART = 5;                // partial dot products per block ...
constexpr int PSTRIDE = 8;              // ... stored with this stride (doubles)

__device__ inline Rsrc make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <int W> __device__ inline void bload(Rsrc r, uint32_t off, float* v) {
    if constexpr (W == 4) {
        const f4 t = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else if constexpr (W == 2) {
        const f2 t = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
        v[0] = t.x; v[1] = t.y;
    } else {
        v[0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
    }
}

template <int W> __device__ inline void bstore(Rsrc r, uint32_t off, const float* v) {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    if constexpr (W == 4) {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, f4{v[0], v[1], v[2], v[3]}), r, (int)off, 0, 0);
    } else if constexpr (W == 2) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, f2{v[0], v[1]}), r, (int)off, 0, 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v[0]), r, (int)off, 0, 0);
    }
}

// Operands i0 .. i0 + n of the lane from a [i / 4][lane][4] table (global or LDS).
template <int NV> __device__ inline void ops_load(const f4* src, int lane, int i0, float* dst) {
#pragma unroll
    for (int i = 0; i < NV / 4; ++i) {
        const f4 t = src[64 * (i0 / 4 + i) + lane];
        dst[4 * i] = t.x; dst[4 * i + 1] = t.y; dst[4 * i + 2] = t.z; dst[4 * i + 3] = t.w;
    }
}

// acc += (one class block, operands ops[mt * KS + ks]) x (slice b, masked)
template <int KS, int MT>
__device__ inline void mfma_block(const float* ops, const float* b, bool mine, f4* acc) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
            acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ops[mt * KS + ks], mine ? b[ks] : 0.0f, acc[mt], 0, 0, 0);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Wavefront totals of four values: every lane gets the total of component
// lane / 16 (the halving exchange sends two values across 32 lanes and one
// across 16 before the plain butterfly; the order is fixed).
__device__ inline double wave_total4(double a0, double a1, double a2, double a3) {
    const int lane = threadIdx.x & 63;
    const bool hi32 = lane & 32, hi16 = lane & 16;
    double k0 = hi32 ? a2 : a0, k1 = hi32 ? a3 : a1;
    k0 += __shfl_xor(hi32 ? a0 : a2, 32, 64);
    k1 += __shfl_xor(hi32 ? a1 : a3, 32, 64);
    double k = hi16 ? k1 : k0;
    k += __shfl_xor(hi16 ? k0 : k1, 16, 64);
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) k += __shfl_xor(k, o, 64);
    return k;
}

// Ordered sums of the partial vectors part[PSTRIDE b + c], b < n, c < NPART,
// by one block of RED_T threads; every thread gets all of them (sh holds
// NPART * RED_T / 64 + NPART doubles).
__device__ void block_totals(const double* __restrict__ part, int64_t n, double (&out)[NPART], double* sh) {
    const Rsrc rp = make_rsrc(part, (uint32_t)(8 * PSTRIDE * n));
    double s[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t b0 = 0; b0 < n; b0 += 4 * RED_T) {
        d2 v[4][2];
        double v4[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t b = b0 + threadIdx.x + j * RED_T;
            const uint32_t off = b < n ? (uint32_t)(8 * PSTRIDE * b) : OOB;
            v[j][0] = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rp, (int)off, 0, 0));
            v[j][1] = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rp, (int)off, 16, 0));
            v4[j] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rp, (int)off, 32, 0));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            s[0] += v[j][0].x; s[1] += v[j][0].y; s[2] += v[j][1].x; s[3] += v[j][1].y; s[4] += v4[j];
        }
    }
    const double w = wave_total4(s[0], s[1], s[2], s[3]);
    const double w4 = wave_sum(s[4]);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 15) == 0) sh[NPART * wv + ((threadIdx.x >> 4) & 3)] = w;
    if ((threadIdx.x & 63) == 0) sh[NPART * wv + 4] = w4;
    __syncthreads();
    if (threadIdx.x < NPART) {
        double t = 0.0;
        for (int k = 0; k < RED_T / 64; ++k) t += sh[NPART * k + threadIdx.x];
        sh[NPART * RED_T / 64 + threadIdx.x] = t;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NPART; ++c) out[c] = sh[NPART * RED_T / 64 + c];
    __syncthreads();
}

// CG scalars of iteration `iter` from the partials of the previous one:
// alpha_{i-1} = (r.z)_{i-1} / (p.q)_{i-1} with the true (r.z)_{i-1}, and
// rz_i by one step of the recurrence from it (restarting the recurrence from
// the reduced r.z every iteration keeps its rounding from accumulating).
__global__ void __launch_bounds__(RED_T) k_cg_red(const double* __restrict__ part, int64_t n_part, int iter,
                                                  double* __restrict__ ab) {
    __shared__ double sh[NPART * RED_T / 64 + NPART];
    double alpha = 0.0, beta = 0.0;
    if (iter > 0) {
        double t[NPART];
        block_totals(part, n_part, t, sh);
        const double pq = t[0], qz = t[1], qw = t[2], rz_prev = t[3];
        alpha = (pq > 0.0 && rz_prev > 0.0) ? rz_prev / pq : 0.0;
        const double rz = fmax(rz_prev - 2.0 * alpha * qz + alpha * alpha * qw, 0.0);
        beta = rz_prev > 0.0 ? rz / rz_prev : 0.0;
    }
    if (threadIdx.x == 0) {
        ab[0] = alpha;
        ab[1] = beta;
    }
}

// x += alpha p with alpha = ab[0]
__global__ void __launch_bounds__(256) k_cg_tail(float* __restrict__ x, const float* __restrict__ p, int64_t n,
                                                 const double* __restrict__ ab) {
    const float alpha = (float)ab[0];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        x[i] += alpha * p[i];
}

// scal[slot] = (r.r) of the partials (one block)
__global__ void __launch_bounds__(RED_T) k_fin_rr(const double* __restrict__ part, int64_t n,
                                                  double* __restrict__ scal, int slot) {
    __shared__ double sh[NPART * RED_T / 64 + NPART];
    double t[NPART];
    block_totals(part, n, t, sh);
    if (threadIdx.x == 0) scal[slot] = t[4];
}

// Wavefront position: tile = wid / G by the multiplier gmul = ceil(2^32 / G)
// (exact for wid < 2^32 / G), time node a; the hardware deals consecutive
// workgroups round-robin to the 8 XCDs (each with its own L2), so XCD x is
// given the contiguous range of tiles x * per .., and neighbouring elements
// are gathered through the same L2.
struct TilePos {
    uint32_t lblock, tile;
    int a;
    bool active;
};
template <int WB>
__device__ inline TilePos tile_pos(int wave, int32_t E, int32_t G, uint64_t gmul) {
    TilePos t;
    t.lblock = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    const uint32_t wid = t.lblock * WB + (uint32_t)__builtin_amdgcn_readfirstlane(wave);
    t.tile = (uint32_t)(((uint64_t)wid * gmul) >> 32);
    t.active = t.tile < ((uint32_t)E + 15) / 16;
    t.a = t.active ? (int)(wid - t.tile * (uint32_t)G) : 0;
    return t;
}

template <int N, bool ITER>
__global__ void __launch_bounds__(64 * WPB) k_cg_op(const float* __restrict__ A, const int32_t* __restrict__ cls,
                                               const int32_t* __restrict__ nbr, float* x, const float* r_in,
                                               const float* p_in, const float* q_in, float* r_out, float* p_out,
                                               float* q_out, const double* __restrict__ ab, float cscale,
                                               int precond, int32_t E, int32_t G, uint64_t gmul, uint32_t vbytes,
                                               double* __restrict__ part_out) {
    typedef SliceShape<N> S;
    constexpr int W = S::W, REM = S::REM, KS = S::KS, MT = S::MT, NB = S::NB, NA = S::NA, NI = S::NI,
                  NT = S::NT;
    __shared__ double sh[WPB * NPART];
    __shared__ f4 As[NT * 16];          // operands of the block's class, [i][lane]
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, kk = lane >> 4;
    const f4* A4 = (const f4*)A;
    float alpha = 0.0f, beta = 0.0f;
    if (ITER) {
        alpha = (float)ab[0];
        beta = (float)ab[1];
    }
    const TilePos tp = tile_pos<WPB>(wave, E, G, gmul);
    const int a = tp.a;
    const int32_t e = (tp.active ? (int32_t)tp.tile * 16 : 0) + col;
    const bool vcol = tp.active && e < E;
    // class and face neighbours of the lane's element (zeros when absent)
    const Rsrc rn = make_rsrc(nbr, 16u * (uint32_t)E);
    const Rsrc rc = make_rsrc(cls, 4u * (uint32_t)E);
    typedef int i4 __attribute__((ext_vector_type(4)));
    const i4 nb = __builtin_bit_cast(i4, __builtin_amdgcn_raw_buffer_load_b128(rn, (int)(vcol ? 16u * e : OOB), 0, 0));
    const int cl = (int)__builtin_amdgcn_raw_buffer_load_b32(rc, (int)(vcol ? 4u * e : OOB), 0, 0);
    // byte offsets of the lane's slice in the five panel rows (own row, then
    // the neighbours across local faces 0..3); OOB where there is no row
    const int32_t rows[5] = {vcol ? e : -1, vcol ? nb.x : -1, vcol ? nb.y : -1, vcol ? nb.z : -1, vcol ? nb.w : -1};
    uint32_t off[5], offr[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const uint32_t base = ((uint32_t)rows[k] * (uint32_t)G + (uint32_t)a) * (uint32_t)(4 * N);
        off[k] = rows[k] >= 0 ? base + 4u * (uint32_t)(W * kk) : OOB;
        offr[k] = (REM > 0 && rows[k] >= 0 && kk < REM) ? base + 4u * (uint32_t)(4 * W + kk) : OOB;
    }
    const int c = vcol ? cl : -1;
    // class of the block: that of its first element, whose operands the four
    // wavefronts share through LDS (copied once per block)
    const uint32_t tile_b = (uint32_t)(((uint64_t)(tp.lblock * WPB) * gmul) >> 32);
    const int cb = tile_b * 16 < (uint32_t)E ? cls[tile_b * 16] : 0;
    // gather: every load of the wavefront (rows, own x, then the block's
    // share of the operand copy) is in flight before the first use
    const Rsrc rr_in = make_rsrc(r_in, vbytes);
    float rv[5][KS], pv[5][KS], qv[5][KS], xo[KS];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        bload<W>(rr_in, off[k], rv[k]);
        if (REM > 0) bload<1>(rr_in, offr[k], &rv[k][W]);
    }
    if (ITER) {
        const Rsrc rp_in = make_rsrc(p_in, vbytes), rq_in = make_rsrc(q_in, vbytes), rx = make_rsrc(x, vbytes);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            bload<W>(rp_in, off[k], pv[k]);
            bload<W>(rq_in, off[k], qv[k]);
            if (REM > 0) {
                bload<1>(rp_in, offr[k], &pv[k][W]);
                bload<1>(rq_in, offr[k], &qv[k][W]);
            }
        }
        bload<W>(rx, off[0], xo);
        if (REM > 0) bload<1>(rx, offr[0], &xo[W]);
    }
    {
        // straight from global memory into LDS, 64 float4 per wavefront and
        // instruction (the table is a whole number of such pieces)
        const f4* src = A4 + (size_t)cb * NT * 16;
        const int wu = __builtin_amdgcn_readfirstlane(wave);
#pragma unroll
        for (int j = 0; j < (NT * 16 + 64 * WPB - 1) / (64 * WPB); ++j) {
            const int i0 = 64 * WPB * j + 64 * wu;
            if (i0 < NT * 16)
                __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)(src + i0 + lane),
                                                 (__attribute__((address_space(3))) void*)(As + i0), 16, 0, 0);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    float aop[NA];
    ops_load<NA>(As, lane, 0, aop);
    // B operands: the rows themselves, or p_i = (z - alpha w) + beta p
    float bv[5][KS], znew[KS];
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (ITER) {
                const float zk = rv[k][s] - alpha * qv[k][s];
                if (k == 0) znew[s] = zk;
                bv[k][s] = zk + beta * pv[k][s];
            } else {
                bv[k][s] = rv[k][s];
            }
        }
    // q = A p: first pass with the block's class (the whole product for a
    // tile of that class; absent columns hold zeros), then one pass per
    // further class present with the other columns masked
    f4 acc[MT];
#pragma unroll
    for (int i = 0; i < MT; ++i) acc[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < 5; ++k) mfma_block<KS, MT>(aop + k * NB, bv[k], c == cb, acc);
    const uint64_t others = __ballot(vcol && lane < 16 && c != cb);
    for (uint64_t todo = others; todo;) {
        const int cur = __builtin_amdgcn_readlane(c, __builtin_ctzll(todo));
        const bool mine = vcol && c == cur;
        todo &= ~__ballot(mine && lane < 16);
        float ac[NA];
        ops_load<NA>(A4 + (size_t)cur * NT * 16, lane, 0, ac);
#pragma unroll
        for (int k = 0; k < 5; ++k) mfma_block<KS, MT>(ac + k * NB, bv[k], mine, acc);
    }
    // result register j of tile mt is slice position 4 mt + j of the lane
    float accs[KS], o[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        accs[s] = acc[s / 4][s % 4];
        o[s] = cscale * accs[s];
    }
    const Rsrc rq_out = make_rsrc(q_out, vbytes);
    if (!ITER) {
        bstore<W>(rq_out, off[0], o);
        if (REM > 0) bstore<1>(rq_out, offr[0], &o[W]);
        return;
    }
    // w = M^-1 q = B_e^-1 (B p) and r = M z = c B_e z on the own rows
    float wv[KS], rr[KS];
    if (precond) {
        float ainv[NI];
        ops_load<NI>(As, lane, NA, ainv);
        f4 aw[MT], ar[MT];
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            aw[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            ar[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        }
        mfma_block<KS, MT>(ainv, accs, c == cb, aw);
        mfma_block<KS, MT>(aop, znew, c == cb, ar);
        for (uint64_t todo = others; todo;) {
            const int cur = __builtin_amdgcn_readlane(c, __builtin_ctzll(todo));
            const bool mine = vcol && c == cur;
            todo &= ~__ballot(mine && lane < 16);
            float a0[NI], ai[NI];
            ops_load<NI>(A4 + (size_t)cur * NT * 16, lane, 0, a0);
            ops_load<NI>(A4 + (size_t)cur * NT * 16, lane, NA, ai);
            mfma_block<KS, MT>(ai, accs, mine, aw);
            mfma_block<KS, MT>(a0, znew, mine, ar);
        }
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            wv[s] = aw[s / 4][s % 4];
            rr[s] = cscale * ar[s / 4][s % 4];
        }
    } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            wv[s] = o[s];
            rr[s] = znew[s];
        }
    }
    const Rsrc rr_out = make_rsrc(r_out, vbytes), rp_out = make_rsrc(p_out, vbytes), rx = make_rsrc(x, vbytes);
    float xn[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) xn[s] = xo[s] + alpha * pv[0][s];
    bstore<W>(rq_out, off[0], wv);
    bstore<W>(rr_out, off[0], znew);
    bstore<W>(rp_out, off[0], bv[0]);
    bstore<W>(rx, off[0], xn);
    if (REM > 0) {
        bstore<1>(rq_out, offr[0], &wv[W]);
        bstore<1>(rr_out, offr[0], &znew[W]);
        bstore<1>(rp_out, offr[0], &bv[0][W]);
        bstore<1>(rx, offr[0], &xn[W]);
    }
    // partial dot products of the own rows in FP64 (absent rows hold zeros;
    // products of FP32 values may be below the FP32 range)
    double d[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const double pd = bv[0][s], qd = o[s], zd = znew[s], wd = wv[s], rd = rr[s];
        d[0] += pd * qd;
        d[1] += qd * zd;
        d[2] += qd * wd;
        d[3] += rd * zd;
        d[4] += rd * rd;
    }
    const double w4 = wave_total4(d[0], d[1], d[2], d[3]);
    const double w5 = wave_sum(d[4]);
    if (col == 0) sh[NPART * wave + kk] = w4;
    if (lane == 0) sh[NPART * wave + 4] = w5;
    __syncthreads();
    if (threadIdx.x < NPART) {
        const int cc = threadIdx.x;
        double t = 0.0;
#pragma unroll
        for (int wv = 0; wv < WPB; ++wv) t += sh[wv * NPART + cc];
        part_out[PSTRIDE * blockIdx.x + cc] = t;
    }
}

// y = scale B_e^-1 x on every element row (block-Jacobi step)
template <int N>
__global__ void __launch_bounds__(256) k_cg_prec(const float* __restrict__ A, const int32_t* __restrict__ cls,
                                                 const float* x, float* y, float scale, int32_t E, int32_t G,
                                                 uint64_t gmul, uint32_t vbytes) {
    typedef SliceShape<N> S;
    constexpr int W = S::W, REM = S::REM, KS = S::KS, MT = S::MT, NA = S::NA, NI = S::NI, NT = S::NT;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, kk = lane >> 4;
    const TilePos tp = tile_pos<4>(wave, E, G, gmul);
    const int32_t e = (tp.active ? (int32_t)tp.tile * 16 : 0) + col;
    const bool vcol = tp.active && e < E;
    const Rsrc rc = make_rsrc(cls, 4u * (uint32_t)E);
    const int c = vcol ? (int)__builtin_amdgcn_raw_buffer_load_b32(rc, (int)(4u * e), 0, 0) : -1;
    const uint32_t base = ((uint32_t)e * (uint32_t)G + (uint32_t)tp.a) * (uint32_t)(4 * N);
    const uint32_t off = vcol ? base + 4u * (uint32_t)(W * kk) : OOB;
    const uint32_t offr = (REM > 0 && vcol && kk < REM) ? base + 4u * (uint32_t)(4 * W + kk) : OOB;
    const Rsrc rxi = make_rsrc(x, vbytes), ryo = make_rsrc(y, vbytes);
    float v[KS];
    bload<W>(rxi, off, v);
    if (REM > 0) bload<1>(rxi, offr, &v[W]);
    f4 acc[MT];
#pragma unroll
    for (int i = 0; i < MT; ++i) acc[i] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    for (uint64_t todo = __ballot(vcol && lane < 16); todo;) {
        const int cur = __builtin_amdgcn_readlane(c, __builtin_ctzll(todo));
        const bool mine = vcol && c == cur;
        todo &= ~__ballot(mine && lane < 16);
        float ai[NI];
        ops_load<NI>((const f4*)A + (size_t)cur * NT * 16, lane, NA, ai);
        mfma_block<KS, MT>(ai, v, mine, acc);
    }
    float o[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) o[s] = scale * acc[s / 4][s % 4];
    bstore<W>(ryo, off, o);
    if (REM > 0) bstore<1>(ryo, offr, &o[W]);
}

// grid of the per-tile kernel k_cg_op: a multiple of the 8 XCDs
int64_t tile_blocks(const stdg_mesh* m) {
    const int64_t waves = (m->E + 15) / 16 * m->G;
    return ((waves + WPB - 1) / WPB + 7) / 8 * 8;
}

int64_t prec_blocks(const stdg_mesh* m) {
    const int64_t waves = (m->E + 15) / 16 * m->G;
    return ((waves + 3) / 4 + 7) / 8 * 8;
}

uint64_t g_multiplier(const stdg_mesh* m) {
    return ((uint64_t(1) << 32) + (uint64_t)m->G - 1) / (uint64_t)m->G;
}

template <int N, bool ITER>
hipError_t op_n(const stdg_mesh* m, float* x, const float* r_in, const float* p_in, const float* q_in, float* r_out,
                float* p_out, float* q_out, const double* ab, float cscale, int precond, double* part_out,
                hipStream_t s) {
    const uint32_t vbytes = (uint32_t)(4 * m->E * m->G * m->N);
    if (lane_supported(m)) {
        if (ITER) return lane_iter_f32(m, x, r_in, p_in, q_in, r_out, p_out, q_out, ab, cscale, precond, part_out, s);
        return lane_apply_f32(m, r_in, q_out, cscale, s);
    }
    if (elem_supported(m)) {
        if (ITER) return elem_iter_f32(m, x, r_in, p_in, q_in, r_out, p_out, q_out, ab, cscale, precond, part_out, s);
        return elem_apply_f32(m, r_in, q_out, cscale, s);
    }
    hipLaunchKernelGGL((k_cg_op<N, ITER>), dim3((unsigned)tile_blocks(m)), dim3(64 * WPB), 0, s, m->d.aop32, m->d.cls,
                       m->d.nbr, x, r_in, p_in, q_in, r_out, p_out, q_out, ab, cscale, precond, (int32_t)m->E,
                       (int32_t)m->G, g_multiplier(m), vbytes, part_out);
    return hipGetLastError();
}

// Operands of k_cg_op per lane; invs receives the inverse own block of every
// class ([n_classes][N][N], zeros unless every own block is SPD).
template <int N> bool cg_operands(const stdg_mesh* m, std::vector<float>& out, std::vector<double>& invs) {
    typedef SliceShape<N> S;
    constexpr int W = S::W, REM = S::REM, KS = S::KS, MT = S::MT, NB = S::NB, NA = S::NA, NT = S::NT;
    out.assign((size_t)m->n_classes * 64 * NT, 0.0f);
    invs.assign((size_t)m->n_classes * N * N, 0.0);
    bool spd = true;
    for (int c = 0; c < m->n_classes; ++c) {
        // the own block and its inverse (the block must be SPD for CG)
        const double* B0 = m->blocks.data() + (size_t)c * 5 * N * N;
        std::vector<real> chol(B0, B0 + N * N), inv(B0, B0 + N * N);
        bool sym = true;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < i; ++j)
                sym = sym && std::fabs(B0[i * N + j] - B0[j * N + i]) <=
                                 1e-12 * (std::fabs(B0[i * N + i]) + std::fabs(B0[j * N + j]));
        if (!sym || !cholesky(N, chol) || !lu_inverse(N, inv)) spd = false;
        for (int i = 0; i < N * N; ++i) invs[(size_t)c * N * N + i] = (double)inv[i];
        auto entry = [&](int l, int v) -> float& { return out[(((size_t)c * (NT / 4) + v / 4) * 64 + l) * 4 + v % 4]; };
        for (int l = 0; l < 64; ++l) {
            // lane l supplies row l % 16 of each 16 x 4 A tile and contraction
            // index l / 16 of each K step; result row 4 g + j of tile mt lands
            // in register j of lane group g, i.e. slice position 4 mt + j of g
            const int g_out = (l % 16) / 4, j = l % 4, g_in = l / 16;
            for (int mt = 0; mt < MT; ++mt)
                for (int ks = 0; ks < KS; ++ks) {
                    const int so = 4 * mt + j;
                    const int row = so < KS ? slice_dof(W, REM, so, g_out) : -1;
                    const int cin = slice_dof(W, REM, ks, g_in);
                    if (row < 0 || cin < 0) continue;
                    for (int k = 0; k < 5; ++k)
                        entry(l, k * NB + mt * KS + ks) = (float)m->blocks[(((size_t)c * 5 + k) * N + row) * N + cin];
                    entry(l, NA + mt * KS + ks) = spd ? (float)inv[row * N + cin] : 0.0f;
                }
        }
    }
    if (!spd) std::fill(invs.begin(), invs.end(), 0.0);
    return spd;
}

}  // namespace

bool cg_fused_supported(const stdg_mesh* m) {
    return (m->N == 4 || m->N == 10 || m->N == 20) && m->d.aop32 &&
           4 * m->E * m->G * m->N < ((int64_t)1 << 31);
}

int upload_cg_operands(stdg_mesh* m) {
    std::vector<float> t;
    std::vector<double> invs;
    bool spd = false;
    switch (m->N) {
        case 4: spd = cg_operands<4>(m, t, invs); break;
        case 10: spd = cg_operands<10>(m, t, invs); break;
        case 20: spd = cg_operands<20>(m, t, invs); break;
        default: {
            // no tile kernel for this degree: the own-block inverses for the
            // element-per-lane operator tables only
            const int N = m->N;
            invs.assign((size_t)m->n_classes * N * N, 0.0);
            for (int c = 0; c < m->n_classes; ++c) {
                const double* B0 = m->blocks.data() + (size_t)c * 5 * N * N;
                std::vector<real> chol(B0, B0 + N * N), inv(B0, B0 + N * N);
                if (!cholesky(N, chol) || !lu_inverse(N, inv)) { invs.assign(invs.size(), 0.0); break; }
                for (int i = 0; i < N * N; ++i) invs[(size_t)c * N * N + i] = (double)inv[i];
            }
            return upload_lane_operands(m, invs);
        }
    }
    m->d.cg_precond_ok = spd ? 1 : 0;
    STDG_HIP(hipMalloc(&m->d.aop32, t.size() * sizeof(float)));
    STDG_HIP(hipMemcpy(m->d.aop32, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice));
    const int e = upload_lane_operands(m, invs);
    if (e != STDG_OK || lane_supported(m)) return e;
    return upload_elem_operands(m, invs);
}

// workgroups (and partial records) of one CG iteration launch
int64_t cg_op_blocks(const stdg_mesh* m) {
    return lane_supported(m) ? lane_iter_blocks(m) : (elem_supported(m) ? elem_iter_blocks(m) : tile_blocks(m));
}

int64_t cg_partial_len(const stdg_mesh* m) { return PSTRIDE * cg_op_blocks(m); }

hipError_t launch_cg_iter_f32(const stdg_mesh* m, float* x, const float* r_in, const float* p_in, const float* q_in,
                              float* r_out, float* p_out, float* q_out, int iter, float cscale, bool precond,
                              const double* part_in, int64_t n_in, double* part_out, double* ab, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_red, dim3(1), dim3(RED_T), 0, s, part_in, n_in, iter, ab);
    const int pc = precond && m->d.cg_precond_ok ? 1 : 0;
#define STDG_OPN(n) \
    case n: return op_n<n, true>(m, x, r_in, p_in, q_in, r_out, p_out, q_out, ab, cscale, pc, part_out, s);
    switch (m->N) {
        STDG_OPN(4) STDG_OPN(10) STDG_OPN(20)
        default: return hipErrorInvalidValue;
    }
#undef STDG_OPN
}

hipError_t launch_cg_apply_f32(const stdg_mesh* m, const float* x, float* y, float cscale, hipStream_t s) {
#define STDG_OPN(n)                                                                                           \
    case n: return op_n<n, false>(m, nullptr, x, nullptr, nullptr, nullptr, nullptr, y, nullptr, cscale, 0, \
                                  nullptr, s);
    switch (m->N) {
        STDG_OPN(4) STDG_OPN(10) STDG_OPN(20)
        default: return hipErrorInvalidValue;
    }
#undef STDG_OPN
}

hipError_t launch_cg_prec_f32(const stdg_mesh* m, const float* x, float* y, float scale, hipStream_t s) {
    if (lane_supported(m)) return lane_prec_f32(m, x, y, scale, s);
    const uint32_t vbytes = (uint32_t)(4 * m->E * m->G * m->N);
#define STDG_OPN(n)                                                                                            \
    case n:                                                                                                    \
        hipLaunchKernelGGL(k_cg_prec<n>, dim3((unsigned)prec_blocks(m)), dim3(256), 0, s, m->d.aop32, m->d.cls, \
                           x, y, scale, (int32_t)m->E, (int32_t)m->G, g_multiplier(m), vbytes);                 \
        return hipGetLastError();
    switch (m->N) {
        STDG_OPN(4) STDG_OPN(10) STDG_OPN(20)
        default: return hipErrorInvalidValue;
    }
#undef STDG_OPN
}

hipError_t launch_cg_tail_f32(float* x, const float* p, int64_t n, const double* part, int64_t n_part, double* ab,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_cg_red, dim3(1), dim3(RED_T), 0, s, part, n_part, 1, ab);
    hipLaunchKernelGGL(k_cg_tail, dim3(CG_UPD_BLOCKS), dim3(256), 0, s, x, p, n, ab);
    return hipGetLastError();
}

hipError_t launch_cg_check_f32(const double* part, int64_t n_part, double* scal, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_fin_rr, dim3(1), dim3(RED_T), 0, s, part, n_part, scal, slot);
    return hipGetLastError();
}

}  // namespace stdg
