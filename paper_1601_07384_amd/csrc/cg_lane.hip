// Element-per-lane FP32 kernels of the inner pressure solve (eq. CS_19): the
// operator y = c B x (B = dt^2 S^sp on one time node) and the block-Jacobi
// step y = s B_e^-1 x (p = 1, 2, 3, 4), and the one-kernel preconditioned CG
// iteration whose recurrences are documented with k_cg_op in cg_fused.hip
// (p = 1, 2, 3).  They serve meshes whose 64-element runs share one geometry
// class (the operator also takes runs of several classes, one pass each).
//
// One wavefront per (64-element run, time node), lane l = element 64 run + l.
// A lane holds whole rows of its element (the N values, loaded with the
// widest aligned vector loads) and of its four face neighbours, so the CG
// updates, the products and the dot products need no lane exchange and no
// LDS.  The products run on v_mfma_f32_4x4x1f32 (16 independent 4 x 4 x 1
// blocks): block b = lanes 4b .. 4b + 3 takes the B operand of lane 4b + j
// as its column j (element 4b + j) and its A column (4 consecutive rows of
// the class matrix) from the lanes 4a .. 4a + 3 of block a = abid, with the
// broadcast field cbsz = 4 sending that one A column to all 16 blocks.  So
// each instruction adds A[4 rb .. 4 rb + 3][c] * x[c] to result rows
// 4 rb .. 4 rb + 3 of all 64 elements: N / 4 row groups times N contraction
// steps per N x N block, no padding when 4 divides N, and the rows of the
// result land in the lane that owns the element.  Because the A column is
// read from one lane quad only, the class matrices are spread over the 16
// quads of the wavefront: operand t = (block * NQ + rb) * N + c sits in
// register t / 16 of quad t % 16 (lane 4 (t % 16) + i holds row 4 rb + i),
// which keeps the six blocks of a class (five operator blocks and the
// inverse of the own block) in 6 NQ N / 16 registers per lane: 38 at N = 20.
// The table is laid out [class][NV / 4][64 lanes][4] on the host and read
// with one coalesced float4 load per four registers.
//
// Vectors of these kernels use the run layout: value k of element
// e = 64 R + l at time node a sits at
//   (((R G + a) (N / w) + k / w) 64 + l) w + k % w,
// w = 4 when 4 divides N, else 2 when 2 does, else 1 (length
// ceil(E / 64) 64 G N; the slots of the missing elements of a ragged last run
// hold zeros).  A wavefront's own rows are then w-wide loads of 64
// consecutive lanes (256 w contiguous bytes), and so are the rows of a
// neighbour run whose elements sit in the same lanes (the faces inside a
// Kuhn hexahedron); the element-major layout [E][G][N] would spread every
// such load over 64 rows of 4 N bytes.

#include <algorithm>
#include <utility>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

namespace stdg {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef int i4v __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t Rsrc;

constexpr uint32_t OOB = 0x80000000u;   // byte offset past every buffer: loads give 0, stores are dropped
constexpr int LWPB = 4;                 // wavefronts per workgroup
constexpr int NPART = 5;                // partial dot products per workgroup, stored with ...
constexpr int PSTRIDE = 8;              // ... this stride (the layout k_cg_red reads)

template <int N> struct LaneShape {
    static constexpr int NQ = (N + 3) / 4;                       // 4-row groups of a result row
    static constexpr int NOPS = 6 * NQ * N;                      // broadcast operands of the six blocks
    static constexpr int NV = ((NOPS + 15) / 16 + 3) / 4 * 4;    // registers per lane (multiple of 4)
    static constexpr int RW = N % 4 == 0 ? 4 : (N % 2 == 0 ? 2 : 1);   // floats per row load
    static constexpr int NJ = N / RW;                            // loads per row
};

// byte offset of the first load of row (element e, time node a)
template <int N> __device__ inline uint32_t run_off(int32_t e, int a, int32_t G) {
    constexpr int RW = LaneShape<N>::RW, NJ = LaneShape<N>::NJ;
    return ((((uint32_t)e >> 6) * (uint32_t)G + (uint32_t)a) * (uint32_t)(NJ * 64) + ((uint32_t)e & 63u)) *
           (uint32_t)(4 * RW);
}

__device__ inline Rsrc make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// the N values of a row of the run layout at byte offset off (OOB: zeros);
// load j of the row is 256 RW bytes after load j - 1
template <int N> __device__ inline void row_load(Rsrc r, uint32_t off, float (&v)[N]) {
    constexpr int RW = LaneShape<N>::RW;
#pragma unroll
    for (int i = 0; i < N / RW; ++i) {
        if constexpr (RW == 4) {
            const f4 t = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 1024 * i, 0));
            v[4 * i] = t.x; v[4 * i + 1] = t.y; v[4 * i + 2] = t.z; v[4 * i + 3] = t.w;
        } else if constexpr (RW == 2) {
            const f2 t = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 512 * i, 0));
            v[2 * i] = t.x; v[2 * i + 1] = t.y;
        } else {
            v[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 256 * i, 0));
        }
    }
}

template <int N> __device__ inline void row_store(Rsrc r, uint32_t off, const float (&v)[N]) {
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    constexpr int RW = LaneShape<N>::RW;
#pragma unroll
    for (int i = 0; i < N / RW; ++i) {
        if constexpr (RW == 4) {
            __builtin_amdgcn_raw_buffer_store_b128(
                __builtin_bit_cast(u4, f4{v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]}), r, (int)off,
                1024 * i, 0);
        } else if constexpr (RW == 2) {
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, f2{v[2 * i], v[2 * i + 1]}), r, (int)off,
                                                  512 * i, 0);
        } else {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v[i]), r, (int)off, 256 * i, 0);
        }
    }
}

// Step I of block BLK: contraction index c = I / NQ, row group rb = I % NQ,
// operand t = (BLK NQ + rb) N + c held by quad t % 16 in register t / 16;
// the A column of that quad is broadcast to the 16 blocks (cbsz 4, abid).
template <int N, int BLK, int I>
__device__ __forceinline__ void lane_step(const float (&ops)[LaneShape<N>::NV], const float (&b)[N],
                                          f4 (&acc)[LaneShape<N>::NQ]) {
    constexpr int NQ = LaneShape<N>::NQ, c = I / NQ, rb = I % NQ, t = (BLK * NQ + rb) * N + c;
    acc[rb] = __builtin_amdgcn_mfma_f32_4x4x1f32(ops[t >> 4], b[c], acc[rb], 4, t & 15, 0);
}

template <int N, int BLK, int... I>
__device__ __forceinline__ void lane_steps(const float (&ops)[LaneShape<N>::NV], const float (&b)[N],
                                           f4 (&acc)[LaneShape<N>::NQ], std::integer_sequence<int, I...>) {
    (lane_step<N, BLK, I>(ops, b, acc), ...);
}

// acc (rows 4 rb + i of the lane's element) += block BLK of the class times b
template <int N, int BLK>
__device__ __forceinline__ void lane_block(const float (&ops)[LaneShape<N>::NV], const float (&b)[N],
                                           f4 (&acc)[LaneShape<N>::NQ]) {
    lane_steps<N, BLK>(ops, b, acc, std::make_integer_sequence<int, N * LaneShape<N>::NQ>{});
}

template <int N> __device__ inline void acc_zero(f4 (&acc)[LaneShape<N>::NQ]) {
#pragma unroll
    for (int rb = 0; rb < LaneShape<N>::NQ; ++rb) acc[rb] = f4{0.0f, 0.0f, 0.0f, 0.0f};
}

// the first N result rows, times s
template <int N> __device__ inline void acc_rows(const f4 (&acc)[LaneShape<N>::NQ], float s, float (&o)[N]) {
#pragma unroll
    for (int r = 0; r < N; ++r) o[r] = s * acc[r / 4][r % 4];
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Wavefront of this lane: run and time node; consecutive workgroups go
// round-robin to the 8 XCDs (each with its own L2), so XCD x is given the
// contiguous range of wavefronts x * per .. and neighbouring runs are read
// through the same L2.
struct LanePos {
    int32_t e;          // the lane's element
    int a;              // time node
    int32_t e0;         // first element of the run
    bool wact, valid;   // wavefront has a run; lane has an element
};
__device__ inline LanePos lane_pos(int32_t E, int32_t G, uint32_t n_waves) {
    LanePos p;
    const uint32_t lblock = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    const uint32_t wid = lblock * LWPB + (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    p.wact = wid < n_waves;
    const uint32_t run = p.wact ? wid / (uint32_t)G : 0u;
    p.a = p.wact ? (int)(wid - run * (uint32_t)G) : 0;
    p.e0 = (int32_t)(run * 64u);
    p.e = p.e0 + (int32_t)(threadIdx.x & 63);
    p.valid = p.wact && p.e < E;
    return p;
}

template <int N> __device__ inline void load_ops(const float* __restrict__ table, int c, float (&ops)[LaneShape<N>::NV]) {
    constexpr int NV = LaneShape<N>::NV;
    const f4* src = (const f4*)table + (size_t)c * (NV / 4) * 64 + (threadIdx.x & 63);
#pragma unroll
    for (int i = 0; i < NV / 4; ++i) {
        const f4 t = src[64 * i];
        ops[4 * i] = t.x; ops[4 * i + 1] = t.y; ops[4 * i + 2] = t.z; ops[4 * i + 3] = t.w;
    }
}

// ---------------------------------------------------------------- operator
// A run whose lanes hold several classes (the class tails of a mesh with
// boundary classes) takes one pass per class present: the class's operands,
// then the products with the rows of the other classes' lanes read as zeros.
// A run of one class takes a single pass.
// y = cscale B x (cscale = c for p_gamma = 0, 1 for one time node of B (x) I);
// the five rows of a pass are loaded one block ahead of their products
template <int N>
__global__ void __launch_bounds__(64 * LWPB) k_lane_op(const float* __restrict__ table, const int32_t* __restrict__ cls,
                                                       const int32_t* __restrict__ nbr, const float* x, float* y,
                                                       float cscale, int32_t E, int32_t G, uint32_t n_waves,
                                                       uint32_t vbytes) {
    const LanePos lp = lane_pos(E, G, n_waves);
    if (!lp.wact) return;
    const int mc = lp.valid ? cls[lp.e] : -1;
    const Rsrc rn = make_rsrc(nbr, 16u * (uint32_t)E);
    const i4v nb = __builtin_bit_cast(i4v, __builtin_amdgcn_raw_buffer_load_b128(rn, (int)(lp.valid ? 16u * lp.e : OOB), 0, 0));
    const int32_t rows[5] = {lp.e, nb.x, nb.y, nb.z, nb.w};
    const Rsrc rx = make_rsrc(x, vbytes);
    f4 acc[LaneShape<N>::NQ];
    acc_zero<N>(acc);
    float ops[LaneShape<N>::NV];
    for (uint64_t todo = __ballot(lp.valid); todo;) {
        const int c = __builtin_amdgcn_readlane(mc, __builtin_ctzll(todo));
        const bool mine = lp.valid && mc == c;
        todo &= ~__ballot(mine);
        load_ops<N>(table, c, ops);
        uint32_t off[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) off[k] = (mine && rows[k] >= 0) ? run_off<N>(rows[k], lp.a, G) : OOB;
        float v[2][N];
        row_load<N>(rx, off[0], v[0]);
        auto blk = [&](auto kc) {
            constexpr int k = decltype(kc)::value;
            if constexpr (k < 4) row_load<N>(rx, off[k + 1], v[(k + 1) & 1]);
            lane_block<N, k>(ops, v[k & 1], acc);
        };
        blk(std::integral_constant<int, 0>{});
        blk(std::integral_constant<int, 1>{});
        blk(std::integral_constant<int, 2>{});
        blk(std::integral_constant<int, 3>{});
        blk(std::integral_constant<int, 4>{});
    }
    float o[N];
    acc_rows<N>(acc, cscale, o);
    // every lane of the run stores (the slots past the mesh get zeros)
    row_store<N>(make_rsrc(y, vbytes), run_off<N>(lp.e, lp.a, G), o);
}

// y = scale B_e^-1 x (block-Jacobi step)
template <int N>
__global__ void __launch_bounds__(64 * LWPB) k_lane_prec(const float* __restrict__ table,
                                                         const int32_t* __restrict__ cls, const float* x, float* y,
                                                         float scale, int32_t E, int32_t G, uint32_t n_waves,
                                                         uint32_t vbytes) {
    const LanePos lp = lane_pos(E, G, n_waves);
    if (!lp.wact) return;
    const int mc = lp.valid ? cls[lp.e] : -1;
    const uint32_t off0 = run_off<N>(lp.e, lp.a, G);
    const Rsrc rx = make_rsrc(x, vbytes);
    f4 acc[LaneShape<N>::NQ];
    acc_zero<N>(acc);
    float ops[LaneShape<N>::NV];
    for (uint64_t todo = __ballot(lp.valid); todo;) {
        const int c = __builtin_amdgcn_readlane(mc, __builtin_ctzll(todo));
        const bool mine = lp.valid && mc == c;
        todo &= ~__ballot(mine);
        load_ops<N>(table, c, ops);
        float v[N];
        row_load<N>(rx, mine ? off0 : OOB, v);
        lane_block<N, 5>(ops, v, acc);
    }
    float o[N];
    acc_rows<N>(acc, scale, o);
    row_store<N>(make_rsrc(y, vbytes), off0, o);
}

// ------------------------------------------------------------ CG iteration
// Buffers and scalars as in k_cg_op: r_in/q_in/p_in hold z, w, p of the
// previous iteration, the new ones go to r_out/q_out/p_out, x is updated in
// place; ab = (alpha_{i-1}, beta_i); five FP64 partial sums per workgroup.
template <int N>
__global__ void __launch_bounds__(64 * LWPB) k_lane_iter(
    const float* __restrict__ table, const int32_t* __restrict__ cls, const int32_t* __restrict__ nbr, float* x,
    const float* r_in, const float* p_in, const float* q_in, float* r_out, float* p_out, float* q_out,
    const double* __restrict__ ab, float cscale, int precond, int32_t E, int32_t G, uint32_t n_waves,
    uint32_t vbytes, double* __restrict__ part_out) {
    __shared__ double sh[LWPB * NPART];
    const LanePos lp = lane_pos(E, G, n_waves);
    double d[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (lp.wact) {
        const float alpha = (float)ab[0], beta = (float)ab[1];
        const int c = __builtin_amdgcn_readfirstlane(cls[lp.e0]);
        const Rsrc rn = make_rsrc(nbr, 16u * (uint32_t)E);
        const i4v nb = __builtin_bit_cast(
            i4v, __builtin_amdgcn_raw_buffer_load_b128(rn, (int)(lp.valid ? 16u * lp.e : OOB), 0, 0));
        const int32_t rows[5] = {lp.e, nb.x, nb.y, nb.z, nb.w};
        // loads skip rows that do not exist (zeros); own-row stores reach
        // every slot of the run, so the slots past the mesh keep zeros
        uint32_t off[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) off[k] = (lp.valid && rows[k] >= 0) ? run_off<N>(rows[k], lp.a, G) : OOB;
        const uint32_t sto = run_off<N>(lp.e, lp.a, G);
        const Rsrc rz = make_rsrc(r_in, vbytes), rw = make_rsrc(q_in, vbytes), rp = make_rsrc(p_in, vbytes);
        const Rsrc rx = make_rsrc(x, vbytes);
        // own rows
        float zo[N], wo[N], po[N], xo[N];
        row_load<N>(rz, off[0], zo);
        row_load<N>(rw, off[0], wo);
        row_load<N>(rp, off[0], po);
        row_load<N>(rx, off[0], xo);
        float ops[LaneShape<N>::NV];
        load_ops<N>(table, c, ops);
        // z_i = z - alpha w, p_i = z_i + beta p, x += alpha p
        float zn[N], pn[N];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            zn[r] = zo[r] - alpha * wo[r];
            pn[r] = zn[r] + beta * po[r];
            xo[r] = xo[r] + alpha * po[r];
        }
        row_store<N>(rx, sto, xo);
        f4 acc[LaneShape<N>::NQ];
        acc_zero<N>(acc);
        lane_block<N, 0>(ops, pn, acc);
        // the four neighbour rows of p_i, each formed from its z, w, p
        auto nbr_block = [&](auto kc) {
            constexpr int k = decltype(kc)::value;
            float zv[N], wv[N], pv[N], b[N];
            row_load<N>(rz, off[k], zv);
            row_load<N>(rw, off[k], wv);
            row_load<N>(rp, off[k], pv);
#pragma unroll
            for (int r = 0; r < N; ++r) b[r] = (zv[r] - alpha * wv[r]) + beta * pv[r];
            lane_block<N, k>(ops, b, acc);
        };
        nbr_block(std::integral_constant<int, 1>{});
        nbr_block(std::integral_constant<int, 2>{});
        nbr_block(std::integral_constant<int, 3>{});
        nbr_block(std::integral_constant<int, 4>{});
        float q[N], accs[N];
        acc_rows<N>(acc, 1.0f, accs);
        acc_rows<N>(acc, cscale, q);
        // w = M^-1 q = B_e^-1 (B p) and r = M z = c B_e z on the own rows
        float wn[N], rr[N];
        if (precond) {
            f4 aw[LaneShape<N>::NQ], ar[LaneShape<N>::NQ];
            acc_zero<N>(aw);
            acc_zero<N>(ar);
            lane_block<N, 5>(ops, accs, aw);
            lane_block<N, 0>(ops, zn, ar);
            acc_rows<N>(aw, 1.0f, wn);
            acc_rows<N>(ar, cscale, rr);
        } else {
#pragma unroll
            for (int r = 0; r < N; ++r) {
                wn[r] = q[r];
                rr[r] = zn[r];
            }
        }
        row_store<N>(make_rsrc(q_out, vbytes), sto, wn);
        row_store<N>(make_rsrc(r_out, vbytes), sto, zn);
        row_store<N>(make_rsrc(p_out, vbytes), sto, pn);
        // partial dot products of the own rows in FP64 (absent rows hold
        // zeros; products of FP32 values may be below the FP32 range)
#pragma unroll
        for (int r = 0; r < N; ++r) {
            const double pd = pn[r], qd = q[r], zd = zn[r], wd = wn[r], rd = rr[r];
            d[0] += pd * qd;
            d[1] += qd * zd;
            d[2] += qd * wd;
            d[3] += rd * zd;
            d[4] += rd * rd;
        }
    }
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NPART; ++k) {
        const double t = wave_sum(d[k]);
        if ((threadIdx.x & 63) == 0) sh[NPART * wave + k] = t;
    }
    __syncthreads();
    if (threadIdx.x < NPART) {
        double t = 0.0;
#pragma unroll
        for (int wv = 0; wv < LWPB; ++wv) t += sh[wv * NPART + threadIdx.x];
        part_out[PSTRIDE * blockIdx.x + threadIdx.x] = t;
    }
}

// ------------------------------------------- chunk-staged CG iteration
// The same iteration with the rows of p_i shared through LDS.  One workgroup
// per (chunk of CH = 6 runs = 384 consecutive elements, time node): on the
// class-chunked Kuhn cubes a chunk holds the six tetrahedra of 64 hexahedra,
// so most face neighbours of its elements (82 % on the structured cubes) are
// in the chunk.  Phase 1: wavefront w forms p_i = (z - alpha w) + beta p,
// z_i and x += alpha p for run w of the chunk from coalesced loads, stores x
// and writes p_i to LDS row w 64 + l; the chunk's halo rows (neighbours
// outside it, listed per chunk on the host) are gathered once, updated the
// same way and written to LDS rows CH + h.  Phase 2: the B operands of the
// four neighbour blocks come from LDS through the per-element slot table.
// Each element's p_i is thus formed once per launch (by the wavefront that
// owns it, or once per chunk for a halo row) instead of once per face that
// reads it, and the chunk's rows are gathered while they are still in the
// caches.  LDS rows use the run layout ([row / 64][NJ][64][RW]).
constexpr int CH = 384;               // elements per chunk
constexpr int CHW = CH / 64;          // wavefronts per workgroup

template <int N> __device__ inline uint32_t lds_off(int row, int j) {
    constexpr int RW = LaneShape<N>::RW, NJ = LaneShape<N>::NJ;
    return (uint32_t)((((row >> 6) * NJ + j) * 64 + (row & 63)) * RW);
}

template <int N> __device__ inline void lds_row_put(float* L, int row, const float (&v)[N]) {
    constexpr int RW = LaneShape<N>::RW, NJ = LaneShape<N>::NJ;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        float* d = L + lds_off<N>(row, j);
        if constexpr (RW == 4) *reinterpret_cast<f4*>(d) = f4{v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]};
        else if constexpr (RW == 2) *reinterpret_cast<f2*>(d) = f2{v[2 * j], v[2 * j + 1]};
        else d[0] = v[j];
    }
}

template <int N> __device__ inline void lds_row_get(const float* L, int row, float (&v)[N]) {
    constexpr int RW = LaneShape<N>::RW, NJ = LaneShape<N>::NJ;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const float* d = L + lds_off<N>(row, j);
        if constexpr (RW == 4) {
            const f4 t = *reinterpret_cast<const f4*>(d);
            v[4 * j] = t.x; v[4 * j + 1] = t.y; v[4 * j + 2] = t.z; v[4 * j + 3] = t.w;
        } else if constexpr (RW == 2) {
            const f2 t = *reinterpret_cast<const f2*>(d);
            v[2 * j] = t.x; v[2 * j + 1] = t.y;
        } else {
            v[j] = d[0];
        }
    }
}

template <int N>
__global__ void __launch_bounds__(64 * CHW, 2) k_lane_chunk(
    const float* __restrict__ table, const int32_t* __restrict__ cls, const int16_t* __restrict__ slot,
    const int32_t* __restrict__ halo, int hmax, uint32_t n_chunks, float* x, const float* r_in, const float* p_in,
    const float* q_in, float* r_out, float* p_out, float* q_out, const double* __restrict__ ab, float cscale,
    int precond, int32_t E, int32_t G, uint32_t vbytes, double* __restrict__ part_out) {
    extern __shared__ float rowsL[];
    __shared__ double sh[CHW * NPART];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // consecutive workgroups go round-robin to the 8 XCDs: XCD x takes the
    // contiguous range of (chunk, time node) pairs x * per ..
    const uint32_t lblock = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    const uint32_t chunk = lblock / (uint32_t)G;
    const int a = (int)(lblock - chunk * (uint32_t)G);
    const bool active = chunk < n_chunks;
    const int32_t e0 = (int32_t)(chunk * CH) + 64 * __builtin_amdgcn_readfirstlane(wave);
    const int32_t e = e0 + lane;
    const bool wact = active && e0 < E, valid = wact && e < E;
    const float alpha = active ? (float)ab[0] : 0.0f, beta = active ? (float)ab[1] : 0.0f;
    const Rsrc rz = make_rsrc(r_in, vbytes), rw = make_rsrc(q_in, vbytes), rp = make_rsrc(p_in, vbytes);
    const Rsrc rx = make_rsrc(x, vbytes);
    // ---- phase 1: halo rows, then the run's own rows
    {
        const int h = 64 * wave + lane;
        const int32_t he = (active && h < hmax) ? halo[(size_t)chunk * hmax + h] : -1;
        if (__builtin_amdgcn_readfirstlane((int)(active && 64 * wave < hmax))) {
            const uint32_t ho = he >= 0 ? run_off<N>(he, a, G) : OOB;
            float zv[N], wv[N], pv[N], b[N];
            row_load<N>(rz, ho, zv);
            row_load<N>(rw, ho, wv);
            row_load<N>(rp, ho, pv);
#pragma unroll
            for (int r = 0; r < N; ++r) b[r] = (zv[r] - alpha * wv[r]) + beta * pv[r];
            if (h < hmax) lds_row_put<N>(rowsL, CH + h, b);
        }
    }
    float zn[N], pn[N];
    const uint32_t sto = run_off<N>(e, a, G);
    if (wact) {
        const uint32_t off = valid ? sto : OOB;
        float zo[N], wo[N], po[N], xo[N];
        row_load<N>(rz, off, zo);
        row_load<N>(rw, off, wo);
        row_load<N>(rp, off, po);
        row_load<N>(rx, off, xo);
#pragma unroll
        for (int r = 0; r < N; ++r) {
            zn[r] = zo[r] - alpha * wo[r];
            pn[r] = zn[r] + beta * po[r];
            xo[r] = xo[r] + alpha * po[r];
        }
        row_store<N>(rx, sto, xo);
        lds_row_put<N>(rowsL, 64 * wave + lane, pn);
    }
    typedef short s4 __attribute__((ext_vector_type(4)));
    const s4 sl = valid ? *reinterpret_cast<const s4*>(slot + 4 * (size_t)e) : s4{-1, -1, -1, -1};
    float ops[LaneShape<N>::NV];
    if (wact) load_ops<N>(table, __builtin_amdgcn_readfirstlane(cls[e0]), ops);
    __syncthreads();
    // ---- phase 2: q = A p, w = M^-1 q, r = M z, stores, dots
    double d[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (wact) {
        f4 acc[LaneShape<N>::NQ];
        acc_zero<N>(acc);
        lane_block<N, 0>(ops, pn, acc);
        auto nbr_block = [&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const int row = sl[k - 1];
            float b[N];
            if (row >= 0) {
                lds_row_get<N>(rowsL, row, b);
            } else {
#pragma unroll
                for (int r = 0; r < N; ++r) b[r] = 0.0f;
            }
            lane_block<N, k>(ops, b, acc);
        };
        nbr_block(std::integral_constant<int, 1>{});
        nbr_block(std::integral_constant<int, 2>{});
        nbr_block(std::integral_constant<int, 3>{});
        nbr_block(std::integral_constant<int, 4>{});
        float q[N], accs[N];
        acc_rows<N>(acc, 1.0f, accs);
        acc_rows<N>(acc, cscale, q);
        float wn[N], rr[N];
        if (precond) {
            f4 aw[LaneShape<N>::NQ], ar[LaneShape<N>::NQ];
            acc_zero<N>(aw);
            acc_zero<N>(ar);
            lane_block<N, 5>(ops, accs, aw);
            lane_block<N, 0>(ops, zn, ar);
            acc_rows<N>(aw, 1.0f, wn);
            acc_rows<N>(ar, cscale, rr);
        } else {
#pragma unroll
            for (int r = 0; r < N; ++r) {
                wn[r] = q[r];
                rr[r] = zn[r];
            }
        }
        row_store<N>(make_rsrc(q_out, vbytes), sto, wn);
        row_store<N>(make_rsrc(r_out, vbytes), sto, zn);
        row_store<N>(make_rsrc(p_out, vbytes), sto, pn);
#pragma unroll
        for (int r = 0; r < N; ++r) {
            const double pd = pn[r], qd = q[r], zd = zn[r], wd = wn[r], rd = rr[r];
            d[0] += pd * qd;
            d[1] += qd * zd;
            d[2] += qd * wd;
            d[3] += rd * zd;
            d[4] += rd * rd;
        }
    }
#pragma unroll
    for (int k = 0; k < NPART; ++k) {
        const double t = wave_sum(d[k]);
        if (lane == 0) sh[NPART * wave + k] = t;
    }
    __syncthreads();
    if (threadIdx.x < NPART) {
        double t = 0.0;
#pragma unroll
        for (int wv = 0; wv < CHW; ++wv) t += sh[wv * NPART + threadIdx.x];
        part_out[PSTRIDE * blockIdx.x + threadIdx.x] = t;
    }
}

// ------------------------------------------------------------ layout moves
// y (run layout) = (float)(scale x), x in [E][G][N]; zeros past the mesh
template <int RW>
__global__ void __launch_bounds__(256) k_to_run(const double* __restrict__ x, float* __restrict__ y, double scale,
                                                int64_t E, int G, int N, int64_t n_run) {
    const int NJ = N / RW;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_run; i += (int64_t)gridDim.x * 256) {
        int64_t t = i / RW;
        const int v = (int)(i - t * RW);
        const int l = (int)(t & 63);
        t >>= 6;
        const int j = (int)(t % NJ);
        t /= NJ;
        const int a = (int)(t % G);
        const int64_t e = (t / G) * 64 + l;
        y[i] = e < E ? (float)(scale * x[(e * G + a) * N + j * RW + v]) : 0.0f;
    }
}

// x[e][a][k] (+)= scale sum_b M[a][b] y(e, b, k) (y in the run layout; M the
// G x G identity when null)
template <int RW>
__global__ void __launch_bounds__(256) k_from_run(const float* __restrict__ y, double* __restrict__ x,
                                                  const double* __restrict__ M, double scale, int add, int64_t E,
                                                  int G, int N) {
    const int NJ = N / RW;
    const int64_t n = E * G * N;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int k = (int)(i % N);
        const int64_t ea = i / N;
        const int a = (int)(ea % G);
        const int64_t e = ea / G;
        const int64_t base = (((e >> 6) * G) * NJ + k / RW) * 64 * RW + (e & 63) * RW + k % RW;
        double s = 0.0;
        if (M) {
            for (int b = 0; b < G; ++b) s += M[a * G + b] * (double)y[base + (int64_t)b * NJ * 64 * RW];
        } else {
            s = (double)y[base + (int64_t)a * NJ * 64 * RW];
        }
        x[i] = (add ? x[i] : 0.0) + scale * s;
    }
}

uint32_t lane_waves(const stdg_mesh* m) { return (uint32_t)((m->E + 63) / 64 * m->G); }
int upload_chunk_tables(stdg_mesh* m);

template <int N> void lane_table(const stdg_mesh* m, const std::vector<double>& inv, std::vector<float>& out) {
    typedef LaneShape<N> S;
    constexpr int NQ = S::NQ, NV = S::NV;
    out.assign((size_t)m->n_classes * NV * 64, 0.0f);
    for (int c = 0; c < m->n_classes; ++c)
        for (int l = 0; l < 64; ++l)
            for (int v = 0; v < NV; ++v) {
                const int t = 16 * v + l / 4;          // operand held by quad l / 4 in register v
                if (t >= S::NOPS) continue;
                const int blk = t / (NQ * N), rb = (t / N) % NQ, col = t % N, row = 4 * rb + l % 4;
                if (row >= N) continue;
                const double val = blk < 5 ? m->blocks[(((size_t)c * 5 + blk) * N + row) * N + col]
                                           : inv[((size_t)c * N + row) * N + col];
                out[(((size_t)c * (NV / 4) + v / 4) * 64 + l) * 4 + v % 4] = (float)val;
            }
}

// Slot and halo tables of the chunk-staged iteration: slot[e][f] = LDS row
// of the neighbour across local face f (the chunk's own rows first, then
// its halo rows), -1 where there is none; halo[chunk][h] = element of halo
// row h.  Not built (the per-run kernel serves the mesh) when a chunk's
// halo exceeds one row per thread or the rows exceed 64 KB of LDS.
int upload_chunk_tables(stdg_mesh* m) {
    const int64_t E = m->E, chunks = (E + CH - 1) / CH;
    std::vector<int16_t> slot((size_t)E * 4, -1);
    std::vector<std::vector<int32_t>> halos((size_t)chunks);
    std::vector<int32_t> where((size_t)E, -1);    // halo row of an element within the current chunk
    size_t hmax = 0;
    for (int64_t c = 0; c < chunks; ++c) {
        const int64_t lo = c * CH, hi = std::min<int64_t>(lo + CH, E);
        auto& hl = halos[(size_t)c];
        for (int64_t e = lo; e < hi; ++e)
            for (int f = 0; f < 4; ++f) {
                const int32_t nb = m->nbr[(size_t)e * 4 + f];
                if (nb < 0) continue;
                if (nb >= lo && nb < hi) {
                    slot[(size_t)e * 4 + f] = (int16_t)(nb - lo);
                    continue;
                }
                if (where[(size_t)nb] < 0) {
                    where[(size_t)nb] = (int32_t)hl.size();
                    hl.push_back(nb);
                }
                slot[(size_t)e * 4 + f] = (int16_t)(CH + where[(size_t)nb]);
            }
        for (int32_t g : hl) where[(size_t)g] = -1;
        hmax = std::max(hmax, hl.size());
    }
    hmax = (hmax + 63) / 64 * 64;
    if (hmax > (size_t)CH || (CH + hmax) * (size_t)m->N * sizeof(float) > 65536) return STDG_OK;
    std::vector<int32_t> hflat((size_t)chunks * std::max<size_t>(hmax, 1), -1);
    for (int64_t c = 0; c < chunks; ++c)
        std::copy(halos[(size_t)c].begin(), halos[(size_t)c].end(), hflat.begin() + (size_t)c * hmax);
    STDG_HIP(hipMalloc(&m->d.chunk_slot, slot.size() * sizeof(int16_t)));
    STDG_HIP(hipMemcpy(m->d.chunk_slot, slot.data(), slot.size() * sizeof(int16_t), hipMemcpyHostToDevice));
    STDG_HIP(hipMalloc(&m->d.chunk_halo, hflat.size() * sizeof(int32_t)));
    STDG_HIP(hipMemcpy(m->d.chunk_halo, hflat.data(), hflat.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    m->d.chunk_hmax = (int)hmax;
    m->d.chunk_chunks = chunks;
    return STDG_OK;
}

}  // namespace

bool lane_supported(const stdg_mesh* m) { return m->d.lane_ops != nullptr; }

// Operand table of the element-per-lane kernels, when every 64-element run
// of the mesh holds one class.  inv: [n_classes][N][N] inverse own blocks
// (zeros where the block is not SPD).
int upload_lane_operands(stdg_mesh* m, const std::vector<double>& inv) {
    if (m->N != 4 && m->N != 10 && m->N != 20 && m->N != 35) return STDG_OK;
    // class passes of the runs (one per distinct class in a run)
    int64_t runs = 0, passes = 0;
    for (int64_t t0 = 0; t0 < m->E; t0 += 64, ++runs) {
        std::vector<int32_t> seen;
        for (int64_t e = t0; e < std::min<int64_t>(t0 + 64, m->E); ++e)
            if (std::find(seen.begin(), seen.end(), m->cls[e]) == seen.end()) seen.push_back(m->cls[e]);
        passes += (int64_t)seen.size();
    }
    // p = 1, 2, 3 keep the element-major tile kernels unless every run has
    // one class; p = 4 (no tile kernel) takes the element-per-lane operator
    // while the extra passes stay few
    if (m->N != 35 ? passes != runs : 2 * passes > 3 * runs) return STDG_OK;
    std::vector<float> t;
    switch (m->N) {
        case 4: lane_table<4>(m, inv, t); break;
        case 10: lane_table<10>(m, inv, t); break;
        case 20: lane_table<20>(m, inv, t); break;
        default: lane_table<35>(m, inv, t); break;
    }
    STDG_HIP(hipMalloc(&m->d.lane_ops, t.size() * sizeof(float)));
    STDG_HIP(hipMemcpy(m->d.lane_ops, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice));
    return m->N == 35 ? STDG_OK : upload_chunk_tables(m);
}

// the one-kernel CG iteration runs in the run layout (p = 1, 2, 3)
bool lane_iter_supported(const stdg_mesh* m) { return m->d.lane_ops != nullptr && m->N != 35; }

// workgroups of the per-run kernels (a multiple of the 8 XCDs)
int64_t lane_run_blocks(const stdg_mesh* m) { return ((int64_t)lane_waves(m) + LWPB - 1) / LWPB / 8 * 8 + 8; }

// workgroups (and partial records) of one CG iteration launch
int64_t lane_iter_blocks(const stdg_mesh* m) {
    return m->d.chunk_hmax > 0 ? (m->d.chunk_chunks * m->G + 7) / 8 * 8 : lane_run_blocks(m);
}

hipError_t lane_iter_f32(const stdg_mesh* m, float* x, const float* r_in, const float* p_in, const float* q_in,
                         float* r_out, float* p_out, float* q_out, const double* ab, float cscale, int precond,
                         double* part_out, hipStream_t s) {
    const uint32_t vbytes = (uint32_t)(4 * lane_len(m));
    if (m->d.chunk_hmax > 0) {
        const size_t lds = (size_t)(CH + m->d.chunk_hmax) * m->N * sizeof(float);
#define STDG_N(n)                                                                                                  \
    case n:                                                                                                        \
        hipLaunchKernelGGL(k_lane_chunk<n>, dim3((unsigned)lane_iter_blocks(m)), dim3(64 * CHW), lds, s,            \
                           m->d.lane_ops, m->d.cls, m->d.chunk_slot, m->d.chunk_halo, m->d.chunk_hmax,                   \
                           (uint32_t)m->d.chunk_chunks, x, r_in, p_in, q_in, r_out, p_out, q_out, ab, cscale,        \
                           precond, (int32_t)m->E, (int32_t)m->G, vbytes, part_out);                               \
        return hipGetLastError();
        switch (m->N) {
            STDG_N(4) STDG_N(10) STDG_N(20)
            default: return hipErrorInvalidValue;
        }
#undef STDG_N
    }
    const dim3 grid((unsigned)lane_run_blocks(m)), block(64 * LWPB);
#define STDG_N(n)                                                                                                 \
    case n:                                                                                                       \
        hipLaunchKernelGGL(k_lane_iter<n>, grid, block, 0, s, m->d.lane_ops, m->d.cls, m->d.nbr, x, r_in, p_in,   \
                           q_in, r_out, p_out, q_out, ab, cscale, precond, (int32_t)m->E, (int32_t)m->G,          \
                           lane_waves(m), vbytes, part_out);                                                      \
        return hipGetLastError();
    switch (m->N) {
        STDG_N(4) STDG_N(10) STDG_N(20)
        default: return hipErrorInvalidValue;
    }
#undef STDG_N
}

hipError_t lane_apply_f32(const stdg_mesh* m, const float* x, float* y, float cscale, hipStream_t s) {
    const uint32_t vbytes = (uint32_t)(4 * lane_len(m));
    const dim3 grid((unsigned)lane_run_blocks(m)), block(64 * LWPB);
#define STDG_N(n)                                                                                                  \
    case n:                                                                                                        \
        hipLaunchKernelGGL(k_lane_op<n>, grid, block, 0, s, m->d.lane_ops, m->d.cls, m->d.nbr, x, y, cscale,       \
                           (int32_t)m->E, (int32_t)m->G, lane_waves(m), vbytes);                                   \
        return hipGetLastError();
    switch (m->N) {
        STDG_N(4) STDG_N(10) STDG_N(20) STDG_N(35)
        default: return hipErrorInvalidValue;
    }
#undef STDG_N
}

hipError_t lane_prec_f32(const stdg_mesh* m, const float* x, float* y, float scale, hipStream_t s) {
    const uint32_t vbytes = (uint32_t)(4 * lane_len(m));
    const dim3 grid((unsigned)lane_run_blocks(m)), block(64 * LWPB);
#define STDG_N(n)                                                                                                  \
    case n:                                                                                                        \
        hipLaunchKernelGGL(k_lane_prec<n>, grid, block, 0, s, m->d.lane_ops, m->d.cls, x, y, scale, (int32_t)m->E, \
                           (int32_t)m->G, lane_waves(m), vbytes);                                                  \
        return hipGetLastError();
    switch (m->N) {
        STDG_N(4) STDG_N(10) STDG_N(20) STDG_N(35)
        default: return hipErrorInvalidValue;
    }
#undef STDG_N
}

int64_t lane_len(const stdg_mesh* m) { return (m->E + 63) / 64 * 64 * m->G * m->N; }

hipError_t lane_pack(const stdg_mesh* m, const double* x, double scale, float* y, hipStream_t s) {
    const int rw = m->N % 4 == 0 ? 4 : (m->N % 2 == 0 ? 2 : 1);
    const int64_t n = lane_len(m);
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    if (rw == 4) hipLaunchKernelGGL(k_to_run<4>, dim3(grid), dim3(256), 0, s, x, y, scale, m->E, m->G, m->N, n);
    else if (rw == 2) hipLaunchKernelGGL(k_to_run<2>, dim3(grid), dim3(256), 0, s, x, y, scale, m->E, m->G, m->N, n);
    else hipLaunchKernelGGL(k_to_run<1>, dim3(grid), dim3(256), 0, s, x, y, scale, m->E, m->G, m->N, n);
    return hipGetLastError();
}

hipError_t lane_unpack(const stdg_mesh* m, const float* y, const double* M, double scale, bool add, double* x,
                       hipStream_t s) {
    const int rw = m->N % 4 == 0 ? 4 : (m->N % 2 == 0 ? 2 : 1);
    const int64_t n = m->E * m->G * m->N;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    const int ad = add ? 1 : 0;
    if (rw == 4) hipLaunchKernelGGL(k_from_run<4>, dim3(grid), dim3(256), 0, s, y, x, M, scale, ad, m->E, m->G, m->N);
    else if (rw == 2) hipLaunchKernelGGL(k_from_run<2>, dim3(grid), dim3(256), 0, s, y, x, M, scale, ad, m->E, m->G, m->N);
    else hipLaunchKernelGGL(k_from_run<1>, dim3(grid), dim3(256), 0, s, y, x, M, scale, ad, m->E, m->G, m->N);
    return hipGetLastError();
}

}  // namespace stdg
