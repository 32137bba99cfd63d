// Per-element FP32 preconditioned CG iteration of the inner pressure solve
// (eq. CS_19) for meshes whose elements carry their own operator blocks:
// unstructured meshes, where almost every element is its own geometry
// class, and curved isoparametric elements (Sec. 2.8).  The recurrences are
// those of k_cg_op in cg_fused.hip (single-reduction block-Jacobi PCG).
//
// There the cost is the blocks themselves: six N x N FP32 matrices per
// element (the five operator blocks and the inverse of the own block,
// 9.6 KB at p = 3) against 4 N bytes per vector row, so an iteration streams
// the blocks once and everything else is small.  A wavefront takes EPW = 64 / L
// consecutive elements with L lanes per element; lane q of an element owns
// its rows q RPL .. q RPL + RPL - 1 (RPL = ceil(N / L)) of every block, which
// it streams with one coalesced 1 KB load per (block, row, four columns) of
// the wavefront, for all G time nodes at once, so each block is read once
// per iteration.  The vectors keep the element-major layout [E][G][N]: each
// lane reads the whole rows it contracts with (its element's and the four
// neighbours', shared by the element's L lanes through the L1 cache), forms
// p_i = (z - alpha w) + beta p for them, and writes its own row slice.  The
// full row of B p that the preconditioner step needs is gathered from the
// element's L lanes by cross-lane reads.  Plain FMAs, no MFMA: the blocks
// differ per lane, there is no shared operand to broadcast.
//
// Block table (host order): entry (((((R 6 + b) RPL + rr) NC4 + c4) 64 + l) 4 + j
// holds row q RPL + rr, column 4 c4 + j of block b of element R EPW + l / L,
// q = l % L (zero past N); b = 0 own block, 1 + f neighbour across local
// face f, 5 inverse of the own block.

#include <algorithm>
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
constexpr int EWPB = 4;                 // wavefronts per workgroup
constexpr int NPART = 5;                // partial sums per workgroup, stored with the stride ...
constexpr int PSTRIDE = 8;              // ... that k_cg_red reads

template <int N> struct ElemShape {
    static constexpr int L = N <= 4 ? 1 : (N <= 10 ? 2 : 4);   // lanes per element
    static constexpr int RPL = (N + L - 1) / L;                // rows per lane
    static constexpr int EPW = 64 / L;                         // elements per wavefront
    static constexpr int NC4 = (N + 3) / 4;                    // four-column groups of a row
    static constexpr int RW = N % 4 == 0 ? 4 : (N % 2 == 0 ? 2 : 1);   // floats per row load
};

__device__ inline Rsrc make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// the N values of the row at byte offset off (OOB: zeros), element-major layout
template <int N> __device__ inline void erow_load(Rsrc r, uint32_t off, float (&v)[N]) {
    constexpr int RW = ElemShape<N>::RW;
#pragma unroll
    for (int i = 0; i < N / RW; ++i) {
        if constexpr (RW == 4) {
            const f4 t = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 16 * i, 0));
            v[4 * i] = t.x; v[4 * i + 1] = t.y; v[4 * i + 2] = t.z; v[4 * i + 3] = t.w;
        } else if constexpr (RW == 2) {
            const f2 t = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 8 * i, 0));
            v[2 * i] = t.x; v[2 * i + 1] = t.y;
        } else {
            v[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 4 * i, 0));
        }
    }
}

// store rows r0 .. r0 + RPL - 1 of v (those below N) at the row's byte offset off
template <int N> __device__ inline void eslice_store(Rsrc r, uint32_t off, int r0, const float (&v)[ElemShape<N>::RPL]) {
#pragma unroll
    for (int i = 0; i < ElemShape<N>::RPL; ++i)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v[i]), r,
                                              (int)(r0 + i < N && off != OOB ? off + 4u * (uint32_t)(r0 + i) : OOB), 0, 0);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// acc[k][a][rr] += rows R0 <= rr < R1 of this lane's slice of a block times
// v[k][a] for the NV vectors and G time nodes (the block's entries are loaded
// first, one coalesced 1 KB load per row and four columns of the wavefront)
template <int N, int G, int NV, int R0, int R1, bool NT>
__device__ __forceinline__ void block_rows(const f4* __restrict__ tb, const float (&v)[NV][G][N],
                                           float (&acc)[NV][G][ElemShape<N>::RPL]) {
    constexpr int NC4 = ElemShape<N>::NC4;
    f4 w[(R1 - R0) * NC4];
#pragma unroll
    for (int i = 0; i < (R1 - R0) * NC4; ++i)
        w[i] = NT ? __builtin_nontemporal_load(tb + 64 * (R0 * NC4 + i)) : tb[64 * (R0 * NC4 + i)];
#pragma unroll
    for (int rr = R0; rr < R1; ++rr)
#pragma unroll
        for (int c4 = 0; c4 < NC4; ++c4) {
            const f4 t = w[(rr - R0) * NC4 + c4];
            const float bv[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = 4 * c4 + j;
                if (c < N)
#pragma unroll
                    for (int k = 0; k < NV; ++k)
#pragma unroll
                        for (int a = 0; a < G; ++a) acc[k][a][rr] = __builtin_fmaf(bv[j], v[k][a][c], acc[k][a][rr]);
            }
        }
}

// the whole slice, CR rows at a time, so that only CR rows of block entries
// are held at once; NT: streamed once (non-temporal loads), else kept in
// the caches for a second pass
template <int N, int G, int NV, int R0 = 0, bool NT = true>
__device__ __forceinline__ void block_slice(const f4* __restrict__ tb, const float (&v)[NV][G][N],
                                            float (&acc)[NV][G][ElemShape<N>::RPL]) {
    constexpr int RPL = ElemShape<N>::RPL, CR = 2;
    constexpr int R1 = R0 + CR < RPL ? R0 + CR : RPL;
    block_rows<N, G, NV, R0, R1, NT>(tb, v, acc);
    if constexpr (R1 < RPL) {
        __builtin_amdgcn_sched_barrier(0);
        block_slice<N, G, NV, R1, NT>(tb, v, acc);
    }
}

// values r0 .. r0 + RPL - 1 of the row at byte offset off (zeros past N)
template <int N> __device__ inline void eslice_load(Rsrc r, uint32_t off, int r0, float (&v)[ElemShape<N>::RPL]) {
#pragma unroll
    for (int i = 0; i < ElemShape<N>::RPL; ++i)
        v[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                             r, (int)(r0 + i < N && off != OOB ? off + 4u * (uint32_t)(r0 + i) : OOB), 0, 0));
}

// One PCG iteration.  Buffers as in k_cg_op: r_in, q_in, p_in hold z, w, p of
// the previous iteration, r_out, q_out, p_out receive z_i, w_i, p_i, x is
// updated in place; ab = (alpha_{i-1}, beta_i) from k_cg_red; five FP64
// partial sums (p.q, q.z, q.w, r.z, r.r) per workgroup.
template <int N, int G>
__global__ void __launch_bounds__(64 * EWPB) k_elem_iter(
    const float* __restrict__ table, const int32_t* __restrict__ nbr, float* x, const float* r_in,
    const float* p_in, const float* q_in, float* r_out, float* p_out, float* q_out, const double* __restrict__ ab,
    float cscale, int precond, int32_t E, uint32_t n_waves, uint32_t vbytes, double* __restrict__ part_out) {
    typedef ElemShape<N> S;
    constexpr int L = S::L, RPL = S::RPL, EPW = S::EPW, NC4 = S::NC4;
    constexpr uint32_t ROWB = 4u * N;                    // bytes of one row
    constexpr size_t BSZ = (size_t)RPL * NC4 * 64;       // f4 entries of one block of a wavefront
    __shared__ double sh[EWPB * NPART];
    // consecutive workgroups go round-robin to the 8 XCDs; XCD x takes the
    // contiguous range of wavefronts x * per .., so neighbouring elements
    // are read through one L2
    const uint32_t lblock = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    const uint32_t wid = lblock * EWPB + (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, q = lane % L, r0 = q * RPL;
    const int32_t e = (int32_t)(wid * EPW) + lane / L;
    const bool valid = wid < n_waves && e < E;
    double d[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (wid < n_waves) {
        const float alpha = (float)ab[0], beta = (float)ab[1];
        const Rsrc rn = make_rsrc(nbr, 16u * (uint32_t)E);
        const i4v nb =
            __builtin_bit_cast(i4v, __builtin_amdgcn_raw_buffer_load_b128(rn, (int)(valid ? 16u * e : OOB), 0, 0));
        const Rsrc rz = make_rsrc(r_in, vbytes), rw = make_rsrc(q_in, vbytes), rp = make_rsrc(p_in, vbytes);
        const Rsrc rx = make_rsrc(x, vbytes);
        const uint32_t own = valid ? (uint32_t)e * G * ROWB : OOB;
        const f4* tb = (const f4*)table + (size_t)wid * 6 * BSZ + lane;
        // own rows: z_i = z - alpha w, p_i = z_i + beta p; x += alpha p on the slice
        float v1[1][G][N];                               // p_i of the own rows, then of a neighbour
        float zs[G][RPL], ps[G][RPL];
#pragma unroll
        for (int a = 0; a < G; ++a) {
            float zo[N], wo[N], po[N], xs[RPL], zl[RPL], wl[RPL], pl[RPL];
            const uint32_t ro = own == OOB ? OOB : own + a * ROWB;
            erow_load<N>(rz, ro, zo);
            erow_load<N>(rw, ro, wo);
            erow_load<N>(rp, ro, po);
            // the lane's own slice again (from the cache): no lane-dependent
            // register indexing
            eslice_load<N>(rz, ro, r0, zl);
            eslice_load<N>(rw, ro, r0, wl);
            eslice_load<N>(rp, ro, r0, pl);
            eslice_load<N>(rx, ro, r0, xs);
#pragma unroll
            for (int r = 0; r < N; ++r) v1[0][a][r] = (zo[r] - alpha * wo[r]) + beta * po[r];
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                xs[i] += alpha * pl[i];
                zs[a][i] = zl[i] - alpha * wl[i];
                ps[a][i] = zs[a][i] + beta * pl[i];
            }
            eslice_store<N>(rx, ro, r0, xs);
            __builtin_amdgcn_sched_barrier(0);
        }
        // own block against p_i, then the four neighbour blocks against the
        // neighbours' p_i
        float acc[1][G][RPL];
#pragma unroll
        for (int a = 0; a < G; ++a)
#pragma unroll
            for (int i = 0; i < RPL; ++i) acc[0][a][i] = 0.0f;
        block_slice<N, G, 1, 0, false>(tb, v1, acc);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll 1
        for (int f = 0; f < 4; ++f) {
            const int32_t k = f == 0 ? nb.x : (f == 1 ? nb.y : (f == 2 ? nb.z : nb.w));
            const uint32_t off = (valid && k >= 0) ? (uint32_t)k * G * ROWB : OOB;
#pragma unroll
            for (int a = 0; a < G; ++a) {
                float zv[N], wv[N], pv[N];
                const uint32_t ro = off == OOB ? OOB : off + a * ROWB;
                erow_load<N>(rz, ro, zv);
                erow_load<N>(rw, ro, wv);
                erow_load<N>(rp, ro, pv);
#pragma unroll
                for (int r = 0; r < N; ++r) v1[0][a][r] = (zv[r] - alpha * wv[r]) + beta * pv[r];
                __builtin_amdgcn_sched_barrier(0);
            }
            block_slice<N, G, 1>(tb + (size_t)(1 + f) * BSZ, v1, acc);
            __builtin_amdgcn_sched_barrier(0);
        }
        float qv[G][RPL], rv[G][RPL], wn[1][G][RPL];
#pragma unroll
        for (int a = 0; a < G; ++a)
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                qv[a][i] = cscale * acc[0][a][i];
                rv[a][i] = zs[a][i];
                wn[0][a][i] = precond ? 0.0f : qv[a][i];
            }
        if (precond) {
            // w_i = B_e^-1 (B p_i): the whole row of B p_i from the element's L lanes
            const int base = lane - q;
#pragma unroll
            for (int qq = 0; qq < L; ++qq)
#pragma unroll
                for (int i = 0; i < RPL; ++i)
                    if (qq * RPL + i < N)
#pragma unroll
                        for (int a = 0; a < G; ++a) v1[0][a][qq * RPL + i] = __shfl(acc[0][a][i], base + qq, 64);
            block_slice<N, G, 1>(tb + (size_t)5 * BSZ, v1, wn);
            __builtin_amdgcn_sched_barrier(0);
            // r = M z_i = c B_e z_i for the partial sums: the own block again
            // (from the cache) against z_i of the own rows, formed again from
            // z and w (inputs of this launch, not overwritten by it)
#pragma unroll
            for (int a = 0; a < G; ++a) {
                float zo[N], wo[N];
                const uint32_t ro = own == OOB ? OOB : own + a * ROWB;
                erow_load<N>(rz, ro, zo);
                erow_load<N>(rw, ro, wo);
#pragma unroll
                for (int r = 0; r < N; ++r) v1[0][a][r] = zo[r] - alpha * wo[r];
                __builtin_amdgcn_sched_barrier(0);
            }
            float ar[1][G][RPL];
#pragma unroll
            for (int a = 0; a < G; ++a)
#pragma unroll
                for (int i = 0; i < RPL; ++i) ar[0][a][i] = 0.0f;
            block_slice<N, G, 1, 0, false>(tb, v1, ar);
#pragma unroll
            for (int a = 0; a < G; ++a)
#pragma unroll
                for (int i = 0; i < RPL; ++i) rv[a][i] = cscale * ar[0][a][i];
        }
        const Rsrc rqo = make_rsrc(q_out, vbytes), rro = make_rsrc(r_out, vbytes), rpo = make_rsrc(p_out, vbytes);
#pragma unroll
        for (int a = 0; a < G; ++a) {
            const uint32_t ro = own == OOB ? OOB : own + a * ROWB;
            eslice_store<N>(rqo, ro, r0, wn[0][a]);
            eslice_store<N>(rro, ro, r0, zs[a]);
            eslice_store<N>(rpo, ro, r0, ps[a]);
            if (valid)
#pragma unroll
                for (int i = 0; i < RPL; ++i)
                    if (r0 + i < N) {
                        const double pd = ps[a][i], qd = qv[a][i], zd = zs[a][i], wd = wn[0][a][i], rd = rv[a][i];
                        d[0] += pd * qd;
                        d[1] += qd * zd;
                        d[2] += qd * wd;
                        d[3] += rd * zd;
                        d[4] += rd * rd;
                    }
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
        for (int wv = 0; wv < EWPB; ++wv) t += sh[wv * NPART + threadIdx.x];
        part_out[PSTRIDE * blockIdx.x + threadIdx.x] = t;
    }
}

// y = cscale (B (x) I) x on the same per-element tables (the operator of the
// inner solve's residual and of stdg_pressure_apply_spatial_f32): the own
// and four neighbour blocks against the rows of x, all time nodes per
// wavefront, each lane storing its row slice.
template <int N, int G>
__global__ void __launch_bounds__(64 * EWPB) k_elem_op(const float* __restrict__ table,
                                                       const int32_t* __restrict__ nbr, const float* x, float* y,
                                                       float cscale, int32_t E, uint32_t n_waves, uint32_t vbytes) {
    typedef ElemShape<N> S;
    constexpr int L = S::L, RPL = S::RPL, EPW = S::EPW, NC4 = S::NC4;
    constexpr uint32_t ROWB = 4u * N;
    constexpr size_t BSZ = (size_t)RPL * NC4 * 64;
    const uint32_t lblock = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    const uint32_t wid = lblock * EWPB + (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wid >= n_waves) return;
    const int lane = threadIdx.x & 63, q = lane % L, r0 = q * RPL;
    const int32_t e = (int32_t)(wid * EPW) + lane / L;
    const bool valid = e < E;
    const Rsrc rn = make_rsrc(nbr, 16u * (uint32_t)E);
    const i4v nb =
        __builtin_bit_cast(i4v, __builtin_amdgcn_raw_buffer_load_b128(rn, (int)(valid ? 16u * e : OOB), 0, 0));
    const Rsrc rx = make_rsrc(x, vbytes);
    const f4* tb = (const f4*)table + (size_t)wid * 6 * BSZ + lane;
    float acc[1][G][RPL];
#pragma unroll
    for (int a = 0; a < G; ++a)
#pragma unroll
        for (int i = 0; i < RPL; ++i) acc[0][a][i] = 0.0f;
#pragma unroll 1
    for (int k = 0; k < 5; ++k) {
        const int32_t src = k == 0 ? (valid ? e : -1) : (k == 1 ? nb.x : (k == 2 ? nb.y : (k == 3 ? nb.z : nb.w)));
        const uint32_t off = src >= 0 ? (uint32_t)src * G * ROWB : OOB;
        float v1[1][G][N];
#pragma unroll
        for (int a = 0; a < G; ++a) erow_load<N>(rx, off == OOB ? OOB : off + a * ROWB, v1[0][a]);
        __builtin_amdgcn_sched_barrier(0);
        block_slice<N, G, 1>(tb + (size_t)k * BSZ, v1, acc);
        __builtin_amdgcn_sched_barrier(0);
    }
    const Rsrc ry = make_rsrc(y, vbytes);
    const uint32_t own = valid ? (uint32_t)e * G * ROWB : OOB;
#pragma unroll
    for (int a = 0; a < G; ++a) {
        float o[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) o[i] = cscale * acc[0][a][i];
        eslice_store<N>(ry, own == OOB ? OOB : own + a * ROWB, r0, o);
    }
}

// y = S x in FP64 on per-element FP64 tables (the five operator blocks,
// rows interleaved over the lanes like the FP32 table, two columns per
// 16-byte load): lane q of an element forms rows q RPL .. of the five
// products for every time node, then applies the G x G time factor C.
// Table entry ((((R 5 + b) RPL + rr) NC2 + c2) 64 + l) 2 + j holds row
// q RPL + rr, column 2 c2 + j of block b of element R EPW + l / L.
template <int N, int G>
__global__ void __launch_bounds__(64 * EWPB) k_elem_apply64(const double* __restrict__ table,
                                                            const int32_t* __restrict__ nbr,
                                                            const double* __restrict__ C, const double* x,
                                                            double* __restrict__ y, int32_t E, uint32_t n_waves,
                                                            uint32_t xbytes) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    typedef ElemShape<N> S;
    constexpr int L = S::L, RPL = S::RPL, EPW = S::EPW, NC2 = (N + 1) / 2;
    constexpr uint32_t ROWB = 8u * N;
    constexpr size_t BSZ = (size_t)RPL * NC2 * 64;      // d2 entries of one block of a wavefront
    const uint32_t lblock = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    const uint32_t wid = lblock * EWPB + (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wid >= n_waves) return;
    const int lane = threadIdx.x & 63, q = lane % L, r0 = q * RPL;
    const int32_t e = (int32_t)(wid * EPW) + lane / L;
    const bool valid = e < E;
    const Rsrc rn = make_rsrc(nbr, 16u * (uint32_t)E);
    const i4v nb =
        __builtin_bit_cast(i4v, __builtin_amdgcn_raw_buffer_load_b128(rn, (int)(valid ? 16u * e : OOB), 0, 0));
    const Rsrc rx = make_rsrc(x, xbytes);
    const d2* tb = (const d2*)table + (size_t)wid * 5 * BSZ + lane;
    double acc[G][RPL];
#pragma unroll
    for (int a = 0; a < G; ++a)
#pragma unroll
        for (int i = 0; i < RPL; ++i) acc[a][i] = 0.0;
#pragma unroll 1
    for (int k = 0; k < 5; ++k) {
        const int32_t src = k == 0 ? (valid ? e : -1) : (k == 1 ? nb.x : (k == 2 ? nb.y : (k == 3 ? nb.z : nb.w)));
        const uint32_t off = src >= 0 ? (uint32_t)src * G * ROWB : OOB;
        double v[G][N];
#pragma unroll
        for (int a = 0; a < G; ++a)
#pragma unroll
            for (int c2 = 0; c2 < N / 2; ++c2) {
                const d2 t = __builtin_bit_cast(
                    d2, __builtin_amdgcn_raw_buffer_load_b128(rx, (int)(off == OOB ? OOB : off + a * ROWB + 16u * c2),
                                                              0, 0));
                v[a][2 * c2] = t.x;
                v[a][2 * c2 + 1] = t.y;
            }
        __builtin_amdgcn_sched_barrier(0);
        const d2* tk = tb + (size_t)k * BSZ;
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            d2 w[NC2];
#pragma unroll
            for (int c2 = 0; c2 < NC2; ++c2) w[c2] = __builtin_nontemporal_load(tk + 64 * (rr * NC2 + c2));
#pragma unroll
            for (int c2 = 0; c2 < NC2; ++c2)
#pragma unroll
                for (int a = 0; a < G; ++a) {
                    acc[a][rr] = __builtin_fma(w[c2].x, v[a][2 * c2], acc[a][rr]);
                    acc[a][rr] = __builtin_fma(w[c2].y, v[a][2 * c2 + 1], acc[a][rr]);
                }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (!valid) return;
    double Cm[G][G];
#pragma unroll
    for (int a = 0; a < G; ++a)
#pragma unroll
        for (int b = 0; b < G; ++b) Cm[a][b] = C[a * G + b];
#pragma unroll
    for (int a = 0; a < G; ++a)
#pragma unroll
        for (int i = 0; i < RPL; ++i)
            if (r0 + i < N) {
                double s = 0.0;
#pragma unroll
                for (int b = 0; b < G; ++b) s += Cm[a][b] * acc[b][i];
                y[((int64_t)e * G + a) * N + r0 + i] = s;
            }
}

template <int N> void elem_table64(const stdg_mesh* m, std::vector<double>& out) {
    typedef ElemShape<N> S;
    constexpr int L = S::L, RPL = S::RPL, EPW = S::EPW, NC2 = (N + 1) / 2;
    const int64_t runs = (m->E + EPW - 1) / EPW;
    out.assign((size_t)runs * 5 * RPL * NC2 * 64 * 2, 0.0);
    for (int64_t e = 0; e < m->E; ++e) {
        const int c = m->cls[e];
        const int64_t R = e / EPW;
        const int el = (int)(e % EPW);
        for (int b = 0; b < 5; ++b) {
            const double* M = m->blocks.data() + ((size_t)c * 5 + b) * N * N;
            for (int qq = 0; qq < L; ++qq)
                for (int rr = 0; rr < RPL; ++rr) {
                    const int row = qq * RPL + rr;
                    if (row >= N) continue;
                    for (int col = 0; col < N; ++col)
                        out[(((((size_t)R * 5 + b) * RPL + rr) * NC2 + col / 2) * 64 + el * L + qq) * 2 + col % 2] =
                            M[row * N + col];
                }
        }
    }
}

template <int N> void elem_table(const stdg_mesh* m, const std::vector<double>& inv, std::vector<float>& out) {
    typedef ElemShape<N> S;
    constexpr int L = S::L, RPL = S::RPL, EPW = S::EPW, NC4 = S::NC4;
    const int64_t runs = (m->E + EPW - 1) / EPW;
    out.assign((size_t)runs * 6 * RPL * NC4 * 64 * 4, 0.0f);
    for (int64_t e = 0; e < m->E; ++e) {
        const int c = m->cls[e];
        const int64_t R = e / EPW;
        const int el = (int)(e % EPW);
        for (int b = 0; b < 6; ++b) {
            const double* M = b < 5 ? m->blocks.data() + ((size_t)c * 5 + b) * N * N : inv.data() + (size_t)c * N * N;
            for (int qq = 0; qq < L; ++qq)
                for (int rr = 0; rr < RPL; ++rr) {
                    const int row = qq * RPL + rr;
                    if (row >= N) continue;
                    for (int col = 0; col < N; ++col)
                        out[(((((size_t)R * 6 + b) * RPL + rr) * NC4 + col / 4) * 64 + el * L + qq) * 4 + col % 4] =
                            (float)M[row * N + col];
                }
        }
    }
}

template <int N> int64_t elem_waves(const stdg_mesh* m) {
    return (m->E + ElemShape<N>::EPW - 1) / ElemShape<N>::EPW;
}

int64_t elem_waves_n(const stdg_mesh* m) {
    switch (m->N) {
        case 4: return elem_waves<4>(m);
        case 10: return elem_waves<10>(m);
        default: return elem_waves<20>(m);
    }
}

}  // namespace

bool elem_supported(const stdg_mesh* m) { return m->d.elem_ops != nullptr; }

int64_t elem_iter_blocks(const stdg_mesh* m) {
    return ((elem_waves_n(m) + EWPB - 1) / EWPB + 7) / 8 * 8;
}

// Per-element tables for meshes whose 16-element tiles mix classes on
// average more than twice (every element of an unstructured or curved mesh
// its own class); inv holds the inverse own blocks per class (zeros when
// some own block is not SPD: then the iteration runs unpreconditioned).
int upload_elem_operands(stdg_mesh* m, const std::vector<double>& inv) {
    if (m->N != 4 && m->N != 10 && m->N != 20) return STDG_OK;
    if ((int64_t)m->n_classes * 8 <= m->E) return STDG_OK;
    if (4 * m->E * m->G * m->N >= ((int64_t)1 << 31)) return STDG_OK;
    if (m->G > 5) return STDG_OK;
    std::vector<float> t;
    switch (m->N) {
        case 4: elem_table<4>(m, inv, t); break;
        case 10: elem_table<10>(m, inv, t); break;
        default: elem_table<20>(m, inv, t); break;
    }
    STDG_HIP(hipMalloc(&m->d.elem_ops, t.size() * sizeof(float)));
    STDG_HIP(hipMemcpy(m->d.elem_ops, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice));
    if (8 * m->E * m->G * m->N < ((int64_t)1 << 31) && m->N % 2 == 0) {
        std::vector<double> t64;
        switch (m->N) {
            case 4: elem_table64<4>(m, t64); break;
            case 10: elem_table64<10>(m, t64); break;
            default: elem_table64<20>(m, t64); break;
        }
        STDG_HIP(hipMalloc(&m->d.elem_ops64, t64.size() * sizeof(double)));
        STDG_HIP(hipMemcpy(m->d.elem_ops64, t64.data(), t64.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    return STDG_OK;
}

bool elem_apply64_supported(const stdg_mesh* m) { return m->d.elem_ops64 != nullptr; }

hipError_t elem_apply_f64(const stdg_mesh* m, const double* C, const double* x, double* y, hipStream_t s) {
    const uint32_t xbytes = (uint32_t)(8 * m->E * m->G * m->N);
    const dim3 grid((unsigned)elem_iter_blocks(m)), block(64 * EWPB);
    const uint32_t nw = (uint32_t)elem_waves_n(m);
#define STDG_NG(n, g)                                                                                            \
    if (m->N == n && m->G == g) {                                                                                \
        hipLaunchKernelGGL((k_elem_apply64<n, g>), grid, block, 0, s, m->d.elem_ops64, m->d.nbr, C, x, y,       \
                           (int32_t)m->E, nw, xbytes);                                                           \
        return hipGetLastError();                                                                                \
    }
    STDG_NG(4, 1) STDG_NG(4, 2) STDG_NG(4, 3) STDG_NG(4, 4) STDG_NG(4, 5)
    STDG_NG(10, 1) STDG_NG(10, 2) STDG_NG(10, 3) STDG_NG(10, 4) STDG_NG(10, 5)
    STDG_NG(20, 1) STDG_NG(20, 2) STDG_NG(20, 3) STDG_NG(20, 4) STDG_NG(20, 5)
#undef STDG_NG
    return hipErrorInvalidValue;
}

hipError_t elem_apply_f32(const stdg_mesh* m, const float* x, float* y, float cscale, hipStream_t s) {
    const uint32_t vbytes = (uint32_t)(4 * m->E * m->G * m->N);
    const dim3 grid((unsigned)elem_iter_blocks(m)), block(64 * EWPB);
    const uint32_t nw = (uint32_t)elem_waves_n(m);
#define STDG_NG(n, g)                                                                                           \
    if (m->N == n && m->G == g) {                                                                               \
        hipLaunchKernelGGL((k_elem_op<n, g>), grid, block, 0, s, m->d.elem_ops, m->d.nbr, x, y, cscale,        \
                           (int32_t)m->E, nw, vbytes);                                                          \
        return hipGetLastError();                                                                               \
    }
    STDG_NG(4, 1) STDG_NG(4, 2) STDG_NG(4, 3) STDG_NG(4, 4) STDG_NG(4, 5)
    STDG_NG(10, 1) STDG_NG(10, 2) STDG_NG(10, 3) STDG_NG(10, 4) STDG_NG(10, 5)
    STDG_NG(20, 1) STDG_NG(20, 2) STDG_NG(20, 3) STDG_NG(20, 4) STDG_NG(20, 5)
#undef STDG_NG
    return hipErrorInvalidValue;
}

hipError_t elem_iter_f32(const stdg_mesh* m, float* x, const float* r_in, const float* p_in, const float* q_in,
                         float* r_out, float* p_out, float* q_out, const double* ab, float cscale, int precond,
                         double* part_out, hipStream_t s) {
    const uint32_t vbytes = (uint32_t)(4 * m->E * m->G * m->N);
    const dim3 grid((unsigned)elem_iter_blocks(m)), block(64 * EWPB);
    const uint32_t nw = (uint32_t)elem_waves_n(m);
#define STDG_NG(n, g)                                                                                              \
    if (m->N == n && m->G == g) {                                                                                  \
        hipLaunchKernelGGL((k_elem_iter<n, g>), grid, block, 0, s, m->d.elem_ops, m->d.nbr, x, r_in, p_in, q_in, \
                           r_out, p_out, q_out, ab, cscale, precond, (int32_t)m->E, nw, vbytes, part_out);        \
        return hipGetLastError();                                                                                  \
    }
    STDG_NG(4, 1) STDG_NG(4, 2) STDG_NG(4, 3) STDG_NG(4, 4) STDG_NG(4, 5)
    STDG_NG(10, 1) STDG_NG(10, 2) STDG_NG(10, 3) STDG_NG(10, 4) STDG_NG(10, 5)
    STDG_NG(20, 1) STDG_NG(20, 2) STDG_NG(20, 3) STDG_NG(20, 4) STDG_NG(20, 5)
#undef STDG_NG
    return hipErrorInvalidValue;
}

}  // namespace stdg
