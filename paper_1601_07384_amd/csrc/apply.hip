// Matrix-free pressure Schur operator y = S x (eq. CS_19, negated; Sec. 2.4).
//
// S = dt^2 S^sp (x) C: for element i with neighbours k_f across its local
// faces f,
//   Y_i = sum_{k in {i, k_0..k_3}} B_{c(i),k} (X_k C^T)
// where X_k is the N x G coefficient matrix of element k ([G][N] in memory),
// B_{c,0..4} the class-deduplicated dt^2-scaled spatial blocks and C the G x G
// time factor.
//
// Work decomposition: one thread per (element, time node a).  The thread
// forms the time-mixed neighbour column x'_m = sum_b C_ab x_k[b][m] on the fly
// and accumulates its N outputs y_i[a][.] in registers.  Elements are ordered
// so that every full wavefront holds 64 elements of one class (Hilbert order
// within each class): the wavefront's block B_{c,k} is then uniform and is
// read through scalar loads (one broadcast per column, stored transposed
// BT[c][k][m][r] so a column is contiguous), and the FP64 FMAs take it as a
// scalar operand.  Wavefronts that mix classes (the tail, or meshes without
// repeated geometry) take the same loop with per-lane block loads.
#include "internal.hpp"
#include "kernels.hpp"

namespace stdg {

template <int N, int G, typename T>
__device__ __forceinline__ void accumulate_block(const T* __restrict__ Bk, const T* __restrict__ xt,
                                                 const T (&Ca)[G], T (&acc)[N]) {
#pragma unroll
    for (int m = 0; m < N; ++m) {
        T xp = T(0);
#pragma unroll
        for (int b = 0; b < G; ++b) xp += Ca[b] * xt[b * N + m];
        const T* col = Bk + m * N;
#pragma unroll
        for (int r = 0; r < N; ++r) acc[r] += col[r] * xp;
    }
}

template <int N, int G, typename T>
__global__ void __launch_bounds__(256) schur_apply_tn(
    const T* __restrict__ BT, const int32_t* __restrict__ cls, const int32_t* __restrict__ nbr,
    const T* __restrict__ C, const T* __restrict__ x, T* __restrict__ y, int64_t E) {
    const int a = (int)(blockIdx.x % G);
    const int64_t i = (int64_t)(blockIdx.x / G) * 256 + threadIdx.x;
    const bool valid = i < E;
    const int64_t ii = valid ? i : E - 1;          // inactive lanes mirror a valid element
    const int c = cls[ii];
    const int c0 = __builtin_amdgcn_readfirstlane(c);
    const bool uniform = __all(c == c0);
    T Ca[G];
#pragma unroll
    for (int b = 0; b < G; ++b) Ca[b] = C[a * G + b];
    T acc[N];
#pragma unroll
    for (int r = 0; r < N; ++r) acc[r] = T(0);
    int nb[5];
    nb[0] = (int)ii;
#pragma unroll
    for (int f = 0; f < 4; ++f) nb[f + 1] = nbr[4 * ii + f];
    if (uniform) {
        const T* Bc = BT + (int64_t)c0 * 5 * N * N;
        for (int k = 0; k < 5; ++k) {
            const int t = nb[k];
            // a uniform class has the same boundary faces on every lane
            if (__builtin_amdgcn_readfirstlane(t) < 0) continue;
            accumulate_block<N, G, T>(Bc + k * N * N, x + (int64_t)t * G * N, Ca, acc);
        }
    } else {
        const T* Bc = BT + (int64_t)c * 5 * N * N;
        for (int k = 0; k < 5; ++k) {
            const int t = nb[k];
            if (t < 0) continue;
            accumulate_block<N, G, T>(Bc + k * N * N, x + (int64_t)t * G * N, Ca, acc);
        }
    }
    if (valid) {
        T* yi = y + (i * G + a) * N;
#pragma unroll
        for (int r = 0; r < N; ++r) yi[r] = acc[r];
    }
}

// Copy the 64 time-mixed rows x'[lane'] = sum_b C_ab x[nb(lane')][b][.] of a
// wavefront into its panel: 64/N rows per instruction group, consecutive
// lanes on consecutive spatial values, G loads per value.
template <int N, int G, int RS, typename T>
__device__ __forceinline__ void load_panel(T* __restrict__ panel, const T* __restrict__ x, int t,
                                           const T (&Ca)[G], int roff, int col0) {
    constexpr int RPI = 64 / N;
#pragma unroll
    for (int j0 = 0; j0 < 64; j0 += RPI) {
        const int row = j0 + roff;
        const int tr = __shfl(t, row < 64 ? row : 63, 64);
        if (roff < RPI && row < 64) {
            T v = T(0);
            if (tr >= 0) {
                const T* xt = x + (int64_t)tr * G * N + col0;
#pragma unroll
                for (int b = 0; b < G; ++b) v += Ca[b] * xt[b * N];
            }
            panel[row * RS + col0] = v;
        }
    }
}

template <int N, typename T>
__device__ __forceinline__ void panel_fma(const T* __restrict__ Bk, const T* __restrict__ xr,
                                          T (&acc)[N]) {
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const T xp = xr[m];
        const T* col = Bk + m * N;
#pragma unroll
        for (int r = 0; r < N; ++r) acc[r] += col[r] * xp;
    }
}

// Panel-staged kernel.  A block of 256 threads holds four wavefronts; each
// wavefront owns 64 elements, one time node a and a private LDS panel.  For
// each of the five couplings k the wavefront first copies the 64 time-mixed
// neighbour rows into its panel (a few cache lines per load instruction
// instead of one line per lane), then every lane runs the N x N block against
// its own row: panel values from LDS (odd row stride), block columns from
// scalar registers when the wavefront holds one class.  Boundary faces load
// zero rows instead of being skipped, so every wavefront reaches every barrier.
template <int N, int G, typename T>
__global__ void __launch_bounds__(256) schur_apply_lds(
    const T* __restrict__ BT, const int32_t* __restrict__ cls, const int32_t* __restrict__ nbr,
    const T* __restrict__ C, const T* __restrict__ x, T* __restrict__ y, int64_t E) {
    static_assert(N <= 64, "panel rows longer than a wavefront");
    constexpr int RS = N | 1;                     // odd row stride (elements)
    __shared__ T panels[4 * 64 * RS];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    T* panel = panels + wave * 64 * RS;
    const int a = (int)(blockIdx.x % G);
    const int64_t i = (int64_t)(blockIdx.x / G) * 256 + threadIdx.x;
    const bool valid = i < E;
    const int64_t ii = valid ? i : E - 1;
    const int c = cls[ii];
    const int c0 = __builtin_amdgcn_readfirstlane(c);
    const bool uniform = __all(c == c0);
    T Ca[G];
#pragma unroll
    for (int b = 0; b < G; ++b) Ca[b] = C[a * G + b];
    T acc[N];
#pragma unroll
    for (int r = 0; r < N; ++r) acc[r] = T(0);
    int nb[5];
    nb[0] = (int)ii;
#pragma unroll
    for (int f = 0; f < 4; ++f) nb[f + 1] = nbr[4 * ii + f];
    const int roff = lane / N;                    // this lane's row within a copy group
    const int col0 = lane - roff * N;
    const T* xr = panel + lane * RS;
    if (uniform) {
        // one class for the whole wavefront: block columns through scalar loads
        const T* Bc = BT + (int64_t)c0 * 5 * N * N;
        for (int k = 0; k < 5; ++k) {
            load_panel<N, G, RS, T>(panel, x, nb[k], Ca, roff, col0);
            __syncthreads();
            panel_fma<N, T>(Bc + k * N * N, xr, acc);
            __syncthreads();
        }
    } else {
        const T* Bc = BT + (int64_t)c * 5 * N * N;
        for (int k = 0; k < 5; ++k) {
            load_panel<N, G, RS, T>(panel, x, nb[k], Ca, roff, col0);
            __syncthreads();
            panel_fma<N, T>(Bc + k * N * N, xr, acc);
            __syncthreads();
        }
    }
    if (valid) {
        T* yi = y + (i * G + a) * N;
#pragma unroll
        for (int r = 0; r < N; ++r) yi[r] = acc[r];
    }
}

// Any (N, G): one thread per (element, spatial row), all time nodes.
template <int G, typename T>
__global__ void __launch_bounds__(256) schur_apply_rows(
    const T* __restrict__ BT, const int32_t* __restrict__ cls, const int32_t* __restrict__ nbr,
    const T* __restrict__ C, const T* __restrict__ x, T* __restrict__ y, int64_t E, int N) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = gid / N;
    const int n = (int)(gid - i * N);
    if (i >= E) return;
    const T* Bc = BT + (int64_t)cls[i] * 5 * N * N;
    T acc[G];
#pragma unroll
    for (int b = 0; b < G; ++b) acc[b] = T(0);
    for (int k = 0; k < 5; ++k) {
        const int64_t t = (k == 0) ? i : (int64_t)nbr[4 * i + (k - 1)];
        if (t < 0) continue;
        const T* xt = x + t * G * N;
        for (int m = 0; m < N; ++m) {
            const T bv = Bc[((int64_t)k * N + m) * N + n];
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

// The elements of the runs of several classes that the matrix-core kernel
// leaves out: one workgroup of 5 N threads per element, thread (k, r)
// forming row r of coupling k for every time node (the five couplings in
// parallel, summed through LDS), then the G x G time factor.
template <int G>
__global__ void __launch_bounds__(5 * 35) schur_apply_list(
    const double* __restrict__ BT, const int32_t* __restrict__ cls, const int32_t* __restrict__ nbr,
    const double* __restrict__ C, const double* __restrict__ x, double* __restrict__ y,
    const int32_t* __restrict__ elems, int N) {
    __shared__ double part[5 * G * 35];
    const int64_t i = elems[blockIdx.x];
    const int k = threadIdx.x / N, r = threadIdx.x - k * N;
    double acc[G];
#pragma unroll
    for (int b = 0; b < G; ++b) acc[b] = 0.0;
    const int64_t t = (k == 0) ? i : (int64_t)nbr[4 * i + (k - 1)];
    if (t >= 0) {
        const double* Bk = BT + ((int64_t)cls[i] * 5 + k) * N * N;
        const double* xt = x + t * G * N;
        for (int mm = 0; mm < N; ++mm) {
            const double bv = Bk[(int64_t)mm * N + r];
#pragma unroll
            for (int b = 0; b < G; ++b) acc[b] += bv * xt[b * N + mm];
        }
    }
#pragma unroll
    for (int b = 0; b < G; ++b) part[(k * G + b) * N + r] = acc[b];
    __syncthreads();
    if (k == 0) {
        double z[G];
#pragma unroll
        for (int b = 0; b < G; ++b) {
            z[b] = 0.0;
            for (int kk = 0; kk < 5; ++kk) z[b] += part[(kk * G + b) * N + r];
        }
        double* yi = y + i * G * N;
#pragma unroll
        for (int a = 0; a < G; ++a) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < G; ++b) s += C[a * G + b] * z[b];
            yi[a * N + r] = s;
        }
    }
}

// Element-per-lane FP64 apply for meshes whose 64-element runs share a class
// (the structured cubes).  One wavefront (and workgroup) per run, lane l =
// element 64 run + l; for each of the five couplings the wavefront first
// moves the 64 rows it needs ([G][N] doubles each, contiguous in memory)
// into its LDS with 16-byte loads that walk the rows in order (a load
// instruction covers about 64 / (N G / 2) consecutive rows instead of one
// row per lane), then every lane reads its own row back and applies the
// class block, taken column by column through scalar loads (uniform on the
// run), to all G time nodes of its element.  The G x G time factor is
// applied to the result, which leaves through LDS the same way.  Row pieces
// sit in LDS at an odd stride of 16-byte units (NP + 1 for even NP), so the
// 16 lanes of each pass of a 16-byte read hit distinct banks.
template <int N, int G>
__global__ void __launch_bounds__(64) schur_apply_run(const double* __restrict__ BT, const int32_t* __restrict__ cls,
                                                      const int32_t* __restrict__ nbr, const double* __restrict__ C,
                                                      const double* __restrict__ x, double* __restrict__ y,
                                                      int64_t E, uint32_t n_runs) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    constexpr int R = N * G, NP = R / 2, STR = NP % 2 == 0 ? NP + 1 : NP;
    static_assert(R % 2 == 0, "rows of whole 16-byte pieces");
    __shared__ d2 L[64 * STR];
    const int lane = threadIdx.x;
    // consecutive workgroups go round-robin to the 8 XCDs: XCD x takes the
    // contiguous range of runs x * per ..
    const uint32_t nb = gridDim.x;
    const uint32_t run = (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8;
    if (run >= n_runs) return;
    const int64_t e0 = (int64_t)run * 64, e = e0 + lane;
    const bool valid = e < E;
    const int c = __builtin_amdgcn_readfirstlane(cls[e0]);
    int nbk[4] = {-1, -1, -1, -1};
    if (valid) {
#pragma unroll
        for (int f = 0; f < 4; ++f) nbk[f] = nbr[4 * e + f];
    }
    double z[G][N];
#pragma unroll
    for (int b = 0; b < G; ++b)
#pragma unroll
        for (int r = 0; r < N; ++r) z[b][r] = 0.0;
    for (int k = 0; k < 5; ++k) {
        const int src = k == 0 ? (valid ? (int)e : -1) : nbk[k - 1];
        if (__builtin_amdgcn_readfirstlane(__ballot(src >= 0) != 0 ? 1 : 0) == 0) continue;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int pc = i * 64 + lane, row = pc / NP, piece = pc - row * NP;
            const int s = __shfl(src, row, 64);
            const d2 v = s >= 0 ? reinterpret_cast<const d2*>(x + (int64_t)s * R)[piece] : d2{0.0, 0.0};
            L[row * STR + piece] = v;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double xr[R];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const d2 t = L[lane * STR + j];
            xr[2 * j] = t.x;
            xr[2 * j + 1] = t.y;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const double* Bk = BT + ((int64_t)c * 5 + k) * N * N;
#pragma unroll
        for (int m = 0; m < N; ++m) {
            const double* col = Bk + m * N;
#pragma unroll
            for (int r = 0; r < N; ++r) {
                const double a = col[r];
#pragma unroll
                for (int b = 0; b < G; ++b) z[b][r] += a * xr[b * N + m];
            }
        }
    }
    double yr[R];
#pragma unroll
    for (int a = 0; a < G; ++a)
#pragma unroll
        for (int r = 0; r < N; ++r) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < G; ++b) s += C[a * G + b] * z[b][r];
            yr[a * N + r] = s;
        }
#pragma unroll
    for (int j = 0; j < NP; ++j) L[lane * STR + j] = d2{yr[2 * j], yr[2 * j + 1]};
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int pc = i * 64 + lane, row = pc / NP, piece = pc - row * NP;
        if (e0 + row < E) reinterpret_cast<d2*>(y + (e0 + row) * R)[piece] = L[row * STR + piece];
    }
}

// FP64 apply on the FP64 matrix cores, meshes whose 64-element runs share a
// class.  v_mfma_f64_4x4x4f64 runs four independent 4 x 4 x 4 products
// (blocks b = 0..3); lane 16 k + 4 b + i holds A_b[i][k], lane 16 k + 4 b + j
// holds B_b[k][j], and D_b[i][j] lands in lane 16 i + 4 b + j (probed on the
// GPU; the broadcast fields have no effect on this instruction, so the A
// operand is simply the same in the four blocks).  One 256-thread workgroup
// per run: the class's five blocks are staged in LDS, zero-padded to
// NP = 4 ceil(N / 4) rows and columns; wavefront w takes elements
// 16 w .. 16 w + 15 of the run as the 16 columns (element 4 b + j in lanes
// 16 k + 4 b + j), so a lane's column is the same element in the B operand
// and in the result.  Per (block, four-column step ks, four-row group rg) an
// instruction adds B_k[4 rg .. +3][4 ks .. +3] x[4 ks .. +3] to rows
// 4 rg .. +3 of the 16 elements, for each time node: the A value comes from
// LDS (lane 16 k + 4 b + i reads B_k[4 rg + i][4 ks + k]), the B value is
// one double of the neighbour's row (four lanes of a column read 32
// consecutive bytes).  No padding at N = 4, 20; the G x G time factor is
// applied to the G accumulators of a lane, which hold one row of one element
// for every time node.
template <int N, int G, int CW>
__global__ void __launch_bounds__(256 / CW) schur_apply_mfma(const double* __restrict__ BT,
                                                             const int32_t* __restrict__ run_cls,
                                                             const int32_t* __restrict__ nbr,
                                                             const double* __restrict__ C, const double* x,
                                                             double* __restrict__ y, int64_t E, uint32_t n_runs,
                                                             uint32_t xbytes) {
    constexpr int NQ = (N + 3) / 4, NP = 4 * NQ, NT = 256 / CW;
    constexpr uint32_t OOBX = 0x80000000u;
    __shared__ double A[5 * NP * NP];
    const uint32_t run = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    if (run >= n_runs) return;                          // uniform over the workgroup
    const int c = run_cls[run];                         // runs of several classes: schur_apply_list
    if (c < 0) return;
    const int64_t e0 = (int64_t)run * 64;
    // A[k][r][col] = B_k[r][col] = BT[c][k][col][r] (r fastest: contiguous reads)
    for (int t = threadIdx.x; t < 5 * NP * NP; t += NT) {
        const int r = t % NP, col = (t / NP) % NP, k = t / (NP * NP);
        A[(k * NP + r) * NP + col] = (r < N && col < N) ? BT[(((int64_t)c * 5 + k) * N + col) * N + r] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int hi = lane >> 4, lo = lane & 3;            // k (B) / i (D) and i (A) / j
    // column group g of this wavefront: elements 16 (CW w + g) + 4 b + j
    int64_t e[CW];
    bool valid[CW];
    int nb[CW][4];
#pragma unroll
    for (int g = 0; g < CW; ++g) {
        e[g] = e0 + 16 * (CW * w + g) + 4 * ((lane >> 2) & 3) + lo;
        valid[g] = e[g] < E;
#pragma unroll
        for (int f = 0; f < 4; ++f) nb[g][f] = valid[g] ? nbr[4 * e[g] + f] : -1;
    }
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(x), (short)0,
                                                                        (int)xbytes, 0x00020000);
    double acc[NQ][CW][G];
#pragma unroll
    for (int rg = 0; rg < NQ; ++rg)
#pragma unroll
        for (int g = 0; g < CW; ++g)
#pragma unroll
            for (int a = 0; a < G; ++a) acc[rg][g][a] = 0.0;
    auto couple = [&](int k) {
        uint32_t base[CW];
#pragma unroll
        for (int g = 0; g < CW; ++g) {
            const int64_t src = k == 0 ? (valid[g] ? e[g] : -1)
                                       : (k == 1 ? nb[g][0] : (k == 2 ? nb[g][1] : (k == 3 ? nb[g][2] : nb[g][3])));
            base[g] = src >= 0 ? (uint32_t)src * (uint32_t)(G * N * 8) : OOBX;
        }
#pragma unroll
        for (int ks = 0; ks < NQ; ++ks) {
            const int col = 4 * ks + hi;
            double bv[CW][G];
#pragma unroll
            for (int g = 0; g < CW; ++g)
#pragma unroll
                for (int a = 0; a < G; ++a) {
                    const uint32_t off =
                        (base[g] != OOBX && col < N) ? base[g] + (uint32_t)((a * N + col) * 8) : OOBX;
                    bv[g][a] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rx, (int)off, 0, 0));
                }
#pragma unroll
            for (int rg = 0; rg < NQ; ++rg) {
                const double av = A[(k * NP + 4 * rg + lo) * NP + 4 * ks + hi];
#pragma unroll
                for (int g = 0; g < CW; ++g)
#pragma unroll
                    for (int a = 0; a < G; ++a)
                        acc[rg][g][a] = __builtin_amdgcn_mfma_f64_4x4x4f64(av, bv[g][a], acc[rg][g][a], 0, 0, 0);
            }
        }
    };
    // large blocks (p = 4) one coupling at a time, so that the loads of the
    // next coupling are not all held at once
    if constexpr (NQ * G * CW > 16) {
#pragma unroll 1
        for (int k = 0; k < 5; ++k) couple(k);
    } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) couple(k);
    }
    double Cm[G][G];
#pragma unroll
    for (int a = 0; a < G; ++a)
#pragma unroll
        for (int b = 0; b < G; ++b) Cm[a][b] = C[a * G + b];
#pragma unroll
    for (int g = 0; g < CW; ++g)
        if (valid[g])
#pragma unroll
            for (int rg = 0; rg < NQ; ++rg) {
                const int row = 4 * rg + hi;
                if (row < N)
#pragma unroll
                    for (int a = 0; a < G; ++a) {
                        double s = 0.0;
#pragma unroll
                        for (int b = 0; b < G; ++b) s += Cm[a][b] * acc[rg][g][b];
                        y[(e[g] * G + a) * N + row] = s;
                    }
            }
}

template <int N, int G, int CW>
static hipError_t launch_mfma(const stdg_mesh* m, const double* C, const double* x, double* y, hipStream_t s) {
    const uint32_t runs = (uint32_t)((m->E + 63) / 64);
    const uint32_t blocks = (runs + 7) / 8 * 8;
    hipLaunchKernelGGL((schur_apply_mfma<N, G, CW>), dim3(blocks), dim3(256 / CW), 0, s, m->d.blocks,
                       m->d.run_cls, m->d.nbr, C, x, y, m->E, runs, (uint32_t)(8 * m->E * m->G * m->N));
    static_assert(N <= 35, "list kernel: at most 5 x 35 threads per element");
    if (m->d.n_mixed_elems > 0)
        hipLaunchKernelGGL((schur_apply_list<G>), dim3((unsigned)m->d.n_mixed_elems), dim3(5 * N), 0, s, m->d.blocks,
                           m->d.cls, m->d.nbr, C, x, y, m->d.mixed_elems, N);
    return hipGetLastError();
}

template <int N, int G>
static hipError_t launch_run(const stdg_mesh* m, const double* C, const double* x, double* y, hipStream_t s) {
    const uint32_t runs = (uint32_t)((m->E + 63) / 64);
    const uint32_t blocks = (runs + 7) / 8 * 8;
    hipLaunchKernelGGL((schur_apply_run<N, G>), dim3(blocks), dim3(64), 0, s, m->d.blocks, m->d.cls, m->d.nbr, C,
                       x, y, m->E, runs);
    return hipGetLastError();
}

template <int N, int G, typename T>
static hipError_t launch_tn(const stdg_mesh* m, const T* BT, const T* C, const T* x, T* y, hipStream_t s) {
    const int64_t blocks = (m->E + 255) / 256 * G;
    hipLaunchKernelGGL((schur_apply_tn<N, G, T>), dim3((unsigned)blocks), dim3(256), 0, s, BT,
                       m->d.cls, m->d.nbr, C, x, y, m->E);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_rows(const stdg_mesh* m, const T* BT, const T* C, const T* x, T* y,
                              hipStream_t s) {
    const int64_t work = m->E * m->N;
    const int threads = 256;
    const int64_t blocks = (work + threads - 1) / threads;
    switch (m->G) {
#define STDG_G(g)                                                                              \
    case g:                                                                                    \
        hipLaunchKernelGGL((schur_apply_rows<g, T>), dim3(blocks), dim3(threads), 0, s, BT,   \
                           m->d.cls, m->d.nbr, C, x, y, m->E, m->N);                          \
        break;
        STDG_G(1) STDG_G(2) STDG_G(3) STDG_G(4) STDG_G(5) STDG_G(6) STDG_G(7)
#undef STDG_G
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int N, int G, typename T>
static hipError_t launch_lds(const stdg_mesh* m, const T* BT, const T* C, const T* x, T* y, hipStream_t s) {
    const int64_t blocks = (m->E + 255) / 256 * G;
    hipLaunchKernelGGL((schur_apply_lds<N, G, T>), dim3((unsigned)blocks), dim3(256), 0, s, BT,
                       m->d.cls, m->d.nbr, C, x, y, m->E);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_apply(const stdg_mesh* m, const T* BT, const T* C, const T* x, T* y,
                               hipStream_t s) {
    // Measured on MI355X (FP64): the panel-staged kernel wins for several time
    // nodes with N >= 20 (N=20,G=2: 92 vs 116 us; N=35,G=5: 364 vs 464 us on
    // the 82,944 / 24,576-element meshes), the direct-gather kernel elsewhere
    // and for FP32 everywhere.
    if constexpr (sizeof(T) == 8) {
        // meshes whose elements carry their own blocks: the per-element FP64 tables
        if (elem_apply64_supported(m)) return elem_apply_f64(m, C, x, y, s);
        // measured on MI355X (HIP events, median): 663,552-element p = 3 cube 174 (tn) -> 118 us
        // (two 16-element column groups per wavefront), 82,944-element p = 3, p_gamma = 1 cube
        // 92 (lds) -> 35 us; at p = 2 the MFMA kernel (32 us) only ties the run kernel
        // runs of several classes (Dirichlet meshes: their boundary-class tails) go to the
        // list kernel; the matrix-core kernel is used while they are at most a quarter of
        // the runs (16^3 Dirichlet cube: 12 of 384)
        const int64_t runs = (m->E + 63) / 64;
        if (4 * m->d.n_mixed_runs <= runs && 8 * m->E * m->G * m->N < (int64_t(1) << 31)) {
            if (m->N == 20 && m->G == 1) return launch_mfma<20, 1, 2>(m, C, x, y, s);
            if (m->N == 20 && m->G == 2) return launch_mfma<20, 2, 1>(m, C, x, y, s);
            if (m->N == 35 && m->G == 1) return launch_mfma<35, 1, 2>(m, C, x, y, s);
            if (m->N == 35 && m->G == 2) return launch_mfma<35, 2, 1>(m, C, x, y, s);
            if (m->N == 35 && m->G == 3) return launch_mfma<35, 3, 1>(m, C, x, y, s);
            if (m->N == 35 && m->G == 4) return launch_mfma<35, 4, 1>(m, C, x, y, s);
            if (m->N == 35 && m->G == 5) return launch_mfma<35, 5, 1>(m, C, x, y, s);
        }
        if (m->d.runs_uniform && m->E < (int64_t(1) << 31)) {
#define STDG_NG(n, g) \
    if (m->N == n && m->G == g) return launch_run<n, g>(m, C, x, y, s);
            // measured on MI355X: 196,608-element p = 2, p_gamma = 1 cube 54 -> 32 us
            STDG_NG(4, 1) STDG_NG(4, 2) STDG_NG(10, 1) STDG_NG(10, 2)
#undef STDG_NG
        }
    }
    if (sizeof(T) == 8 && m->G >= 2) {
#define STDG_NG(n, g) \
    if (m->N == n && m->G == g) return launch_lds<n, g, T>(m, BT, C, x, y, s);
        STDG_NG(20, 2) STDG_NG(20, 3) STDG_NG(20, 4) STDG_NG(20, 5)
        STDG_NG(35, 2) STDG_NG(35, 3) STDG_NG(35, 4) STDG_NG(35, 5)
#undef STDG_NG
    }
#define STDG_NG(n, g) \
    if (m->N == n && m->G == g) return launch_tn<n, g, T>(m, BT, C, x, y, s);
    STDG_NG(4, 1) STDG_NG(4, 2) STDG_NG(4, 3) STDG_NG(4, 4) STDG_NG(4, 5)
    STDG_NG(10, 1) STDG_NG(10, 2) STDG_NG(10, 3) STDG_NG(10, 4) STDG_NG(10, 5)
    STDG_NG(20, 1) STDG_NG(20, 2) STDG_NG(20, 3) STDG_NG(20, 4) STDG_NG(20, 5)
    STDG_NG(35, 1) STDG_NG(35, 2) STDG_NG(35, 3) STDG_NG(35, 4) STDG_NG(35, 5)
#undef STDG_NG
    return launch_rows<T>(m, BT, C, x, y, s);
}

hipError_t launch_apply_f64_c(const stdg_mesh* m, const double* C, const double* x, double* y,
                              hipStream_t s) {
    return launch_apply<double>(m, m->d.blocks, C, x, y, s);
}

hipError_t launch_apply_f32_c(const stdg_mesh* m, const float* C, const float* x, float* y, hipStream_t s) {
    return launch_apply<float>(m, m->d.blocks32, C, x, y, s);
}

// y[e][a][n] = sum_b M[a][b] x[e][b][n]  (time mixing)
template <typename T>
__global__ void k_tmix(const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ M, int64_t E,
                       int G, int N) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= E * N) return;
    const int64_t e = t / N;
    const int n = (int)(t - e * N);
    T v[8];
    for (int b = 0; b < G; ++b) v[b] = x[(e * G + b) * N + n];
    for (int a = 0; a < G; ++a) {
        T s = T(0);
        for (int b = 0; b < G; ++b) s += M[a * G + b] * v[b];
        y[(e * G + a) * N + n] = s;
    }
}

hipError_t time_mix_f64(const stdg_mesh* m, const double* M, const double* x, double* y, hipStream_t s) {
    hipLaunchKernelGGL(k_tmix<double>, dim3((unsigned)((m->E * m->N + 255) / 256)), dim3(256), 0, s, x, y, M,
                       m->E, m->G, m->N);
    return hipGetLastError();
}

hipError_t time_mix_f32(const stdg_mesh* m, const float* M, const float* x, float* y, hipStream_t s) {
    hipLaunchKernelGGL(k_tmix<float>, dim3((unsigned)((m->E * m->N + 255) / 256)), dim3(256), 0, s, x, y, M,
                       m->E, m->G, m->N);
    return hipGetLastError();
}

hipError_t launch_apply_f64(const stdg_mesh* m, const double* x, double* y, hipStream_t s) {
    return launch_apply<double>(m, m->d.blocks, m->d.C, x, y, s);
}

hipError_t launch_apply_f32(const stdg_mesh* m, const float* x, float* y, hipStream_t s) {
    return launch_apply<float>(m, m->d.blocks32, m->d.C32, x, y, s);
}

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
