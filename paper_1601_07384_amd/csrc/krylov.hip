// Pressure solve (Sec. 2.4 eq. CS_19 / Sec. 2.6 eq. A2_mod): unpreconditioned
// CG for p_gamma = 0 (symmetric positive semi-definite, Corollaries 1-2 of
// Sec. 2.7) and restarted GMRES otherwise (Sec. 3.2), both matrix-free.
//
// The pressure is fixed to zero at the anchor node (every time node).  Instead
// of the anchored matrix (which has one eigenvalue of order one among
// eigenvalues of order dt^2 h, i.e. a badly scaled row), the solver works on
// the equivalent consistent singular system S x = b~, b~ = b except at the
// anchor rows where b~_a = -sum_{i != a} b_i (per time node), which has the
// same solutions up to a constant per time node (the null space of S); the
// result is shifted so that x_a = 0.  The stopping test is the anchored
// relative residual ||b_a - S_a x|| / ||b_a||.
//
// Reductions accumulate in FP64 in a fixed order (per-block partial sums,
// then one block), so results are bitwise reproducible.  Scalars (alpha,
// beta, the Hessenberg matrix and Givens rotations) live on the device; the
// host reads a convergence estimate every `check_every` iterations.
//
// Precision STDG_FP32: FP64 iterative refinement whose inner solves use FP32
// vectors and FP32 operator blocks (FP64 dot products, Hessenberg and Givens);
// the outer residual b~ - S x is recomputed in FP64 each refinement step.
#include <chrono>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include <type_traits>

#include "internal.hpp"
#include "kernels.hpp"

namespace stdg {

namespace {

constexpr int RT = 256;     // threads per reduction block
constexpr int NBLK = 1024;  // reduction blocks (fixed: determinism)

enum Slot {
    S_RR = 0, S_PQ, S_ALPHA, S_BETA, S_RES, S_BN2, S_RN2, S_NORM, S_INV, S_TMP,
    S_FRR = 10,         // fused CG: rr of even / odd iterations (two slots)
    S_CHK = 12,         // fused CG: lagged residual checks (two slots)
    S_TIME = 16,        // G per-time-node sums
    S_ANCH = 32,        // G anchor values
    S_BRHO = 64,        // BiCGStab: rho = (r^, r) and |r|^2 (adjacent), (t.s) and (t.t) (adjacent),
    S_BRR = 65,         //   the previous rho, alpha, omega and sigma = (r^, v)
    S_BTS = 66,
    S_BTT = 67,
    S_BRHOP = 68,
    S_BALPHA = 69,
    S_BOMEGA = 70,
    S_BSIG = 71,
    S_COUNT = 72
};

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sum over the block; result valid in thread 0.  Requires blockDim.x == RT.
__device__ inline double block_sum(double v, double* smem) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) smem[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < RT / 64; ++k) s += smem[k];
    return s;
}

template <typename A, typename B>
__global__ void __launch_bounds__(RT) k_dot(const A* __restrict__ a, const B* __restrict__ b,
                                            int64_t n, double* __restrict__ partial) {
    __shared__ double sm[RT / 64];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT)
        acc += (double)a[i] * (double)b[i];
    double s = block_sum(acc, sm);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out = sum(partial[0..np)); mode selects a scalar update done by thread 0.
enum FinMode { FIN_STORE = 0, FIN_CG_ALPHA = 1, FIN_CG_BETA = 2, FIN_SQRT = 3 };
__global__ void __launch_bounds__(RT) k_finalize(const double* __restrict__ partial, int np,
                                                 double* __restrict__ scal, int slot, int mode) {
    __shared__ double sm[RT / 64];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += RT) acc += partial[i];
    double s = block_sum(acc, sm);
    if (threadIdx.x != 0) return;
    if (mode == FIN_STORE) {
        scal[slot] = s;
    } else if (mode == FIN_CG_ALPHA) {            // s = p.q
        const double rr = scal[S_RR];
        scal[S_PQ] = s;
        scal[S_ALPHA] = (s > 0.0 && rr > 0.0) ? rr / s : 0.0;
    } else if (mode == FIN_CG_BETA) {             // s = r.r (new)
        const double rr = scal[S_RR];
        scal[S_BETA] = (rr > 0.0 && scal[S_ALPHA] != 0.0) ? s / rr : 0.0;
        scal[S_RR] = s;
    } else if (mode == FIN_SQRT) {
        scal[slot] = sqrt(s);
    }
}

// CG: x += alpha p; r -= alpha q; partial sums of r.r
template <typename T>
__global__ void __launch_bounds__(RT) k_cg_xr(T* __restrict__ x, T* __restrict__ r,
                                              const T* __restrict__ p, const T* __restrict__ q,
                                              const double* __restrict__ scal, int64_t n,
                                              double* __restrict__ partial) {
    __shared__ double sm[RT / 64];
    const T alpha = (T)scal[S_ALPHA];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
        x[i] += alpha * p[i];
        const T ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += (double)ri * (double)ri;
    }
    double s = block_sum(acc, sm);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename T>
__global__ void k_cg_p(T* __restrict__ p, const T* __restrict__ r, const double* __restrict__ scal,
                       int64_t n) {
    const T beta = (T)scal[S_BETA];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = r[i] + beta * p[i];
}

// r = b - q (types may differ), partial sums of r.r
template <typename TB, typename TR>
__global__ void __launch_bounds__(RT) k_resid(const TB* __restrict__ b, const TR* __restrict__ q,
                                              TR* __restrict__ r, int64_t n, double* __restrict__ partial) {
    __shared__ double sm[RT / 64];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
        const TR ri = (TR)b[i] - q[i];
        r[i] = ri;
        acc += (double)ri * (double)ri;
    }
    double s = block_sum(acc, sm);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename T>
__global__ void k_fill(T* __restrict__ v, T val, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = val;
}

// x += (double) d
// x += scale d
__global__ void k_add_f32(double* __restrict__ x, const float* __restrict__ d, double scale, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] += scale * (double)d[i];
}

// b = (float)(scale a)
__global__ void k_d2f_scaled(const double* __restrict__ a, float* __restrict__ b, double scale, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)(scale * a[i]);
}

template <typename T>
__global__ void k_copy(const T* __restrict__ a, T* __restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

// Per-time-node sums of a [E][G][N] vector: partial[g * NBLK + block]
__global__ void __launch_bounds__(RT) k_time_sums(const double* __restrict__ v, int64_t E, int G, int N,
                                                  double* __restrict__ partial) {
    __shared__ double sm[RT / 64];
    const int64_t n = E * G * N;
    for (int g = 0; g < G; ++g) {
        double acc = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT)
            if ((int)((i / N) % G) == g) acc += v[i];
        double s = block_sum(acc, sm);
        if (threadIdx.x == 0) partial[(int64_t)g * gridDim.x + blockIdx.x] = s;
    }
}

__global__ void __launch_bounds__(RT) k_fin_multi(const double* __restrict__ partial, int np,
                                                  double* __restrict__ out, double* __restrict__ acc_out,
                                                  double sgn) {
    __shared__ double sm[RT / 64];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += RT) acc += partial[(int64_t)j * np + i];
    double s = block_sum(acc, sm);
    if (threadIdx.x == 0) {
        out[j] = s;
        if (acc_out) acc_out[j] += sgn * s;
    }
}

// b~: anchor rows replaced by minus the sum of all other rows (per time node)
__global__ void k_set_anchor(double* __restrict__ bt, const double* __restrict__ tsum, int64_t anchor,
                             int node, int G, int N) {
    const int g = threadIdx.x;
    if (g < G) {
        const int64_t k = (anchor * G + g) * N + node;
        bt[k] = -(tsum[g] - bt[k]);
    }
}

// subtract the per-time-node mean (projection onto the range of S)
template <typename T>
__global__ void k_remove_mean(T* __restrict__ v, const double* __restrict__ tsum, int64_t E, int G, int N) {
    const int64_t n = E * G * N;
    const double cnt = (double)(E * N);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int g = (int)((i / N) % G);
        v[i] -= (T)(tsum[g] / cnt);
    }
}

__global__ void k_read_anchor(const double* __restrict__ x, double* __restrict__ out, int64_t anchor,
                              int node, int G, int N) {
    const int g = threadIdx.x;
    if (g < G) out[g] = x[(anchor * G + g) * N + node];
}

__global__ void k_shift(double* __restrict__ x, const double* __restrict__ a, int64_t E, int G, int N) {
    const int64_t n = E * G * N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] -= a[(i / N) % G];
}

// anchored residual: sum (b - q)^2 and sum b^2 over non-anchor rows
__global__ void __launch_bounds__(RT) k_anch_res(const double* __restrict__ b, const double* __restrict__ q,
                                                 int64_t anchor, int node, int64_t E, int G, int N,
                                                 double* __restrict__ partial) {
    __shared__ double sm[RT / 64];
    const int64_t n = E * G * N;
    double rr = 0.0, bb = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
        const int64_t e = i / ((int64_t)G * N);
        const int nn = (int)(i % N);
        if (e == anchor && nn == node) continue;
        const double r = b[i] - q[i];
        rr += r * r;
        bb += b[i] * b[i];
    }
    double s1 = block_sum(rr, sm);
    __syncthreads();
    double s2 = block_sum(bb, sm);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = s1;
        partial[gridDim.x + blockIdx.x] = s2;
    }
}

// ---- GMRES pieces ---------------------------------------------------------
// partial[j * NBLK + block] = sum over the block's rows of V_j . w, j < k1
template <typename T>
__global__ void __launch_bounds__(RT) k_multidot(const T* __restrict__ V, int k1, int64_t n,
                                                 const T* __restrict__ w, double* __restrict__ partial) {
    __shared__ double sm[RT / 64];
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    for (int j = 0; j < k1; ++j) {
        const T* vj = V + (int64_t)j * n;
        double acc = 0.0;
        for (int64_t i = lo + threadIdx.x; i < hi; i += RT) acc += (double)vj[i] * (double)w[i];
        double s = block_sum(acc, sm);
        if (threadIdx.x == 0) partial[(int64_t)j * gridDim.x + blockIdx.x] = s;
    }
}

// w += sgn * sum_j h_j V_j
template <typename T>
__global__ void k_multiaxpy(const T* __restrict__ V, int k1, int64_t n, const double* __restrict__ h,
                            double sgn, T* __restrict__ w) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < k1; ++j) s += h[j] * (double)V[(int64_t)j * n + i];
        w[i] = (T)((double)w[i] + sgn * s);
    }
}

// v *= 1/scal[slot]  (skipped when the norm is zero)
template <typename T>
__global__ void k_scale_inv(T* __restrict__ v, const double* __restrict__ src, int64_t n) {
    const double nrm = *src;
    if (!(nrm > 0.0)) return;
    const double inv = 1.0 / nrm;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = (T)((double)v[i] * inv);
}

// Hessenberg column k (H is (m+1) x m column-major: H[j + (m+1) k]):
// apply the previous rotations, form a new one, update g; residual estimate.
__global__ void k_givens(double* __restrict__ H, double* __restrict__ g, double* __restrict__ cs,
                         double* __restrict__ sn, int k, int m, double* __restrict__ scal) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double* h = H + (int64_t)(m + 1) * k;
    for (int i = 0; i < k; ++i) {
        const double t = cs[i] * h[i] + sn[i] * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t;
    }
    const double a = h[k], b = h[k + 1];
    const double r = sqrt(a * a + b * b);
    double c = 1.0, s = 0.0;
    if (r > 0.0) { c = a / r; s = b / r; }
    cs[k] = c; sn[k] = s;
    h[k] = r; h[k + 1] = 0.0;
    g[k + 1] = -s * g[k];
    g[k] = c * g[k];
    scal[S_RES] = fabs(g[k + 1]);
}

// y = R^-1 g for the leading (k1 x k1) triangle
__global__ void k_backsolve(const double* __restrict__ H, const double* __restrict__ g,
                            double* __restrict__ y, int k1, int m) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = k1 - 1; i >= 0; --i) {
        double s = g[i];
        for (int j = i + 1; j < k1; ++j) s -= H[i + (int64_t)(m + 1) * j] * y[j];
        const double d = H[i + (int64_t)(m + 1) * i];
        y[i] = d != 0.0 ? s / d : 0.0;
    }
}

__global__ void k_init_g(double* g, int m, const double* beta) {
    for (int i = threadIdx.x; i <= m; i += blockDim.x) g[i] = (i == 0) ? *beta : 0.0;
}

int grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

struct Ctx {
    const stdg_mesh* m;
    hipStream_t s;
    int64_t n;
    double* partial;
    double* scal;
    double* hscal;
    double* gm;        // GMRES small arrays: H, g, cs, sn, y, h
    int op = 0;        // 0: pressure Schur operator, 1: viscous operator (3 components),
                       // 2: B (x) I, 3: block-Jacobi preconditioned viscous operator D^-1 A
    double* tmp = nullptr;   // op 3: holds A x before D^-1
    bool precond = false;    // block-Jacobi preconditioning of the fused FP32 CG
    int applies = 0;
    double loop_ms = 0.0;    // device time of the one-kernel CG iterations (HIP events)
    int loop_iters = 0;
    bool run_layout = false; // FP32 vectors in the run layout of the element-per-lane kernels (n padded)
};

template <typename T> struct Apply;
// op 0: S = B (x) C; op 1: viscous operator; op 2: B (x) I (the spatial
// pressure operator on every time node, B = dt^2 S^sp).
template <> struct Apply<double> {
    static hipError_t run(const Ctx& c, const double* x, double* y) {
        if (c.op == 0) return launch_apply_f64(c.m, x, y, c.s);
        if (c.op == 2) return launch_apply_f64_c(c.m, c.m->d.Cid, x, y, c.s);
        if (c.op == 3) {
            const hipError_t e = launch_visc_apply(c.m, x, c.tmp, c.s);
            return e != hipSuccess ? e : launch_visc_precond(c.m, c.tmp, y, c.s);
        }
        return launch_visc_apply(c.m, x, y, c.s);
    }
    static hipError_t tmix(const Ctx& c, bool inverse, const double* x, double* y) {
        return time_mix_f64(c.m, inverse ? c.m->d.Cinv : c.m->d.C, x, y, c.s);
    }
};
template <> struct Apply<float> {
    static hipError_t run(const Ctx& c, const float* x, float* y) {
        if (c.run_layout) {
            if (c.op != 0 && c.op != 2) return hipErrorInvalidValue;
            return lane_apply_f32(c.m, x, y, c.op == 2 ? 1.0f : (float)c.m->Ctime[0], c.s);
        }
        if (c.op == 0) return launch_apply_f32(c.m, x, y, c.s);
        if (c.op == 2) return launch_apply_f32_c(c.m, c.m->d.Cid32, x, y, c.s);
        return hipErrorInvalidValue;
    }
    static hipError_t tmix(const Ctx& c, bool inverse, const float* x, float* y) {
        return time_mix_f32(c.m, inverse ? c.m->d.Cinv32 : c.m->d.C32, x, y, c.s);
    }
};

#define CK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { set_error(std::string(#x) + ": " + hipGetErrorString(e_)); return STDG_ERR_DEVICE; } } while (0)

int read_scal(Ctx& c, int slot, double& v) {
    CK(hipMemcpyAsync(c.hscal, c.scal + slot, sizeof(double), hipMemcpyDeviceToHost, c.s));
    CK(hipStreamSynchronize(c.s));
    v = c.hscal[0];
    return STDG_OK;
}

// Per-time-node sums into scal[S_TIME..]
int time_sums(Ctx& c, const double* v) {
    const stdg_mesh* m = c.m;
    hipLaunchKernelGGL(k_time_sums, dim3(NBLK), dim3(RT), 0, c.s, v, m->E, m->G, m->N, c.partial);
    hipLaunchKernelGGL(k_fin_multi, dim3(m->G), dim3(RT), 0, c.s, c.partial, NBLK, c.scal + S_TIME,
                       (double*)nullptr, 0.0);
    CK(hipGetLastError());
    return STDG_OK;
}

// FP32 CG with the one-kernel iteration (operator B (x) I only).
bool cg_fusable(const Ctx& c) {
    const stdg_mesh* m = c.m;
    return (c.op == 2 || (c.op == 0 && m->G == 1)) && cg_fused_supported(m) && m->ws.p32b && m->ws.r32b &&
           m->ws.q32b && 2 * cg_partial_len(m) <= (int64_t)NBLK * 208;
}

int cg_fused(Ctx& c, const float* b, float* x, float* r, float* p, float* q, double tol_abs, int max_it,
             int check_every, int& iters, double& res_out) {
    const stdg_mesh* m = c.m;
    const int64_t n = c.n;
    const int gb = grid_for(n);
    float* rb[2] = {r, m->ws.r32b};
    float* pb[2] = {p, m->ws.p32b};
    float* qb[2] = {q, m->ws.q32b};
    const int64_t nb = cg_op_blocks(m);
    double* part[2] = {c.partial, c.partial + cg_partial_len(m)};
    const bool precond = c.precond && m->d.cg_precond_ok;
    const float cscale = c.op == 2 ? 1.0f : (float)m->Ctime[0];
    // r_0 = b - A x, rr_0 into the even rr slot; p_{-1} = q_{-1} = 0
    CK(Apply<float>::run(c, x, qb[1])); c.applies++;
    hipLaunchKernelGGL((k_resid<float, float>), dim3(NBLK), dim3(RT), 0, c.s, b, qb[1], rb[0], n, c.partial);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, c.s, c.partial, NBLK, c.scal, (int)S_FRR, (int)FIN_STORE);
    // the iteration carries z = M^-1 r and w = M^-1 q (M = c diag(B_e)) in
    // the r and q buffers; p_{-1} = w_{-1} = 0
    if (precond) CK(launch_cg_prec_f32(m, rb[0], rb[0], 1.0f / cscale, c.s));
    hipLaunchKernelGGL(k_fill<float>, dim3(gb), dim3(256), 0, c.s, pb[0], 0.0f, n);
    hipLaunchKernelGGL(k_fill<float>, dim3(gb), dim3(256), 0, c.s, qb[0], 0.0f, n);
    CK(hipGetLastError());
    double rr;
    if (int e = read_scal(c, S_FRR, rr)) return e;
    iters = 0;
    res_out = std::sqrt(rr);
    if (res_out <= tol_abs) return STDG_OK;
    // Residual checks lag one polling interval: the check enqueued after
    // iteration i is read once iteration i + check_every has been enqueued,
    // so the device queue never drains while the host waits.  A solve thus
    // runs up to check_every iterations past the one that met the tolerance.
    hipEvent_t const* ev = m->ws.ev;
    int slot = 0, pending = -1, status = STDG_NOT_CONVERGED;
    auto enqueue_check = [&](int sl) -> int {
        CK(launch_cg_check_f32(part[(iters - 1) & 1], nb, c.scal, (int)S_CHK + sl, c.s));
        CK(hipMemcpyAsync(c.hscal + 2 + sl, c.scal + S_CHK + sl, sizeof(double), hipMemcpyDeviceToHost, c.s));
        CK(hipEventRecord(ev[sl], c.s));
        return STDG_OK;
    };
    auto read_check = [&](int sl, double& v) -> int {
        CK(hipEventSynchronize(ev[sl]));
        v = c.hscal[2 + sl];
        if (!std::isfinite(v)) { set_error("non-finite residual in CG"); return STDG_ERR_NUMERIC; }
        return STDG_OK;
    };
    const hipEvent_t t0ev = m->ws.ev[2], t1ev = m->ws.ev[3];
    CK(hipEventRecord(t0ev, c.s));
    // an iteration with alpha = 0 (p.q not positive: breakdown) changes
    // nothing, so r.r repeating bit for bit between two checks means the
    // iteration has stalled; the solve then stops, not converged
    double last_rr = -1.0;
    bool stalled = false;
    while (iters < max_it && status != STDG_OK && !stalled) {
        const int i = iters, in = i & 1, out = in ^ 1;
        CK(launch_cg_iter_f32(m, x, rb[in], pb[in], qb[in], rb[out], pb[out], qb[out], i, cscale, precond,
                              part[out], nb, part[in], c.scal + S_FRR, c.s));
        c.applies++;
        ++iters;
        if (iters % check_every == 0 || iters == max_it) {
            if (int e = enqueue_check(slot)) return e;
            if (pending >= 0) {
                if (int e = read_check(slot ^ 1, rr)) return e;
                if (std::sqrt(rr) <= tol_abs) status = STDG_OK;
                else if (rr == last_rr) stalled = true;
                last_rr = rr;
            }
            pending = iters;
            slot ^= 1;
        }
    }
    CK(hipEventRecord(t1ev, c.s));
    if (iters == 0) return STDG_NOT_CONVERGED;
    // x += alpha p of the last iteration, then the newest residual
    CK(launch_cg_tail_f32(x, pb[iters & 1], n, part[(iters - 1) & 1], nb, c.scal + S_FRR, c.s));
    {
        float ms = 0.0f;
        CK(hipEventSynchronize(t1ev));
        CK(hipEventElapsedTime(&ms, t0ev, t1ev));
        c.loop_ms += ms;
        c.loop_iters += iters;
    }
    if (pending >= 0) {
        if (int e = read_check(slot ^ 1, rr)) return e;
        res_out = std::sqrt(rr);
        if (res_out <= tol_abs) status = STDG_OK;
    }
    return status;
}

// CG on S x = b (consistent); x, b, work vectors of type T.  Stops when the
// recursive residual norm <= tol_abs or after max_it iterations.
template <typename T>
int cg(Ctx& c, const T* b, T* x, T* r, T* p, T* q, double tol_abs, int max_it, int check_every,
       int& iters, double& res_out) {
    if constexpr (std::is_same<T, float>::value) {
        if (cg_fusable(c)) return cg_fused(c, b, x, r, p, q, tol_abs, max_it, check_every, iters, res_out);
    }
    const int64_t n = c.n;
    const int gb = grid_for(n);
    CK(Apply<T>::run(c, x, q)); c.applies++;
    hipLaunchKernelGGL((k_resid<T, T>), dim3(NBLK), dim3(RT), 0, c.s, b, q, r, n, c.partial);
    if constexpr (std::is_same<T, double>::value) {
        if (c.op == 0 || c.op == 2) {
            // the starting residual projected on the range of the pressure
            // operator (per-time-node mean removed): near the FP64 floor the
            // rounding of b - S x leaves a part along the null space that CG
            // cannot reduce and would amplify
            if (int e = time_sums(c, r)) return e;
            hipLaunchKernelGGL(k_remove_mean<double>, dim3(gb), dim3(256), 0, c.s, r, c.scal + S_TIME, c.m->E,
                               c.m->G, c.m->N);
            hipLaunchKernelGGL((k_dot<double, double>), dim3(NBLK), dim3(RT), 0, c.s, r, r, n, c.partial);
        }
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, c.s, c.partial, NBLK, c.scal, (int)S_RR, (int)FIN_STORE);
    hipLaunchKernelGGL(k_copy<T>, dim3(gb), dim3(256), 0, c.s, r, p, n);
    CK(hipGetLastError());
    double rr;
    if (int e = read_scal(c, S_RR, rr)) return e;
    iters = 0;
    res_out = std::sqrt(rr);
    if (res_out <= tol_abs) return STDG_OK;
    while (iters < max_it) {
        CK(Apply<T>::run(c, p, q)); c.applies++;
        hipLaunchKernelGGL((k_dot<T, T>), dim3(NBLK), dim3(RT), 0, c.s, p, q, n, c.partial);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, c.s, c.partial, NBLK, c.scal, 0, (int)FIN_CG_ALPHA);
        hipLaunchKernelGGL(k_cg_xr<T>, dim3(NBLK), dim3(RT), 0, c.s, x, r, p, q, c.scal, n, c.partial);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, c.s, c.partial, NBLK, c.scal, 0, (int)FIN_CG_BETA);
        hipLaunchKernelGGL(k_cg_p<T>, dim3(gb), dim3(256), 0, c.s, p, r, c.scal, n);
        CK(hipGetLastError());
        ++iters;
        if (iters % check_every == 0 || iters == max_it) {
            if (int e = read_scal(c, S_RR, rr)) return e;
            if (!std::isfinite(rr)) { set_error("non-finite residual in CG"); return STDG_ERR_NUMERIC; }
            res_out = std::sqrt(rr);
            if (res_out <= tol_abs) return STDG_OK;
        }
    }
    return STDG_NOT_CONVERGED;
}

// ---------------------------------------------------------------- BiCGStab
// Scalars live in scal: rho = (r^, r_i), its previous value, alpha = rho /
// (r^, v), omega = (t.s) / (t.t) (see bicgstab()).

__global__ void k_bcg_init(double* __restrict__ scal) {
    scal[S_BRHO] = scal[S_BRR];
    scal[S_BRHOP] = 1.0;
    scal[S_BALPHA] = 1.0;
    scal[S_BOMEGA] = 1.0;
}

// p = r + beta (p - omega v), beta = (rho / rho_prev) (alpha / omega)
template <typename T>
__global__ void k_bcg_p(T* __restrict__ p, const T* __restrict__ r, const T* __restrict__ v,
                        const double* __restrict__ scal, int64_t n) {
    const double om = scal[S_BOMEGA];
    const double beta = (scal[S_BRHO] / scal[S_BRHOP]) * (scal[S_BALPHA] / om);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (T)((double)r[i] + beta * ((double)p[i] - om * (double)v[i]));
}

// s = r - alpha v with alpha = rho / sigma (stored for the x update)
template <typename T>
__global__ void k_bcg_s(T* __restrict__ s, const T* __restrict__ r, const T* __restrict__ v,
                        double* __restrict__ scal, int64_t n) {
    const double alpha = scal[S_BRHO] / scal[S_BSIG];
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_BALPHA] = alpha;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s[i] = (T)((double)r[i] - alpha * (double)v[i]);
}

// block partials of (a . b) and (a . a): partial[blk] and partial[gridDim.x + blk]
template <typename T>
__global__ void __launch_bounds__(RT) k_dot2(const T* __restrict__ a, const T* __restrict__ b, int64_t n,
                                             double* __restrict__ partial) {
    __shared__ double sm[RT / 64];
    double ab = 0.0, aa = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
        const double ai = (double)a[i];
        ab += ai * (double)b[i];
        aa += ai * ai;
    }
    const double t0 = block_sum(ab, sm);
    const double t1 = block_sum(aa, sm);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = t0;
        partial[gridDim.x + blockIdx.x] = t1;
    }
}

// omega = (t.s) / (t.t); x += alpha p + omega s; r = s - omega t; block
// partials of (r^, r) and (r . r); rho moves to rho_prev
template <typename T>
__global__ void __launch_bounds__(RT) k_bcg_xr(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                                               const T* __restrict__ s, const T* __restrict__ t,
                                               const T* __restrict__ rh, double* __restrict__ scal, int64_t n,
                                               double* __restrict__ partial) {
    __shared__ double sm[RT / 64];
    const double alpha = scal[S_BALPHA];
    const double tt = scal[S_BTT];
    const double om = tt > 0.0 ? scal[S_BTS] / tt : 0.0;
    double a0 = 0.0, a1 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
        const double si = (double)s[i];
        x[i] = (T)((double)x[i] + alpha * (double)p[i] + om * si);
        const T ri = (T)(si - om * (double)t[i]);
        r[i] = ri;
        a0 += (double)rh[i] * (double)ri;
        a1 += (double)ri * (double)ri;
    }
    const double t0 = block_sum(a0, sm);
    const double t1 = block_sum(a1, sm);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = t0;
        partial[gridDim.x + blockIdx.x] = t1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[S_BOMEGA] = om;
        scal[S_BRHOP] = scal[S_BRHO];
    }
}

// Restarted GMRES(m) with classical Gram-Schmidt applied twice.
template <typename T>
int gmres(Ctx& c, const T* b, T* x, T* r, T* V, int mres, double tol_abs, int max_it, int check_every,
          int& iters, double& res_out) {
    const int64_t n = c.n;
    const int gb = grid_for(n);
    double* H = c.gm;
    double* g = H + (mres + 1) * mres;
    double* cs = g + (mres + 1);
    double* sn = cs + mres;
    double* y = sn + mres;
    double* h = y + mres;            // mres + 1 scratch dots
    iters = 0;
    while (true) {
        // r = b - S x, beta = ||r||, V_0 = r / beta
        CK(Apply<T>::run(c, x, r)); c.applies++;
        hipLaunchKernelGGL((k_resid<T, T>), dim3(NBLK), dim3(RT), 0, c.s, b, r, V, n, c.partial);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, c.s, c.partial, NBLK, c.scal, (int)S_NORM, (int)FIN_SQRT);
        double beta;
        if (int e = read_scal(c, S_NORM, beta)) return e;
        if (!std::isfinite(beta)) { set_error("non-finite residual in GMRES"); return STDG_ERR_NUMERIC; }
        res_out = beta;
        if (beta <= tol_abs) return STDG_OK;
        if (iters >= max_it) return STDG_NOT_CONVERGED;
        hipLaunchKernelGGL(k_scale_inv<T>, dim3(gb), dim3(256), 0, c.s, V, c.scal + S_NORM, n);
        hipLaunchKernelGGL(k_fill<double>, dim3(grid_for((mres + 1) * mres)), dim3(256), 0, c.s, H, 0.0,
                           (int64_t)(mres + 1) * mres);
        hipLaunchKernelGGL(k_init_g, dim3(1), dim3(256), 0, c.s, g, mres, c.scal + S_NORM);
        int k = 0;
        bool conv = false;
        for (; k < mres && iters < max_it; ++k) {
            T* w = V + (int64_t)(k + 1) * n;
            CK(Apply<T>::run(c, V + (int64_t)k * n, w)); c.applies++;
            double* Hk = H + (int64_t)(mres + 1) * k;
            for (int pass = 0; pass < 2; ++pass) {
                hipLaunchKernelGGL(k_multidot<T>, dim3(NBLK), dim3(RT), 0, c.s, V, k + 1, n, w, c.partial);
                hipLaunchKernelGGL(k_fin_multi, dim3(k + 1), dim3(RT), 0, c.s, c.partial, NBLK, h, Hk, 1.0);
                hipLaunchKernelGGL(k_multiaxpy<T>, dim3(gb), dim3(256), 0, c.s, V, k + 1, n, h, -1.0, w);
            }
            hipLaunchKernelGGL((k_dot<T, T>), dim3(NBLK), dim3(RT), 0, c.s, w, w, n, c.partial);
            hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, c.s, c.partial, NBLK, Hk, k + 1, (int)FIN_SQRT);
            hipLaunchKernelGGL(k_scale_inv<T>, dim3(gb), dim3(256), 0, c.s, w, Hk + k + 1, n);
            hipLaunchKernelGGL(k_givens, dim3(1), dim3(1), 0, c.s, H, g, cs, sn, k, mres, c.scal);
            CK(hipGetLastError());
            ++iters;
            if ((k + 1) % check_every == 0 || k + 1 == mres || iters == max_it) {
                double est;
                if (int e = read_scal(c, S_RES, est)) return e;
                if (!std::isfinite(est)) { set_error("non-finite residual in GMRES"); return STDG_ERR_NUMERIC; }
                res_out = est;
                if (est <= tol_abs) { conv = true; ++k; break; }
            }
        }
        // x += V y
        hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(1), 0, c.s, H, g, y, k, mres);
        hipLaunchKernelGGL(k_multiaxpy<T>, dim3(gb), dim3(256), 0, c.s, V, k, n, y, 1.0, x);
        CK(hipGetLastError());
        (void)conv;
    }
}

template <typename T>
int bicgstab(Ctx& c, const T* b, T* x, T* r, T* rh, T* p, T* v, T* s, T* t, double tol_abs, int max_it,
             int check_every, int& iters, double& res_out);

template <typename T>
int run_krylov(Ctx& c, int method, const T* b, T* x, T* r, T* p, T* q, T* V, int mres, double tol_abs,
               int max_it, int check_every, int& iters, double& res) {
    if (method == STDG_CG) return cg<T>(c, b, x, r, p, q, tol_abs, max_it, check_every, iters, res);
    if (method == STDG_CG_TIME && c.op == 0) {
        // S x = b  <=>  (B (x) I) w = b with w = (I (x) C) x; the residual is the same vector
        CK(Apply<T>::tmix(c, false, x, q));
        hipLaunchKernelGGL(k_copy<T>, dim3(grid_for(c.n)), dim3(256), 0, c.s, q, x, c.n);
        c.op = 2;
        const int st = cg<T>(c, b, x, r, p, q, tol_abs, max_it, check_every, iters, res);
        c.op = 0;
        CK(Apply<T>::tmix(c, true, x, q));
        hipLaunchKernelGGL(k_copy<T>, dim3(grid_for(c.n)), dim3(256), 0, c.s, q, x, c.n);
        CK(hipGetLastError());
        return st;
    }
    if (method == STDG_BICGSTAB)    // r^, s, t in the first three basis vectors (mres >= 2)
        return bicgstab<T>(c, b, x, r, V, p, q, V + c.n, V + 2 * c.n, tol_abs, max_it, check_every, iters, res);
    return gmres<T>(c, b, x, r, V, mres, tol_abs, max_it, check_every, iters, res);
}

// BiCGStab (van der Vorst): short recurrences, two operator applies per
// iteration and no basis to orthogonalise against.  r^ = r_0; scalars and
// the stopping quantity |r|^2 stay on the device, the host reads |r| every
// check_every iterations.  Vectors: r, r^, p, v, s, t (s may share x's
// storage only through the caller's buffers, none alias here).
template <typename T>
int bicgstab(Ctx& c, const T* b, T* x, T* r, T* rh, T* p, T* v, T* s, T* t, double tol_abs, int max_it,
             int check_every, int& iters, double& res_out) {
    const int64_t n = c.n;
    const int gb = grid_for(n);
    CK(Apply<T>::run(c, x, v)); c.applies++;
    hipLaunchKernelGGL((k_resid<T, T>), dim3(NBLK), dim3(RT), 0, c.s, b, v, r, n, c.partial);
    if constexpr (std::is_same<T, double>::value) {
        if (c.op == 0 || c.op == 2) {
            // starting residual on the range of the pressure operator (as in cg())
            if (int e = time_sums(c, r)) return e;
            hipLaunchKernelGGL(k_remove_mean<double>, dim3(gb), dim3(256), 0, c.s, r, c.scal + S_TIME, c.m->E,
                               c.m->G, c.m->N);
            hipLaunchKernelGGL((k_dot<double, double>), dim3(NBLK), dim3(RT), 0, c.s, r, r, n, c.partial);
        }
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, c.s, c.partial, NBLK, c.scal, (int)S_BRR, (int)FIN_STORE);
    hipLaunchKernelGGL(k_copy<T>, dim3(gb), dim3(256), 0, c.s, r, rh, n);
    hipLaunchKernelGGL(k_fill<T>, dim3(gb), dim3(256), 0, c.s, p, (T)0, n);
    hipLaunchKernelGGL(k_fill<T>, dim3(gb), dim3(256), 0, c.s, v, (T)0, n);
    hipLaunchKernelGGL(k_bcg_init, dim3(1), dim3(1), 0, c.s, c.scal);
    CK(hipGetLastError());
    double rr;
    if (int e = read_scal(c, S_BRR, rr)) return e;
    iters = 0;
    res_out = std::sqrt(rr);
    if (!std::isfinite(res_out)) { set_error("non-finite residual in BiCGStab"); return STDG_ERR_NUMERIC; }
    if (res_out <= tol_abs) return STDG_OK;
    while (iters < max_it) {
        hipLaunchKernelGGL(k_bcg_p<T>, dim3(gb), dim3(256), 0, c.s, p, r, v, c.scal, n);
        CK(Apply<T>::run(c, p, v)); c.applies++;
        hipLaunchKernelGGL((k_dot<T, T>), dim3(NBLK), dim3(RT), 0, c.s, rh, v, n, c.partial);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, c.s, c.partial, NBLK, c.scal, (int)S_BSIG,
                           (int)FIN_STORE);
        hipLaunchKernelGGL(k_bcg_s<T>, dim3(gb), dim3(256), 0, c.s, s, r, v, c.scal, n);
        CK(Apply<T>::run(c, s, t)); c.applies++;
        hipLaunchKernelGGL(k_dot2<T>, dim3(NBLK), dim3(RT), 0, c.s, t, s, n, c.partial);
        hipLaunchKernelGGL(k_fin_multi, dim3(2), dim3(RT), 0, c.s, c.partial, NBLK, c.scal + S_BTS,
                           (double*)nullptr, 0.0);
        hipLaunchKernelGGL(k_bcg_xr<T>, dim3(NBLK), dim3(RT), 0, c.s, x, r, p, s, t, rh, c.scal, n, c.partial);
        hipLaunchKernelGGL(k_fin_multi, dim3(2), dim3(RT), 0, c.s, c.partial, NBLK, c.scal + S_BRHO,
                           (double*)nullptr, 0.0);
        CK(hipGetLastError());
        ++iters;
        if (iters % check_every == 0 || iters == max_it) {
            if (int e = read_scal(c, S_BRR, rr)) return e;
            if (!std::isfinite(rr)) { set_error("non-finite residual in BiCGStab"); return STDG_ERR_NUMERIC; }
            res_out = std::sqrt(rr);
            if (res_out <= tol_abs) return STDG_OK;
        }
    }
    return STDG_NOT_CONVERGED;
}

int ensure_workspace(stdg_mesh* m, int mres, bool need32) {
    Workspace& w = m->ws;
    const size_t n = (size_t)m->E * m->Nst;
    if (w.n != n) {
        // first use on this mesh
        w.n = n;
        STDG_HIP(hipMalloc(&w.r, n * sizeof(double)));
        STDG_HIP(hipMalloc(&w.p, n * sizeof(double)));
        STDG_HIP(hipMalloc(&w.q, n * sizeof(double)));
        STDG_HIP(hipMalloc(&w.z, n * sizeof(double)));
        STDG_HIP(hipMalloc(&w.partial, sizeof(double) * NBLK * 208));
        STDG_HIP(hipMalloc(&w.scal, sizeof(double) * (S_COUNT + 4 * 256 + 208 * 208)));
        STDG_HIP(hipHostMalloc(&w.hscal, sizeof(double) * 8));
    }
    if (need32) {
        // long enough for the run layout as well (padded to whole 64-element runs)
        const size_t n32 = std::max<size_t>(n, (size_t)lane_len(m));
        for (float** f : {&w.r32, &w.p32, &w.q32, &w.x32, &w.b32, &w.p32b, &w.r32b, &w.q32b})
            if (!*f) STDG_HIP(hipMalloc(f, n32 * sizeof(float)));
        if (!w.ev[0])
            for (hipEvent_t& e : w.ev) STDG_HIP(hipEventCreate(&e));
    }
    if (mres > w.restart) {
        if (w.V) STDG_HIP(hipFree(w.V));
        if (w.V32) STDG_HIP(hipFree(w.V32));
        w.V = nullptr; w.V32 = nullptr;
        STDG_HIP(hipMalloc(&w.V, n * sizeof(double) * (mres + 1)));
        w.restart = mres;
    }
    if (need32 && mres > 0 && !w.V32) STDG_HIP(hipMalloc(&w.V32, n * sizeof(float) * (w.restart + 1)));
    return STDG_OK;
}

}  // namespace

void free_workspace(stdg_mesh* m) {
    Workspace& w = m->ws;
    for (void* p : {(void*)w.r, (void*)w.p, (void*)w.q, (void*)w.z, (void*)w.V, (void*)w.r32, (void*)w.p32,
                    (void*)w.q32, (void*)w.x32, (void*)w.b32, (void*)w.V32, (void*)w.partial, (void*)w.scal,
                    (void*)w.p32b, (void*)w.r32b, (void*)w.q32b})
        if (p) (void)hipFree(p);
    if (w.hscal) (void)hipHostFree(w.hscal);
    for (hipEvent_t e : w.ev)
        if (e) (void)hipEventDestroy(e);
    w = Workspace();
}

// out[i] = a[i] . b[i] (i < k) in FP64, deterministic; synchronises s.
int device_dots(stdg_mesh* m, int k, const double* const* a, const double* const* b, int64_t n, hipStream_t s,
                double* out) {
    if (int e = ensure_workspace(m, 0, false)) return e;
    Ctx c;
    c.m = m;
    c.s = s;
    c.partial = m->ws.partial;
    c.scal = m->ws.scal;
    c.hscal = m->ws.hscal;
    for (int i = 0; i < k; ++i) {
        hipLaunchKernelGGL((k_dot<double, double>), dim3(NBLK), dim3(RT), 0, s, a[i], b[i], n, c.partial);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, s, c.partial, NBLK, c.scal, (int)S_TMP, (int)FIN_STORE);
        CK(hipGetLastError());
        if (int e = read_scal(c, S_TMP, out[i])) return e;
    }
    return STDG_OK;
}

// Plain (non-singular) solve A_v x = b of the viscous system with the
// library's CG/GMRES; x holds the guess.  Vectors [3][E][G][N]; work vectors
// are taken from `work` ((restart + 6) * n doubles).  GMRES runs on the
// left block-Jacobi preconditioned system D^-1 A x = D^-1 b, D the exact
// space-time diagonal block of each element; convergence is judged on the
// true residual of A x = b.
int viscous_solve(stdg_mesh* m, const double* b, double* x, const stdg_solve_opts& o, double* work,
                  hipStream_t s, int& iters, double& rel) {
    if (int e = ensure_workspace(m, 0, false)) return e;
    Ctx c;
    c.m = m;
    c.s = s;
    c.n = 3 * m->E * m->Nst;
    c.partial = m->ws.partial;
    c.scal = m->ws.scal;
    c.hscal = m->ws.hscal;
    c.gm = m->ws.scal + S_COUNT;
    c.op = 1;
    const int64_t n = c.n;
    double* r = work;
    double* pp = work + n;
    double* q = work + 2 * n;
    double* V = work + 3 * n;
    const int method = o.method == STDG_AUTO ? STDG_GMRES : o.method;
    const bool pre = method == STDG_GMRES || method == STDG_BICGSTAB;
    if (method == STDG_GMRES && o.restart < 1) { set_error("viscous GMRES restart must be >= 1"); return STDG_ERR_ARG; }
    if (method == STDG_BICGSTAB && o.restart < 2) {
        set_error("viscous BiCGStab keeps r^, s, t in the first three basis vectors: restart must be >= 2");
        return STDG_ERR_ARG;
    }
    if (method != STDG_GMRES && method != STDG_CG && method != STDG_BICGSTAB) {
        set_error("viscous method must be CG, GMRES or BiCGStab");
        return STDG_ERR_ARG;
    }
    double* bp = work + (int64_t)(o.restart + 5) * n;
    c.tmp = work + (int64_t)(o.restart + 4) * n;
    hipLaunchKernelGGL((k_dot<double, double>), dim3(NBLK), dim3(RT), 0, s, b, b, n, c.partial);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, s, c.partial, NBLK, c.scal, (int)S_BN2, (int)FIN_STORE);
    double bn2;
    if (int e = read_scal(c, S_BN2, bn2)) return e;
    if (!std::isfinite(bn2)) { set_error("non-finite viscous right-hand side"); return STDG_ERR_NUMERIC; }
    const double bn = std::sqrt(bn2);
    iters = 0;
    rel = 0.0;
    if (bn == 0.0) {
        hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n)), dim3(256), 0, s, x, 0.0, n);
        return STDG_OK;
    }
    double tol = o.rtol * bn;
    const double* rhs = b;
    if (pre) {
        CK(launch_visc_precond(m, b, bp, s));
        hipLaunchKernelGGL((k_dot<double, double>), dim3(NBLK), dim3(RT), 0, s, bp, bp, n, c.partial);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, s, c.partial, NBLK, c.scal, (int)S_BN2, (int)FIN_STORE);
        double pn2;
        if (int e = read_scal(c, S_BN2, pn2)) return e;
        tol = o.rtol * std::sqrt(pn2);
        rhs = bp;
        c.op = 3;
    }
    int status = STDG_OK;
    for (int round = 0; round < 6; ++round) {
        int it = 0;
        double res = 0.0;
        const int left = o.max_iter - iters;
        if (left <= 0) { status = STDG_NOT_CONVERGED; break; }
        status = run_krylov<double>(c, method, rhs, x, r, pp, q, V, o.restart, tol, left, o.check_every, it, res);
        iters += it;
        if (status < 0) return status;
        // true residual
        CK(launch_visc_apply(m, x, q, s));
        hipLaunchKernelGGL((k_resid<double, double>), dim3(NBLK), dim3(RT), 0, s, b, q, r, n, c.partial);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, s, c.partial, NBLK, c.scal, (int)S_RN2, (int)FIN_STORE);
        double rn2;
        if (int e = read_scal(c, S_RN2, rn2)) return e;
        rel = std::sqrt(rn2) / bn;
        if (rel <= o.rtol) { status = STDG_OK; break; }
        if (status == STDG_NOT_CONVERGED) break;
        tol *= std::min(0.25, std::max(1e-4, 0.5 * o.rtol / rel));
    }
    if (status == STDG_OK && rel > o.rtol) status = STDG_NOT_CONVERGED;
    return status;
}

}  // namespace stdg

using namespace stdg;

extern "C" void stdg_solve_opts_default(stdg_solve_opts* o) {
    if (!o) return;
    o->method = STDG_AUTO;
    o->restart = 50;
    o->rtol = 1e-10;
    o->max_iter = 20000;
    o->precision = STDG_FP64;
    o->inner_rtol = 1e-4;
    o->max_outer = 30;
    o->check_every = 8;
    o->precond = STDG_PRECOND_BLOCK_JACOBI;
}

namespace stdg {
namespace {

// Checks the options of a pressure solve and resolves STDG_AUTO; mres is set
// to the number of basis vectors the method keeps (0 for the CG methods).
int check_solve_opts(const stdg_mesh* m, stdg_solve_opts& o, int& mres) {
    if (o.method == STDG_AUTO) o.method = (m->G == 1) ? STDG_CG : STDG_GMRES;
    if (o.method != STDG_CG && o.method != STDG_GMRES && o.method != STDG_CG_TIME && o.method != STDG_BICGSTAB) {
        set_error("unknown method");
        return STDG_ERR_ARG;
    }
    if (o.method == STDG_CG && m->G > 1) {
        set_error("CG needs p_gamma = 0 (the space-time operator is not symmetric); use STDG_CG_TIME");
        return STDG_ERR_ARG;
    }
    if (o.method == STDG_GMRES && (o.restart < 1 || o.restart > 200)) { set_error("restart out of range"); return STDG_ERR_ARG; }
    if (!(o.rtol > 0.0) || o.max_iter < 1 || o.check_every < 1) { set_error("bad tolerance/iteration options"); return STDG_ERR_ARG; }
    if (o.precond != STDG_PRECOND_NONE && o.precond != STDG_PRECOND_BLOCK_JACOBI) { set_error("bad preconditioner"); return STDG_ERR_ARG; }
    if (o.precision != STDG_FP64 && o.precision != STDG_FP32) { set_error("bad precision"); return STDG_ERR_ARG; }
    if (o.precision == STDG_FP32 && (!(o.inner_rtol > 0.0) || o.max_outer < 1)) {
        set_error("bad refinement options");
        return STDG_ERR_ARG;
    }
    mres = (o.method == STDG_GMRES) ? o.restart : (o.method == STDG_BICGSTAB ? 2 : 0);
    return STDG_OK;
}

// The anchored solve itself, on the work buffers of w (vectors r, p, q, z of
// w.n doubles, the GMRES/BiCGStab basis V, the FP32 vectors when o asks for
// refinement, reduction partials, device scalars and a host mirror).
int solve_with(stdg_mesh* m, const double* b, double* x, const stdg_solve_opts& o, int mres,
               stdg_solve_report* rep, void* stream, Workspace& w, std::chrono::steady_clock::time_point t0) {
    const bool ir = o.precision == STDG_FP32;
    Ctx c;
    c.m = m;
    c.s = (hipStream_t)stream;
    c.n = (int64_t)w.n;
    c.partial = w.partial;
    c.scal = w.scal;
    c.hscal = w.hscal;
    c.gm = w.scal + S_COUNT;
    c.precond = o.precond == STDG_PRECOND_BLOCK_JACOBI;
    const int64_t n = c.n;
    const int gb = grid_for(n);
    const int G = m->G, N = m->N;
    // b~ (consistent right-hand side) in w.z
    hipLaunchKernelGGL(k_copy<double>, dim3(gb), dim3(256), 0, c.s, b, w.z, n);
    if (int e = time_sums(c, w.z)) return e;
    hipLaunchKernelGGL(k_set_anchor, dim3(1), dim3(64), 0, c.s, w.z, c.scal + S_TIME, m->anchor, m->anchor_node, G, N);
    // ||b_a||
    hipLaunchKernelGGL(k_anch_res, dim3(NBLK), dim3(RT), 0, c.s, b, b, m->anchor, m->anchor_node, m->E, G, N, c.partial);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, c.s, c.partial + NBLK, NBLK, c.scal, (int)S_BN2, (int)FIN_STORE);
    double bn2;
    if (int e = read_scal(c, S_BN2, bn2)) return e;
    if (!std::isfinite(bn2)) { set_error("non-finite right-hand side"); return STDG_ERR_NUMERIC; }
    const double bnorm = std::sqrt(bn2);
    int status = STDG_OK, inner_total = 0, outer = 0;
    double rel = 0.0, rel0 = 0.0;
    // shift x to x_anchor = 0, set q = S x, r = b~ - S x (consistent residual)
    // and return the anchored relative residual ||b_a - S_a x|| / ||b_a||.
    auto check = [&](double& out) -> int {
        hipLaunchKernelGGL(k_read_anchor, dim3(1), dim3(64), 0, c.s, x, c.scal + S_ANCH, m->anchor, m->anchor_node, G, N);
        hipLaunchKernelGGL(k_shift, dim3(gb), dim3(256), 0, c.s, x, c.scal + S_ANCH, m->E, G, N);
        CK(launch_apply_f64(m, x, w.q, c.s)); c.applies++;
        hipLaunchKernelGGL((k_resid<double, double>), dim3(NBLK), dim3(RT), 0, c.s, w.z, w.q, w.r, n, c.partial);
        hipLaunchKernelGGL(k_anch_res, dim3(NBLK), dim3(RT), 0, c.s, b, w.q, m->anchor, m->anchor_node, m->E, G, N,
                           c.partial + NBLK);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, c.s, c.partial + NBLK, NBLK, c.scal, (int)S_RN2, (int)FIN_STORE);
        CK(hipGetLastError());
        double rn2;
        if (int e = read_scal(c, S_RN2, rn2)) return e;
        out = std::sqrt(rn2) / bnorm;
        if (!std::isfinite(out)) { set_error("non-finite residual"); return STDG_ERR_NUMERIC; }
        return STDG_OK;
    };
    if (bnorm == 0.0) {
        hipLaunchKernelGGL(k_fill<double>, dim3(gb), dim3(256), 0, c.s, x, 0.0, n);
    } else if (!ir) {
        int it = 0;
        double res = 0.0, tol_abs = o.rtol * bnorm;
        outer = 1;
        if (int e = check(rel0)) return e;
        rel = rel0;
        // the recursive residual may drift from the true one: restart from the
        // true residual (with a tighter target) until the anchored residual
        // meets the tolerance
        for (int round = 0; round < 6 && rel > o.rtol; ++round) {
            const int left = o.max_iter - inner_total;
            if (left <= 0) { status = STDG_NOT_CONVERGED; break; }
            status = run_krylov<double>(c, o.method, w.z, x, w.r, w.p, w.q, w.V, mres, tol_abs, left,
                                        o.check_every, it, res);
            inner_total += it;
            if (status < 0) return status;
            if (int e = check(rel)) return e;
            if (rel <= o.rtol) { status = STDG_OK; break; }
            if (status == STDG_NOT_CONVERGED) break;
            tol_abs *= 0.25;
        }
        if (status == STDG_OK && rel > o.rtol) status = STDG_NOT_CONVERGED;
    } else {
        // FP64 iterative refinement around FP32 Krylov solves
        const bool run_inner = lane_supported(m) && (o.method == STDG_CG || o.method == STDG_CG_TIME) &&
                               w.p32b && 2 * cg_partial_len(m) <= (int64_t)NBLK * 208;
        for (outer = 1; outer <= o.max_outer + 1; ++outer) {
            if (int e = check(rel)) return e;
            if (outer == 1) rel0 = rel;
            if (rel <= o.rtol) { status = STDG_OK; break; }
            if (outer > o.max_outer || inner_total >= o.max_iter) { status = STDG_NOT_CONVERGED; break; }
            // inner right-hand side: the consistent residual projected on the
            // range of S (per-time-node mean removed), in FP32
            if (int e = time_sums(c, w.r)) return e;
            hipLaunchKernelGGL(k_remove_mean<double>, dim3(gb), dim3(256), 0, c.s, w.r, c.scal + S_TIME, m->E, G, N);
            hipLaunchKernelGGL((k_dot<double, double>), dim3(NBLK), dim3(RT), 0, c.s, w.r, w.r, n, c.partial);
            hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, c.s, c.partial, NBLK, c.scal, (int)S_NORM, (int)FIN_SQRT);
            double rn;
            if (int e = read_scal(c, S_NORM, rn)) return e;
            if (!(rn > 0.0)) { status = STDG_NOT_CONVERGED; break; }
            // the inner system is solved for the unit-norm right-hand side
            // r / |r| (FP32 vectors and products then stay far from the ends
            // of the FP32 range whatever the scale of the problem) and the
            // correction scaled back by |r|
            int it = 0;
            double res = 0.0;
            // each inner solve reduces the residual by inner_rtol, but never
            // further than the final tolerance needs (a good initial guess
            // then saves inner iterations instead of overshooting)
            const double inner_abs = std::max(o.inner_rtol * rn, 0.25 * o.rtol * bnorm);
            if (run_inner) {
                // element-per-lane kernels: CG on c B (STDG_CG) or on B (x) I
                // (STDG_CG_TIME, correction (I (x) C^-1) w) in the run layout
                const int64_t n32 = lane_len(m);
                CK(lane_pack(m, w.r, 1.0 / rn, w.b32, c.s));
                hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n32)), dim3(256), 0, c.s, w.x32, 0.0f, n32);
                c.n = n32;
                c.run_layout = true;
                c.op = o.method == STDG_CG ? 0 : 2;
                status = cg<float>(c, w.b32, w.x32, w.r32, w.p32, w.q32, inner_abs / rn, o.max_iter - inner_total,
                                   o.check_every, it, res);
                c.n = n;
                c.run_layout = false;
                c.op = 0;
                inner_total += it;
                if (status < 0) return status;
                CK(lane_unpack(m, w.x32, o.method == STDG_CG ? nullptr : m->d.Cinv, rn, true, x, c.s));
            } else {
                hipLaunchKernelGGL(k_d2f_scaled, dim3(gb), dim3(256), 0, c.s, w.r, w.b32, 1.0 / rn, n);
                hipLaunchKernelGGL(k_fill<float>, dim3(gb), dim3(256), 0, c.s, w.x32, 0.0f, n);
                status = run_krylov<float>(c, o.method, w.b32, w.x32, w.r32, w.p32, w.q32, w.V32, mres,
                                           inner_abs / rn, o.max_iter - inner_total, o.check_every, it, res);
                inner_total += it;
                if (status < 0) return status;
                hipLaunchKernelGGL(k_add_f32, dim3(gb), dim3(256), 0, c.s, x, w.x32, rn, n);
            }
            CK(hipGetLastError());
        }
        outer = std::min(outer, o.max_outer);
    }
    CK(hipStreamSynchronize(c.s));
    if (rep) {
        rep->status = status;
        rep->outer_iters = outer;
        rep->inner_iters = inner_total;
        rep->applies = c.applies;
        rep->rel_residual = rel;
        rep->initial_rel_residual = rel0;
        rep->fused_iter_us = c.loop_iters ? 1e3 * c.loop_ms / c.loop_iters : 0.0;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

}  // namespace
}  // namespace stdg

extern "C" int stdg_pressure_solve(const stdg_mesh* cm, const double* b, double* x,
                                   const stdg_solve_opts* opts, stdg_solve_report* rep, void* stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (!cm || !b || !x || !opts) { set_error("null argument"); return STDG_ERR_ARG; }
    stdg_mesh* m = const_cast<stdg_mesh*>(cm);
    if (!m->d.blocks) { set_error("mesh was built host-only"); return STDG_ERR_ARG; }
    stdg_solve_opts o = *opts;
    int mres = 0;
    if (int e = check_solve_opts(m, o, mres)) return e;
    if (int e = ensure_workspace(m, mres, o.precision == STDG_FP32)) return e;
    return solve_with(m, b, x, o, mres, rep, stream, m->ws, t0);
}

// ------------------------------------------------------------------ no-allocation solve
// The FP64 CG solves (STDG_CG, STDG_CG_TIME) with every work buffer in one
// file-scope device array: four vectors of at most NOALLOC_MAX_DOF doubles,
// the reduction partials and the device scalars (35.6 MB per GPU, held until
// the process ends).  Host code never uses the array's name as an address:
// each device's copy is looked up once with hipGetSymbolAddress.
namespace stdg {
namespace {

constexpr int64_t NOALLOC_MAX_DOF = int64_t(1) << 20;
constexpr int64_t SCR_PARTIAL = (int64_t)NBLK * 208;
constexpr int64_t SCR_SCAL = S_COUNT + 4 * 256 + 208 * 208;
constexpr int64_t SCR_DOUBLES = 4 * NOALLOC_MAX_DOF + SCR_PARTIAL + SCR_SCAL;

static __device__ __align__(256) double scratch[SCR_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_dev[MAX_DEVICES] = {};

// Device address of the current device's scratch array (looked up on the
// first call on that device).
int scratch_address(double** out) {
    int dev = 0;
    STDG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) { set_error("device index out of range"); return STDG_ERR_DEVICE; }
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void* ptr = nullptr;
        STDG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) { set_error("no device address for the scratch array"); return STDG_ERR_DEVICE; }
        scratch_dev[dev] = static_cast<double*>(ptr);
    }
    *out = scratch_dev[dev];
    return STDG_OK;
}

}  // namespace
}  // namespace stdg

extern "C" int stdg_pressure_solve_noalloc(const stdg_mesh* cm, const double* b, double* x,
                                           const stdg_solve_opts* opts, stdg_solve_report* rep, void* stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (!cm || !b || !x || !opts) { set_error("null argument"); return STDG_ERR_ARG; }
    stdg_mesh* m = const_cast<stdg_mesh*>(cm);
    if (!m->d.blocks) { set_error("mesh was built host-only"); return STDG_ERR_ARG; }
    stdg_solve_opts o = *opts;
    int mres = 0;
    if (int e = check_solve_opts(m, o, mres)) return e;
    if (o.precision != STDG_FP64 || (o.method != STDG_CG && o.method != STDG_CG_TIME)) {
        set_error("the no-allocation solve supports FP64 precision with STDG_CG or STDG_CG_TIME only");
        return STDG_ERR_ARG;
    }
    const int64_t n = m->E * (int64_t)m->Nst;
    if (n > NOALLOC_MAX_DOF) {
        set_error("the no-allocation solve holds at most " + std::to_string(NOALLOC_MAX_DOF) +
                  " pressure unknowns; this mesh has " + std::to_string(n));
        return STDG_ERR_ARG;
    }
    double* base = nullptr;
    if (int e = scratch_address(&base)) return e;
    Workspace w;
    w.n = (size_t)n;
    w.r = base;
    w.p = base + NOALLOC_MAX_DOF;
    w.q = base + 2 * NOALLOC_MAX_DOF;
    w.z = base + 3 * NOALLOC_MAX_DOF;
    w.partial = base + 4 * NOALLOC_MAX_DOF;
    w.scal = w.partial + SCR_PARTIAL;
    double host_mirror[8] = {0.0};
    w.hscal = host_mirror;
    // the previous call's scalars are cleared by a kernel (no memset node)
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(SCR_SCAL)), dim3(256), 0, (hipStream_t)stream, w.scal, 0.0,
                       SCR_SCAL);
    CK(hipGetLastError());
    return solve_with(m, b, x, o, mres, rep, stream, w, t0);
}

namespace stdg {
namespace {
__global__ void k_f2d_scaled(const float* __restrict__ a, double* __restrict__ b, double scale, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = scale * (double)a[i];
}
}  // namespace
}  // namespace stdg

extern "C" int stdg_inner_from_f64(const stdg_mesh* m, const double* x, double scale, float* y, void* stream) {
    if (!m || !x || !y) { set_error("null argument"); return STDG_ERR_ARG; }
    if (!m->d.blocks) { set_error("mesh was built host-only"); return STDG_ERR_ARG; }
    const hipStream_t s = (hipStream_t)stream;
    if (lane_supported(m)) {
        CK(lane_pack(m, x, scale, y, s));
    } else {
        const int64_t n = m->E * m->G * m->N;
        hipLaunchKernelGGL(k_d2f_scaled, dim3(grid_for(n)), dim3(256), 0, s, x, y, scale, n);
        CK(hipGetLastError());
    }
    return STDG_OK;
}

extern "C" int stdg_inner_to_f64(const stdg_mesh* m, const float* y, double scale, double* x, void* stream) {
    if (!m || !x || !y) { set_error("null argument"); return STDG_ERR_ARG; }
    if (!m->d.blocks) { set_error("mesh was built host-only"); return STDG_ERR_ARG; }
    const hipStream_t s = (hipStream_t)stream;
    if (lane_supported(m)) {
        CK(lane_unpack(m, y, nullptr, scale, false, x, s));
    } else {
        const int64_t n = m->E * m->G * m->N;
        hipLaunchKernelGGL(k_f2d_scaled, dim3(grid_for(n)), dim3(256), 0, s, y, x, scale, n);
        CK(hipGetLastError());
    }
    return STDG_OK;
}

// y = (B (x) I) x in FP32 with the CG operator kernel (inner layout).
extern "C" int stdg_pressure_apply_spatial_f32(const stdg_mesh* cm, const float* x, float* y, void* stream) {
    if (!cm || !x || !y) { set_error("null argument"); return STDG_ERR_ARG; }
    stdg_mesh* m = const_cast<stdg_mesh*>(cm);
    if (!m->d.blocks) { set_error("mesh was built host-only"); return STDG_ERR_ARG; }
    hipError_t e;
    if (lane_supported(m)) {
        e = lane_apply_f32(m, x, y, 1.0f, (hipStream_t)stream);
    } else if (cg_fused_supported(m)) {
        e = launch_cg_apply_f32(m, x, y, 1.0f, (hipStream_t)stream);
    } else {
        set_error("no FP32 MFMA spatial operator for this mesh (p = 1, 2, 3, or p = 4 on meshes whose "
                  "64-element runs mostly share a geometry class)");
        return STDG_ERR_ARG;
    }
    if (e != hipSuccess) { set_error(std::string("spatial apply: ") + hipGetErrorString(e)); return STDG_ERR_DEVICE; }
    return STDG_OK;
}
