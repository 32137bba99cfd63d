// One Picard pressure-correction time step of the staggered space-time DG
// scheme (Sec. 2.6, steps 0-6) on the device, with the tables built by
// picard_tables.cpp.
//
// Layouts: dual velocity [3][F][G][N] (faces in the library's order: interior
// first, then boundary), main-grid velocity [3][E][G][N], pressure [E][G][N].
// Every spatial block is N x N row-major; a kernel thread computes one output
// row r of one (component, element or face, time node).
#include <chrono>
#include <cmath>

#include "internal.hpp"
#include "kernels.hpp"

namespace stdg {

namespace {

#define CKP(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { set_error(std::string(#x) + ": " + hipGetErrorString(e_)); return STDG_ERR_DEVICE; } } while (0)

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// value at the end of the previous slab, broadcast over the new slab's nodes
__global__ void k_time_end(const double* __restrict__ in, double* __restrict__ out,
                           const double* __restrict__ g1, int64_t rows, int G, int N) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (row, n)
    if (t >= rows * N) return;
    const int64_t row = t / N;
    const int n = (int)(t - row * N);
    double s = 0.0;
    for (int b = 0; b < G; ++b) s += g1[b] * in[(row * G + b) * N + n];
    for (int a = 0; a < G; ++a) out[(row * G + a) * N + n] = s;
}

// eq. goback: Fv_j = GB_l vbar_l + GB_r vbar_r (interior); one side from
// `vbdry` on boundary faces (the projected Dirichlet data).  Faces [f0, f1).
__global__ void k_goback(const double* __restrict__ GB, const int32_t* __restrict__ cls,
                         const int64_t* __restrict__ fl, const int32_t* __restrict__ flf,
                         const int64_t* __restrict__ fr, const int32_t* __restrict__ frf,
                         const double* __restrict__ vbar, const double* __restrict__ vbdry,
                         double* __restrict__ out, int64_t f0, int64_t f1, int64_t F, int64_t E,
                         int G, int N) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nf = f1 - f0;
    if (t >= 3 * nf * G * N) return;
    const int r = (int)(t % N);
    const int a = (int)((t / N) % G);
    const int64_t j = f0 + (t / ((int64_t)N * G)) % nf;
    const int c = (int)(t / ((int64_t)N * G * nf));
    const int64_t l = fl[j], rr = fr[j];
    const double* src = rr >= 0 ? vbar : vbdry;
    const double* B = GB + (((int64_t)cls[l] * 4 + flf[j]) * N + r) * N;
    const double* x = src + ((c * E + l) * G + a) * N;
    double s = 0.0;
    for (int m = 0; m < N; ++m) s += B[m] * x[m];
    if (rr >= 0) {
        const double* B2 = GB + (((int64_t)cls[rr] * 4 + frf[j]) * N + r) * N;
        const double* x2 = vbar + ((c * E + rr) * G + a) * N;
        for (int m = 0; m < N; ++m) s += B2[m] * x2[m];
    }
    out[((c * F + j) * G + a) * N + r] = s;
}

// eq. average: vbar_i = sum_f A_f vhat_face(i,f)   (3 components)
__global__ void k_average(const double* __restrict__ A, const int32_t* __restrict__ cls,
                          const int64_t* __restrict__ tet_face, const double* __restrict__ vhat,
                          double* __restrict__ vbar, int64_t E, int64_t F, int G, int N) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * E * G * N) return;
    const int r = (int)(t % N);
    const int a = (int)((t / N) % G);
    const int64_t i = (t / ((int64_t)N * G)) % E;
    const int c = (int)(t / ((int64_t)N * G * E));
    double s = 0.0;
    for (int f = 0; f < 4; ++f) {
        const int64_t j = tet_face[4 * i + f];
        const double* B = A + (((int64_t)cls[i] * 4 + f) * N + r) * N;
        const double* x = vhat + ((c * F + j) * G + a) * N;
        for (int m = 0; m < N; ++m) s += B[m] * x[m];
    }
    vbar[((c * E + i) * G + a) * N + r] = s;
}

// Dual-grid pressure gradient (eqs. prevpress / A3_mod):
// w_j[d][a] = dt sum_b TW_ab (US_d p_l[b] + UN_d p_r[b]) with the left
// element's tables; boundary faces: US (volume part) only.
__global__ void k_dualgrad(const double* __restrict__ US, const double* __restrict__ UN,
                           const int32_t* __restrict__ cls, const int64_t* __restrict__ fl,
                           const int32_t* __restrict__ flf, const int64_t* __restrict__ fr,
                           const double* __restrict__ TW, const double* __restrict__ p, double dt,
                           double* __restrict__ w, int64_t F, int G, int N) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * F * G * N) return;
    const int r = (int)(t % N);
    const int a = (int)((t / N) % G);
    const int64_t j = (t / ((int64_t)N * G)) % F;
    const int d = (int)(t / ((int64_t)N * G * F));
    const int64_t l = fl[j], rr = fr[j];
    const int64_t blk = (((int64_t)cls[l] * 4 + flf[j]) * 3 + d) * N + r;
    const double* Bs = US + blk * N;
    const double* Bn = UN + blk * N;
    double s = 0.0;
    for (int b = 0; b < G; ++b) {
        const double tw = TW[a * G + b];
        if (tw == 0.0) continue;
        const double* pl = p + (l * G + b) * N;
        double u = 0.0;
        for (int m = 0; m < N; ++m) u += Bs[m] * pl[m];
        if (rr >= 0) {
            const double* pr = p + (rr * G + b) * N;
            for (int m = 0; m < N; ++m) u += Bn[m] * pr[m];
        }
        s += tw * u;
    }
    w[((d * F + j) * G + a) * N + r] = dt * s;
}

// Viscous right-hand side (eq. A1_mod):
// Mbar_i^- vbar^n - Upsilon - Mbar_i Lambda - nu dt sum_bdry (BB (x) W) vbc
__global__ void k_visc_rhs(const double* __restrict__ MI, const double* __restrict__ BB,
                           const int32_t* __restrict__ cls, const int32_t* __restrict__ nbr,
                           const int64_t* __restrict__ tet_face, const double* __restrict__ g0g1,
                           const double* __restrict__ Tm, const double* __restrict__ W,
                           const double* __restrict__ vprev, const double* __restrict__ ups,
                           const double* __restrict__ lam, const double* __restrict__ vbc,
                           double nu_dt, double* __restrict__ rhs, int64_t E, int64_t F, int G, int N) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * E * G * N) return;
    const int r = (int)(t % N);
    const int a = (int)((t / N) % G);
    const int64_t i = (t / ((int64_t)N * G)) % E;
    const int c = (int)(t / ((int64_t)N * G * E));
    const double* Mr = MI + ((int64_t)cls[i] * N + r) * N;
    double s = 0.0;
    for (int b = 0; b < G; ++b) {
        const double* xp = vprev + ((c * E + i) * G + b) * N;
        const double* xl = lam + ((c * E + i) * G + b) * N;
        double u1 = 0.0, u2 = 0.0;
        for (int m = 0; m < N; ++m) {
            u1 += Mr[m] * xp[m];
            u2 += Mr[m] * xl[m];
        }
        s += g0g1[a * G + b] * u1 - Tm[a * G + b] * u2;
    }
    s -= ups[((c * E + i) * G + a) * N + r];
    for (int f = 0; f < 4; ++f) {
        if (nbr[4 * i + f] >= 0) continue;
        const int64_t j = tet_face[4 * i + f];
        const double* Br = BB + (((int64_t)cls[i] * 4 + f) * N + r) * N;
        const double* xb = vbc + ((c * F + j) * G + a) * N;
        double u = 0.0;
        for (int m = 0; m < N; ++m) u += Br[m] * xb[m];
        s -= nu_dt * W[a] * u;
    }
    rhs[((c * E + i) * G + a) * N + r] = s;
}

// pressure right-hand side (eq. A2_mod): b_i = dt W_a sum_f sum_d QT_fd Fv_face[d][a]
__global__ void k_rhs_pressure(const double* __restrict__ QT, const int32_t* __restrict__ cls,
                               const int64_t* __restrict__ tet_face, const double* __restrict__ W,
                               const double* __restrict__ Fv, double dt, double* __restrict__ b,
                               int64_t E, int64_t F, int G, int N) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= E * G * N) return;
    const int r = (int)(t % N);
    const int a = (int)((t / N) % G);
    const int64_t i = t / ((int64_t)N * G);
    double s = 0.0;
    for (int f = 0; f < 4; ++f) {
        const int64_t j = tet_face[4 * i + f];
        for (int d = 0; d < 3; ++d) {
            const double* B = QT + ((((int64_t)cls[i] * 4 + f) * 3 + d) * N + r) * N;
            const double* x = Fv + ((d * F + j) * G + a) * N;
            for (int m = 0; m < N; ++m) s += B[m] * x[m];
        }
    }
    b[(i * G + a) * N + r] = dt * W[a] * s;
}

// eq. A3_mod: vhat = Fv - w on interior faces, the prescribed data on boundary faces
__global__ void k_update(const double* __restrict__ Fv, const double* __restrict__ w,
                         double* __restrict__ vhat, int64_t F, int64_t n_int, int G, int N) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * F * G * N) return;
    const int64_t j = (t / ((int64_t)N * G)) % F;
    vhat[t] = j < n_int ? Fv[t] - w[t] : Fv[t];
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] += a * x[t];
}

__global__ void k_copyd(const double* __restrict__ x, double* __restrict__ y, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = x[t];
}

// p <- (pi - (1 - theta) p) / theta: the end-of-step pressure of the theta-method
__global__ void k_theta_end(const double* __restrict__ pi, double* __restrict__ p, double theta, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (pi[i] - (1.0 - theta) * p[i]) / theta;
}

__global__ void k_zero(double* __restrict__ y, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = 0.0;
}

// Viscous operator (eq. A1_mod): y = (MI (x) T) x_i + nu dt sum_k (SV_k (x) W) x_nb(k)
__global__ void k_visc_apply(const double* __restrict__ SV, const double* __restrict__ MI,
                             const int32_t* __restrict__ cls, const int32_t* __restrict__ nbr,
                             const double* __restrict__ Tm, const double* __restrict__ W, double nu_dt,
                             const double* __restrict__ x, double* __restrict__ y, int64_t E, int G, int N) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * E * G * N) return;
    const int r = (int)(t % N);
    const int a = (int)((t / N) % G);
    const int64_t i = (t / ((int64_t)N * G)) % E;
    const int c = (int)(t / ((int64_t)N * G * E));
    const int64_t cbase = (int64_t)c * E;
    double s = 0.0;
    for (int k = 0; k < 5; ++k) {
        const int64_t nb = k == 0 ? i : (int64_t)nbr[4 * i + k - 1];
        if (nb < 0) continue;
        const double* B = SV + (((int64_t)cls[i] * 5 + k) * N + r) * N;
        const double* xk = x + ((cbase + nb) * G + a) * N;
        double u = 0.0;
        for (int m = 0; m < N; ++m) u += B[m] * xk[m];
        s += nu_dt * W[a] * u;
    }
    const double* Mr = MI + ((int64_t)cls[i] * N + r) * N;
    for (int b = 0; b < G; ++b) {
        const double* xb = x + ((cbase + i) * G + b) * N;
        double u = 0.0;
        for (int m = 0; m < N; ++m) u += Mr[m] * xb[m];
        s += Tm[a * G + b] * u;
    }
    y[t] = s;
}

// Viscous operator, fast form: one thread per (component, element, time node
// a) with the same class-uniform wavefronts as the pressure kernel (block
// columns through scalar loads, blocks stored column-major):
//   y_a = nu dt W_a sum_k SV_k x_k[a] + MI sum_b T_ab x_i[b].
template <int N, int G>
__global__ void __launch_bounds__(256) k_visc_tn(
    const double* __restrict__ SVt, const double* __restrict__ MIt, const int32_t* __restrict__ cls,
    const int32_t* __restrict__ nbr, const double* __restrict__ Tm, const double* __restrict__ W, double nu_dt,
    const double* __restrict__ x, double* __restrict__ y, int64_t E) {
    // the 3 G (component, time node) workgroups of one 256-element tile are
    // consecutive on one XCD (workgroups go round-robin over the 8 XCDs), so
    // a tile's blocks are re-read from cache while still resident
    const int64_t nbE = (E + 255) / 256;
    const int64_t j = blockIdx.x >> 3;
    const int v = (int)(j % (3 * G));
    const int64_t tile = (j / (3 * G)) * 8 + (blockIdx.x & 7);
    if (tile >= nbE) return;
    const int a = v % G;
    const int comp = v / G;
    const int64_t i = tile * 256 + threadIdx.x;
    const bool valid = i < E;
    const int64_t ii = valid ? i : E - 1;
    const int c = cls[ii];
    const int c0 = __builtin_amdgcn_readfirstlane(c);
    const bool uniform = __all(c == c0);
    const double* xc = x + (int64_t)comp * E * G * N;
    const double wa = nu_dt * W[a];
    double Ta[G];
#pragma unroll
    for (int b = 0; b < G; ++b) Ta[b] = Tm[a * G + b];
    double acc[N];
#pragma unroll
    for (int r = 0; r < N; ++r) acc[r] = 0.0;
    int nb[5];
    nb[0] = (int)ii;
#pragma unroll
    for (int f = 0; f < 4; ++f) nb[f + 1] = nbr[4 * ii + f];
    if (uniform) {
        const double* Bc = SVt + (int64_t)c0 * 5 * N * N;
        for (int k = 0; k < 5; ++k) {
            const int t = nb[k];
            if (__builtin_amdgcn_readfirstlane(t) < 0) continue;
            const double* xt = xc + ((int64_t)t * G + a) * N;
#pragma unroll
            for (int m = 0; m < N; ++m) {
                const double xp = wa * xt[m];
                const double* col = Bc + k * N * N + m * N;
#pragma unroll
                for (int r = 0; r < N; ++r) acc[r] += col[r] * xp;
            }
        }
        const double* Mc = MIt + (int64_t)c0 * N * N;
        const double* xi = xc + (int64_t)ii * G * N;
#pragma unroll
        for (int m = 0; m < N; ++m) {
            double xp = 0.0;
#pragma unroll
            for (int b = 0; b < G; ++b) xp += Ta[b] * xi[b * N + m];
            const double* col = Mc + m * N;
#pragma unroll
            for (int r = 0; r < N; ++r) acc[r] += col[r] * xp;
        }
    } else {
        const double* Bc = SVt + (int64_t)c * 5 * N * N;
        for (int k = 0; k < 5; ++k) {
            const int t = nb[k];
            if (t < 0) continue;
            const double* xt = xc + ((int64_t)t * G + a) * N;
            for (int m = 0; m < N; ++m) {
                const double xp = wa * xt[m];
                const double* col = Bc + k * N * N + m * N;
#pragma unroll
                for (int r = 0; r < N; ++r) acc[r] += col[r] * xp;
            }
        }
        const double* Mc = MIt + (int64_t)c * N * N;
        const double* xi = xc + (int64_t)ii * G * N;
        for (int m = 0; m < N; ++m) {
            double xp = 0.0;
#pragma unroll
            for (int b = 0; b < G; ++b) xp += Ta[b] * xi[b * N + m];
            const double* col = Mc + m * N;
#pragma unroll
            for (int r = 0; r < N; ++r) acc[r] += col[r] * xp;
        }
    }
    if (valid) {
        double* yi = y + (int64_t)comp * E * G * N + (i * G + a) * N;
#pragma unroll
        for (int r = 0; r < N; ++r) yi[r] = acc[r];
    }
}

// The same operator for meshes whose wavefronts mix classes (classes holding
// fewer elements than a wavefront): one thread per (element, time node a)
// applies its element's blocks to all three components, so each block entry
// is read once for the three (per component the same sums in the same order).
template <int N, int G>
__global__ void __launch_bounds__(256) k_visc_tn3(
    const double* __restrict__ SVt, const double* __restrict__ MIt, const int32_t* __restrict__ cls,
    const int32_t* __restrict__ nbr, const double* __restrict__ Tm, const double* __restrict__ W, double nu_dt,
    const double* __restrict__ x, double* __restrict__ y, int64_t E) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= E * G) return;
    const int a = (int)(t % G);
    const int64_t i = t / G;
    const int c = cls[i];
    const int64_t cs = E * G * N;                 // component stride
    const double wa = nu_dt * W[a];
    double Ta[G];
#pragma unroll
    for (int b = 0; b < G; ++b) Ta[b] = Tm[a * G + b];
    double acc[3][N];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
        for (int r = 0; r < N; ++r) acc[cc][r] = 0.0;
    int nb[5];
    nb[0] = (int)i;
#pragma unroll
    for (int f = 0; f < 4; ++f) nb[f + 1] = nbr[4 * i + f];
    const double* Bc = SVt + (int64_t)c * 5 * N * N;
    for (int k = 0; k < 5; ++k) {
        const int tk = nb[k];
        if (tk < 0) continue;
        const double* xt = x + ((int64_t)tk * G + a) * N;
        for (int m = 0; m < N; ++m) {
            const double x0 = wa * xt[m], x1 = wa * xt[cs + m], x2 = wa * xt[2 * cs + m];
            const double* col = Bc + k * N * N + m * N;
#pragma unroll
            for (int r = 0; r < N; ++r) {
                const double bv = col[r];
                acc[0][r] += bv * x0;
                acc[1][r] += bv * x1;
                acc[2][r] += bv * x2;
            }
        }
    }
    const double* Mc = MIt + (int64_t)c * N * N;
    const double* xi = x + i * G * N;
    for (int m = 0; m < N; ++m) {
        double xp[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < G; ++b)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) xp[cc] += Ta[b] * xi[cc * cs + b * N + m];
        const double* col = Mc + m * N;
#pragma unroll
        for (int r = 0; r < N; ++r) {
            const double bv = col[r];
            acc[0][r] += bv * xp[0];
            acc[1][r] += bv * xp[1];
            acc[2][r] += bv * xp[2];
        }
    }
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
        double* yi = y + cc * cs + (i * G + a) * N;
#pragma unroll
        for (int r = 0; r < N; ++r) yi[r] = acc[cc][r];
    }
}

// y_i = D_i^-1 x_i for the viscous diagonal blocks (per component), DV
// column-major so that the threads of one element read consecutive values.
__global__ void k_blockdiag(const double* __restrict__ DV, const int32_t* __restrict__ cls,
                            const double* __restrict__ x, double* __restrict__ y, int64_t E, int NG) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * E * NG) return;
    const int row = (int)(t % NG);
    const int64_t ce = t / NG;                 // comp * E + element
    const int64_t i = ce % E;
    const double* D = DV + (int64_t)cls[i] * NG * NG + row;
    const double* xi = x + ce * NG;
    double s = 0.0;
    for (int col = 0; col < NG; ++col) s += D[(int64_t)col * NG] * xi[col];
    y[t] = s;
}

// Space-time DG convection with the Rusanov flux (eq. convdg), one block of
// 64 threads per element.  For each time point of the rule: the lanes first
// evaluate the velocity at the volume points (flux tensor pulled back by the
// element Jacobian) and at the four faces' points (Rusanov flux, own trace
// against the neighbour's trace or the boundary dual velocity) into LDS; then
// each lane accumulates the test-function sums for its outputs (c, k).
template <int N, int G>
__global__ void __launch_bounds__(64) k_convection(
    const double* __restrict__ vbar, const double* __restrict__ vbc, const int32_t* __restrict__ cls,
    const int32_t* __restrict__ nbr, const int64_t* __restrict__ tet_face, const double* __restrict__ cJinv,
    const double* __restrict__ cdet, const double* __restrict__ cnrm, const double* __restrict__ PHf,
    const double* __restrict__ PHn, const double* __restrict__ FW, const double* __restrict__ PHv,
    const double* __restrict__ dPHv, const double* __restrict__ wv, const double* __restrict__ tw,
    const double* __restrict__ gq, int nqv, int nqf, int qt, double dt, double* __restrict__ ups,
    int64_t E, int64_t F) {
    extern __shared__ double sh[];
    double* vol = sh;                      // [nqv][3][3]  w |J| (J^-T) (v v^T)
    double* fac = sh + (size_t)nqv * 9;    // [4][nqf][3]  w area * flux
    const int64_t i = blockIdx.x;
    const int lane = threadIdx.x;
    const int c = cls[i];
    const double* Ji = cJinv + (int64_t)c * 9;
    const double det = cdet[c];
    constexpr int NOUT = 3 * N;
    constexpr int NP = (NOUT + 63) / 64;   // outputs per lane
    double acc[NP][G];
#pragma unroll
    for (int u = 0; u < NP; ++u)
#pragma unroll
        for (int a = 0; a < G; ++a) acc[u][a] = 0.0;
    for (int t = 0; t < qt; ++t) {
        double gt[G];
#pragma unroll
        for (int b = 0; b < G; ++b) gt[b] = gq[t * G + b];
        const double wt = tw[t];
        // ---- phase A: volume points
        for (int q = lane; q < nqv; q += 64) {
            double v[3] = {0, 0, 0};
            const double* ph = PHv + (int64_t)q * N;
            for (int cc = 0; cc < 3; ++cc)
                for (int b = 0; b < G; ++b) {
                    const double* x = vbar + ((cc * E + i) * G + b) * N;
                    double s = 0.0;
                    for (int n = 0; n < N; ++n) s += ph[n] * x[n];
                    v[cc] += gt[b] * s;
                }
            const double w = wt * wv[q] * det;
            for (int cc = 0; cc < 3; ++cc)
                for (int e = 0; e < 3; ++e) {
                    // sum_d Jinv[e][d] F_cd, F_cd = v_c v_d
                    double s = Ji[e * 3 + 0] * v[0] + Ji[e * 3 + 1] * v[1] + Ji[e * 3 + 2] * v[2];
                    vol[(q * 3 + cc) * 3 + e] = w * v[cc] * s;
                }
        }
        // ---- phase A: face points
        for (int qq = lane; qq < 4 * nqf; qq += 64) {
            const int f = qq / nqf, q = qq - f * nqf;
            const int64_t off = ((int64_t)c * 4 + f) * nqf + q;
            const double* ph = PHf + off * N;
            const double* pn = PHn + off * N;
            const int64_t k = nbr[4 * i + f];
            double vm[3] = {0, 0, 0}, vp[3] = {0, 0, 0};
            for (int cc = 0; cc < 3; ++cc)
                for (int b = 0; b < G; ++b) {
                    const double* xm = vbar + ((cc * E + i) * G + b) * N;
                    const double* xp = k >= 0 ? vbar + ((cc * E + k) * G + b) * N
                                              : vbc + ((cc * F + tet_face[4 * i + f]) * G + b) * N;
                    double sm = 0.0, sp = 0.0;
                    for (int n = 0; n < N; ++n) {
                        sm += ph[n] * xm[n];
                        sp += pn[n] * xp[n];
                    }
                    vm[cc] += gt[b] * sm;
                    vp[cc] += gt[b] * sp;
                }
            const double* nr = cnrm + (int64_t)c * 12 + f * 3;
            const double unm = vm[0] * nr[0] + vm[1] * nr[1] + vm[2] * nr[2];
            const double unp = vp[0] * nr[0] + vp[1] * nr[1] + vp[2] * nr[2];
            const double am = sqrt(vm[0] * vm[0] + vm[1] * vm[1] + vm[2] * vm[2]);
            const double ap = sqrt(vp[0] * vp[0] + vp[1] * vp[1] + vp[2] * vp[2]);
            const double smax = 2.0 * (am > ap ? am : ap);
            const double w = wt * FW[off];
            for (int cc = 0; cc < 3; ++cc)
                fac[qq * 3 + cc] = w * (0.5 * (vp[cc] * unp + vm[cc] * unm) - 0.5 * smax * (vp[cc] - vm[cc]));
        }
        __syncthreads();
        // ---- phase B: test-function sums for outputs (cc, kk)
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            const int o = lane + 64 * u;
            if (o >= NOUT) continue;
            const int cc = o / N, kk = o - cc * N;
            double s = 0.0;
            for (int q = 0; q < nqv; ++q) {
                const double* dp = dPHv + ((int64_t)q * N + kk) * 3;
                const double* vq = vol + (q * 3 + cc) * 3;
                s -= dp[0] * vq[0] + dp[1] * vq[1] + dp[2] * vq[2];
            }
            for (int f = 0; f < 4; ++f)
                for (int q = 0; q < nqf; ++q) {
                    const int64_t off = ((int64_t)c * 4 + f) * nqf + q;
                    s += PHf[off * N + kk] * fac[(f * nqf + q) * 3 + cc];
                }
#pragma unroll
            for (int a = 0; a < G; ++a) acc[u][a] += gt[a] * s;
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < NP; ++u) {
        const int o = lane + 64 * u;
        if (o >= NOUT) continue;
        const int cc = o / N, kk = o - cc * N;
#pragma unroll
        for (int a = 0; a < G; ++a) ups[((cc * E + i) * G + a) * N + kk] = dt * acc[u][a];
    }
}

template <int N, int G>
hipError_t launch_conv_ng(const stdg_mesh* m, const double* vbar, const double* vbc, double* ups, hipStream_t s) {
    const PicardTables& t = m->pt;
    const PicardDevice& d = m->pd;
    const size_t lds = ((size_t)t.nqv * 9 + (size_t)4 * t.nqf * 3) * sizeof(double);
    hipLaunchKernelGGL((k_convection<N, G>), dim3((unsigned)m->E), dim3(64), lds, s, vbar, vbc, m->d.cls,
                       m->d.nbr, d.tet_face, d.cJinv, d.cdet, d.cnrm, d.PHf, d.PHn, d.FW, d.PHv, d.dPHv, d.wv,
                       d.tw, d.gq, t.nqv, t.nqf, t.qt, m->cfg.dt, ups, m->E, (int64_t)m->faces.size());
    return hipGetLastError();
}

hipError_t launch_convection(const stdg_mesh* m, const double* vbar, const double* vbc, double* ups,
                             hipStream_t s) {
    {
        const hipError_t e = fast_convection(m, vbar, vbc, ups, s);
        if (e != hipErrorNotSupported) return e;
    }
#define STDG_CV(n, g) \
    if (m->N == n && m->G == g) return launch_conv_ng<n, g>(m, vbar, vbc, ups, s);
    STDG_CV(4, 1) STDG_CV(4, 2) STDG_CV(4, 3) STDG_CV(4, 4) STDG_CV(4, 5)
    STDG_CV(10, 1) STDG_CV(10, 2) STDG_CV(10, 3) STDG_CV(10, 4) STDG_CV(10, 5)
    STDG_CV(20, 1) STDG_CV(20, 2) STDG_CV(20, 3) STDG_CV(20, 4) STDG_CV(20, 5)
    STDG_CV(35, 1) STDG_CV(35, 2) STDG_CV(35, 3) STDG_CV(35, 4) STDG_CV(35, 5)
    STDG_CV(56, 1) STDG_CV(56, 2) STDG_CV(56, 3) STDG_CV(56, 4) STDG_CV(56, 5)
    STDG_CV(84, 1) STDG_CV(84, 2) STDG_CV(84, 3) STDG_CV(84, 4) STDG_CV(84, 5)
#undef STDG_CV
    return hipErrorInvalidValue;
}

template <typename T>
int upload(T*& dst, const std::vector<T>& src) {
    if (src.empty()) { dst = nullptr; return STDG_OK; }
    STDG_HIP(hipMalloc(&dst, src.size() * sizeof(T)));
    STDG_HIP(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return STDG_OK;
}

}  // namespace

// Block-row steps: the register kernels of picard_fast.hip for p <= 4, the
// thread-per-coefficient kernels above otherwise.
hipError_t run_goback(const stdg_mesh* m, const double* vbar, const double* vbdry, double* out, int64_t f0,
                      int64_t f1, hipStream_t s) {
    if (fast_rows_supported(m)) return fast_goback(m, vbar, vbdry, out, f0, f1, s);
    const PicardDevice& d = m->pd;
    const int64_t n = 3 * (f1 - f0) * m->G * m->N;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_goback, dim3(nblk(n)), dim3(256), 0, s, d.GB, m->d.cls, d.fl, d.flf, d.fr, d.frf, vbar, vbdry,
                       out, f0, f1, (int64_t)m->faces.size(), m->E, m->G, m->N);
    return hipGetLastError();
}

hipError_t run_average(const stdg_mesh* m, const double* vhat, double* vbar, hipStream_t s) {
    if (fast_rows_supported(m)) return fast_average(m, vhat, vbar, s);
    const int64_t n = 3 * m->E * m->Nst;
    hipLaunchKernelGGL(k_average, dim3(nblk(n)), dim3(256), 0, s, m->pd.A, m->d.cls, m->pd.tet_face, vhat, vbar, m->E,
                       (int64_t)m->faces.size(), m->G, m->N);
    return hipGetLastError();
}

hipError_t run_dualgrad(const stdg_mesh* m, const double* p, double dt, double* w, hipStream_t s) {
    if (fast_rows_supported(m)) return fast_dualgrad(m, p, dt, w, s);
    const PicardDevice& d = m->pd;
    const int64_t F = (int64_t)m->faces.size();
    hipLaunchKernelGGL(k_dualgrad, dim3(nblk(3 * F * m->Nst)), dim3(256), 0, s, d.US, d.UN, m->d.cls, d.fl, d.flf, d.fr,
                       d.TW, p, dt, w, F, m->G, m->N);
    return hipGetLastError();
}

hipError_t run_rhs_pressure(const stdg_mesh* m, const double* Fv, double dt, double* b, hipStream_t s) {
    if (fast_rows_supported(m)) return fast_rhs_pressure(m, Fv, dt, b, s);
    hipLaunchKernelGGL(k_rhs_pressure, dim3(nblk(m->E * m->Nst)), dim3(256), 0, s, m->pd.QT, m->d.cls, m->pd.tet_face,
                       m->pd.W, Fv, dt, b, m->E, (int64_t)m->faces.size(), m->G, m->N);
    return hipGetLastError();
}

hipError_t run_visc_rhs(const stdg_mesh* m, const double* vprev, const double* ups, const double* lam,
                        const double* vbc, double* rhs, hipStream_t s) {
    if (fast_rows_supported(m)) return fast_visc_rhs(m, vprev, ups, lam, vbc, rhs, s);
    const PicardDevice& d = m->pd;
    hipLaunchKernelGGL(k_visc_rhs, dim3(nblk(3 * m->E * m->Nst)), dim3(256), 0, s, d.MIT, d.BB, m->d.cls, m->d.nbr,
                       d.tet_face, d.g0g1, d.Tm, d.W, vprev, ups, lam, vbc, m->cfg.nu * m->cfg.dt, rhs, m->E,
                       (int64_t)m->faces.size(), m->G, m->N);
    return hipGetLastError();
}

template <int N, int G>
static hipError_t launch_visc_ng(const stdg_mesh* m, const double* x, double* y, hipStream_t s) {
    const PicardDevice& d = m->pd;
    if ((int64_t)m->n_classes * 64 > m->E) {
        const int64_t blocks = (m->E * G + 255) / 256;
        hipLaunchKernelGGL((k_visc_tn3<N, G>), dim3((unsigned)blocks), dim3(256), 0, s, d.SVt, d.MIt, m->d.cls,
                           m->d.nbr, d.Tm, d.W, m->cfg.nu * m->cfg.dt, x, y, m->E);
        return hipGetLastError();
    }
    const int64_t blocks = ((m->E + 255) / 256 + 7) / 8 * 8 * G * 3;
    hipLaunchKernelGGL((k_visc_tn<N, G>), dim3((unsigned)blocks), dim3(256), 0, s, d.SVt, d.MIt, m->d.cls,
                       m->d.nbr, d.Tm, d.W, m->cfg.nu * m->cfg.dt, x, y, m->E);
    return hipGetLastError();
}

hipError_t launch_visc_apply(const stdg_mesh* m, const double* x, double* y, hipStream_t s) {
#define STDG_VN(n, g) \
    if (m->N == n && m->G == g) return launch_visc_ng<n, g>(m, x, y, s);
    STDG_VN(4, 1) STDG_VN(4, 2) STDG_VN(4, 3) STDG_VN(4, 4) STDG_VN(4, 5)
    STDG_VN(10, 1) STDG_VN(10, 2) STDG_VN(10, 3) STDG_VN(10, 4) STDG_VN(10, 5)
    STDG_VN(20, 1) STDG_VN(20, 2) STDG_VN(20, 3) STDG_VN(20, 4) STDG_VN(20, 5)
    STDG_VN(35, 1) STDG_VN(35, 2) STDG_VN(35, 3) STDG_VN(35, 4) STDG_VN(35, 5)
#undef STDG_VN
    const PicardDevice& d = m->pd;
    const int64_t n = 3 * m->E * m->Nst;
    hipLaunchKernelGGL(k_visc_apply, dim3(nblk(n)), dim3(256), 0, s, d.SVT, d.MIT, m->d.cls, m->d.nbr, d.Tm, d.W,
                       m->cfg.nu * m->cfg.dt, x, y, m->E, m->G, m->N);
    return hipGetLastError();
}

hipError_t launch_visc_precond(const stdg_mesh* m, const double* x, double* y, hipStream_t s) {
    if (fast_blockdiag(m, x, y, s) == hipSuccess) return hipSuccess;
    const int NG = m->Nst;
    const int64_t n = 3 * m->E * NG;
    hipLaunchKernelGGL(k_blockdiag, dim3(nblk(n)), dim3(256), 0, s, m->pd.DV, m->d.cls, x, y, m->E, NG);
    return hipGetLastError();
}

int upload_picard_tables(stdg_mesh* m) {
    PicardTables& t = m->pt;
    PicardDevice& d = m->pd;
    int e = STDG_OK;
    for (auto pr : std::initializer_list<std::pair<double**, std::vector<double>*>>{
             {&d.A, &t.A}, {&d.GB, &t.GB}, {&d.QT, &t.QT}, {&d.US, &t.US}, {&d.UN, &t.UN}, {&d.BB, &t.BB},
             {&d.SVT, &t.SV}, {&d.MIT, &t.MI}, {&d.cJinv, &t.cJinv}, {&d.cdet, &t.cdet}, {&d.cnrm, &t.cnrm},
             {&d.PHf, &t.PHf}, {&d.PHn, &t.PHn}, {&d.FW, &t.FW}, {&d.PHv, &t.PHv}, {&d.dPHv, &t.dPHv},
             {&d.wv, &t.wv}, {&d.tq, &t.tq}, {&d.tw, &t.tw}, {&d.gq, &t.gq}, {&d.Tm, &t.Tm}, {&d.TW, &t.TW},
             {&d.W, &t.W}, {&d.g0g1, &t.g0g1}, {&d.g1, &t.g1}})
        if ((e = upload(*pr.first, *pr.second))) return e;
    {
        const int N = m->N;
        const size_t NN = (size_t)N * N;
        std::vector<double> svt(t.SV.size()), mit(t.MI.size());
        for (size_t blk = 0; blk < t.SV.size() / NN; ++blk)
            for (int r = 0; r < N; ++r)
                for (int c = 0; c < N; ++c) svt[blk * NN + (size_t)c * N + r] = t.SV[blk * NN + (size_t)r * N + c];
        for (size_t blk = 0; blk < t.MI.size() / NN; ++blk)
            for (int r = 0; r < N; ++r)
                for (int c = 0; c < N; ++c) mit[blk * NN + (size_t)c * N + r] = t.MI[blk * NN + (size_t)r * N + c];
        if ((e = upload(d.SVt, svt)) || (e = upload(d.MIt, mit)) || (e = upload(d.DV, t.DV))) return e;
        auto transposed = [&](const std::vector<double>& v) {
            std::vector<double> o(v.size());
            for (size_t blk = 0; blk < v.size() / NN; ++blk)
                for (int r = 0; r < N; ++r)
                    for (int c = 0; c < N; ++c) o[blk * NN + (size_t)c * N + r] = v[blk * NN + (size_t)r * N + c];
            return o;
        };
        if ((e = upload(d.At, transposed(t.A))) || (e = upload(d.GBt, transposed(t.GB))) ||
            (e = upload(d.QTt, transposed(t.QT))) || (e = upload(d.USt, transposed(t.US))) ||
            (e = upload(d.UNt, transposed(t.UN))) || (e = upload(d.BBt, transposed(t.BB))))
            return e;
    }
    const int64_t F = (int64_t)m->faces.size();
    std::vector<int64_t> fl(F), fr(F);
    std::vector<int32_t> flf(F), frf(F);
    for (int64_t j = 0; j < F; ++j) {
        fl[j] = m->faces[j].left; fr[j] = m->faces[j].right;
        flf[j] = m->faces[j].lf; frf[j] = m->faces[j].rf;
    }
    if ((e = upload(d.fl, fl)) || (e = upload(d.fr, fr)) || (e = upload(d.flf, flf)) || (e = upload(d.frf, frf)) ||
        (e = upload(d.tet_face, m->tet_face)))
        return e;
    return STDG_OK;
}

void free_picard(stdg_mesh* m) {
    PicardDevice& d = m->pd;
    for (void* p : {(void*)d.A, (void*)d.GB, (void*)d.QT, (void*)d.US, (void*)d.UN, (void*)d.BB, (void*)d.SVT,
                    (void*)d.MIT, (void*)d.cJinv, (void*)d.cdet, (void*)d.cnrm, (void*)d.PHf, (void*)d.PHn,
                    (void*)d.FW, (void*)d.PHv, (void*)d.dPHv, (void*)d.wv, (void*)d.tq, (void*)d.tw, (void*)d.gq,
                    (void*)d.Tm, (void*)d.TW, (void*)d.W, (void*)d.g0g1, (void*)d.g1, (void*)d.tet_face,
                    (void*)d.fl, (void*)d.fr, (void*)d.flf, (void*)d.frf, (void*)d.work, (void*)d.DV,
                    (void*)d.SVt, (void*)d.MIt, (void*)d.At, (void*)d.GBt, (void*)d.QTt, (void*)d.USt,
                    (void*)d.UNt, (void*)d.BBt, (void*)d.conv_tmp})
        if (p) (void)hipFree(p);
    d = PicardDevice();
}

}  // namespace stdg

using namespace stdg;

extern "C" void stdg_step_opts_default(stdg_step_opts* o) {
    if (!o) return;
    o->n_picard = 0;
    o->pressure_guess = STDG_GUESS_ZERO;
    stdg_solve_opts_default(&o->pressure);
    stdg_solve_opts_default(&o->viscous);
    o->viscous.rtol = 1e-12;
    o->krylov_guess = STDG_KRYLOV_ZERO;
    o->model = nullptr;
    o->hist = nullptr;
    o->rec_b = nullptr;
    o->rec_x = nullptr;
    o->theta = 1.0;
}

static const char* kCurvedPicard =
    "curved elements: only the pressure system is built, the Picard-step tables need affine elements";

extern "C" int stdg_dual_from_main(const stdg_mesh* m, const double* vbar, double* vhat, void* stream) {
    if (!m || !vbar || !vhat) { set_error("null argument"); return STDG_ERR_ARG; }
    if (m->curved) { set_error(kCurvedPicard); return STDG_ERR_ARG; }
    if (!m->d.blocks || !m->pd.GB) { set_error("mesh was built host-only"); return STDG_ERR_ARG; }
    const int64_t F = (int64_t)m->faces.size();
    const int64_t n = 3 * F * m->Nst;
    (void)n;
    STDG_HIP(run_goback(m, vbar, vbar, vhat, 0, F, (hipStream_t)stream));
    return STDG_OK;
}

extern "C" int stdg_main_from_dual(const stdg_mesh* m, const double* vhat, double* vbar, void* stream) {
    if (!m || !vbar || !vhat) { set_error("null argument"); return STDG_ERR_ARG; }
    if (m->curved) { set_error(kCurvedPicard); return STDG_ERR_ARG; }
    if (!m->d.blocks || !m->pd.A) { set_error("mesh was built host-only"); return STDG_ERR_ARG; }
    const int64_t n = 3 * m->E * m->Nst;
    (void)n;
    STDG_HIP(run_average(m, vhat, vbar, (hipStream_t)stream));
    return STDG_OK;
}

extern "C" int stdg_divergence(const stdg_mesh* m, const double* vhat, double* div, void* stream) {
    if (!m || !vhat || !div) { set_error("null argument"); return STDG_ERR_ARG; }
    if (m->curved) { set_error(kCurvedPicard); return STDG_ERR_ARG; }
    if (!m->d.blocks || !m->pd.QT) { set_error("mesh was built host-only"); return STDG_ERR_ARG; }
    // sum_j D_ij vhat_j = -sum_j Q_ij^T vhat_j
    const int64_t n = m->E * m->Nst;
    (void)n;
    STDG_HIP(run_rhs_pressure(m, vhat, -m->cfg.dt, div, (hipStream_t)stream));
    return STDG_OK;
}

extern "C" int stdg_picard_step(const stdg_mesh* cm, double* vhat, double* vbar, double* p, const double* g_nodal,
                                const stdg_step_opts* opts, stdg_step_report* rep, void* stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (!cm || !vhat || !vbar || !p || !opts) { set_error("null argument"); return STDG_ERR_ARG; }
    stdg_mesh* m = const_cast<stdg_mesh*>(cm);
    if (m->curved) { set_error(kCurvedPicard); return STDG_ERR_ARG; }
    if (!m->d.blocks || !m->pd.A) { set_error("mesh was built host-only"); return STDG_ERR_ARG; }
    if (m->G > 5) { set_error("the Picard step is implemented for p_gamma <= 4"); return STDG_ERR_ARG; }
    const double theta = opts->theta;
    if (!(theta >= 0.5 && theta <= 1.0)) { set_error("theta must lie in [1/2, 1]"); return STDG_ERR_ARG; }
    if (theta != 1.0 && m->G != 1) { set_error("the theta-method is defined for p_gamma = 0"); return STDG_ERR_ARG; }
    const int64_t F = (int64_t)m->faces.size(), E = m->E, NI = m->n_interior;
    if (F > NI && !g_nodal) { set_error("Dirichlet data required on a mesh with boundary faces"); return STDG_ERR_ARG; }
    const int npic = opts->n_picard > 0 ? opts->n_picard : m->G;
    if (opts->pressure_guess != STDG_GUESS_ZERO && opts->pressure_guess != STDG_GUESS_PREVIOUS) {
        set_error("unknown pressure guess");
        return STDG_ERR_ARG;
    }
    const int kg = opts->krylov_guess;
    if (kg != STDG_KRYLOV_ZERO && kg != STDG_KRYLOV_PREVIOUS && kg != STDG_KRYLOV_EXTRAPOLATE &&
        kg != STDG_KRYLOV_LEARNED) {
        set_error("unknown Krylov guess");
        return STDG_ERR_ARG;
    }
    if (kg != STDG_KRYLOV_ZERO && !opts->hist) { set_error("this Krylov guess needs hist"); return STDG_ERR_ARG; }
    if (kg == STDG_KRYLOV_LEARNED && !opts->model) { set_error("the learned guess needs a model"); return STDG_ERR_ARG; }
    hipStream_t s = (hipStream_t)stream;
    const int G = m->G, N = m->N;
    const int64_t nD = 3 * F * G * N, nM = 3 * E * G * N, nP = E * G * N;
    const int mres = std::max(1, opts->viscous.restart);
    // workspace: 4 dual + 6 main + 3 pressure vectors + viscous Krylov (mres + 6) main
    const size_t need = 4 * nD + 6 * nM + 3 * nP + (size_t)(mres + 6) * nM +
                        (kg == STDG_KRYLOV_LEARNED ? 4 * nP : 0);   // learned-start vectors
    const bool zero_base = opts->pressure_guess == STDG_GUESS_ZERO;
    PicardDevice& d = m->pd;
    if (d.work_len < need) {
        if (d.work) STDG_HIP(hipFree(d.work));
        d.work = nullptr;
        STDG_HIP(hipMalloc(&d.work, need * sizeof(double)));
        d.work_len = need;
    }
    double* vk = d.work;            // dual velocity of the current iterate
    double* Fv = vk + nD;
    double* wg = Fv + nD;           // dual-grid pressure gradient
    double* vbc = wg + nD;          // prescribed boundary dual velocity
    double* vbk = vbc + nD;         // averaged velocity
    double* lam = vbk + nM;
    double* ups = lam + nM;
    double* rhs = ups + nM;
    double* vhalf = rhs + nM;
    double* vprev = vhalf + nM;
    double* pk = vprev + nM;
    double* bp = pk + nP;
    double* dp = bp + nP;
    double* kw = dp + nP;           // viscous Krylov work
    double* ls = kw + (size_t)(mres + 6) * nM;   // learned guess: least-squares vectors
    // history per Picard iteration k (two previous steps): slot 2k holds the
    // last step's value, slot 2k + 1 the one before; the value is the new
    // pressure p^{n+1,1} for k = 0 and the correction for k >= 1
    auto hist_at = [&](int k, int which) -> double* {
        return opts->hist ? opts->hist + (size_t)(2 * k + which) * nP : nullptr;
    };
    // learned start of the first solve: x0 = x_e + g d with the extrapolation
    // x_e = 2 h0 - h1, the network correction d, and g minimising
    // ||b + S base - S x0|| (g = 0 gives x_e back); returned as x0 - base
    auto learned_guess = [&](const double* h0, const double* h1, const double* d, double* out,
                             double& g) -> int {
        double* xe = ls;
        double* rb = ls + nP;
        double* Sd = ls + 2 * nP;
        hipLaunchKernelGGL(k_copyd, dim3(nblk(nP)), dim3(256), 0, s, h0, xe, nP);
        hipLaunchKernelGGL(k_axpy, dim3(nblk(nP)), dim3(256), 0, s, xe, h0, 1.0, nP);
        hipLaunchKernelGGL(k_axpy, dim3(nblk(nP)), dim3(256), 0, s, xe, h1, -1.0, nP);
        if (!zero_base) hipLaunchKernelGGL(k_axpy, dim3(nblk(nP)), dim3(256), 0, s, xe, pk, -1.0, nP);
        STDG_HIP(hipGetLastError());
        STDG_HIP(launch_apply_f64(m, xe, rb, s));                     // S (x_e - base)
        hipLaunchKernelGGL(k_axpy, dim3(nblk(nP)), dim3(256), 0, s, rb, bp, -1.0, nP);   // S (x_e - base) - b
        STDG_HIP(launch_apply_f64(m, d, Sd, s));
        STDG_HIP(hipGetLastError());
        const double* da[2] = {Sd, Sd};
        const double* db[2] = {Sd, rb};
        double v[2];
        if (int e2 = device_dots(m, 2, da, db, nP, s, v)) return e2;
        g = v[0] > 0.0 ? -v[1] / v[0] : 0.0;
        hipLaunchKernelGGL(k_copyd, dim3(nblk(nP)), dim3(256), 0, s, xe, out, nP);
        if (g != 0.0) hipLaunchKernelGGL(k_axpy, dim3(nblk(nP)), dim3(256), 0, s, out, d, g, nP);
        STDG_HIP(hipGetLastError());
        return STDG_OK;
    };
    const double dt = m->cfg.dt;
    // step 0
    hipLaunchKernelGGL(k_copyd, dim3(nblk(nM)), dim3(256), 0, s, vbar, vprev, nM);
    hipLaunchKernelGGL(k_time_end, dim3(nblk(3 * F * N)), dim3(256), 0, s, vhat, vk, d.g1, 3 * F, G, N);
    hipLaunchKernelGGL(k_zero, dim3(nblk(nD)), dim3(256), 0, s, vbc, nD);
    if (F > NI) {
        STDG_HIP(run_goback(m, g_nodal, g_nodal, vbc, NI, F, s));
        // boundary part of the iterate = prescribed data
        for (int c = 0; c < 3; ++c)
            hipLaunchKernelGGL(k_copyd, dim3(nblk((F - NI) * G * N)), dim3(256), 0, s,
                               vbc + ((int64_t)c * F + NI) * G * N, vk + ((int64_t)c * F + NI) * G * N,
                               (F - NI) * G * N);
    }
    // pk holds the pressure that the momentum equation carries: p^{n+1,k}, or
    // for the theta-method pi = theta p^{n+1,k} + (1 - theta) p^n, which makes
    // every later stage the theta = 1 step in pi (corrections of pi are theta
    // times those of p^{n+1}, with the same anchor)
    if (opts->pressure_guess == STDG_GUESS_PREVIOUS) {
        hipLaunchKernelGGL(k_copyd, dim3(nblk(nP)), dim3(256), 0, s, p, pk, nP);
    } else {
        hipLaunchKernelGGL(k_zero, dim3(nblk(nP)), dim3(256), 0, s, pk, nP);
        if (theta != 1.0) hipLaunchKernelGGL(k_axpy, dim3(nblk(nP)), dim3(256), 0, s, pk, p, 1.0 - theta, nP);
    }
    STDG_HIP(hipGetLastError());
    int piters = 0, viters = 0, papplies = 0, first_iters = 0;
    double guess_w = 0.0;
    double fused_us_sum = 0.0, fused_w = 0.0;
    double pres = 0.0, vres = 0.0, psec = 0.0, vsec = 0.0, first_sec = 0.0, first_res0 = 0.0;
    int status = STDG_OK;   // STDG_NOT_CONVERGED once a solve stops at its limit
    for (int k = 0; k < npic; ++k) {
        // step 1
        if (int e = stdg_main_from_dual(m, vk, vbk, s)) return e;
        STDG_HIP(run_dualgrad(m, pk, dt, wg, s));
        STDG_HIP(run_average(m, wg, lam, s));
        // step 2
        CKP(launch_convection(m, vbk, vbc, ups, s));
        // step 3
        STDG_HIP(run_visc_rhs(m, vprev, ups, lam, vbc, rhs, s));
        hipLaunchKernelGGL(k_copyd, dim3(nblk(nM)), dim3(256), 0, s, vbk, vhalf, nM);
        STDG_HIP(hipGetLastError());
        int vit = 0;
        double vrel = 0.0;
        STDG_HIP(hipStreamSynchronize(s));
        auto tv0 = std::chrono::steady_clock::now();
        int e = viscous_solve(m, rhs, vhalf, opts->viscous, kw, s, vit, vrel);
        if (e < 0) return e;
        if (e == STDG_NOT_CONVERGED) status = STDG_NOT_CONVERGED;
        STDG_HIP(hipStreamSynchronize(s));
        vsec += std::chrono::duration<double>(std::chrono::steady_clock::now() - tv0).count();
        viters += vit;
        vres = std::max(vres, vrel);
        // step 4
        STDG_HIP(run_goback(m, vhalf, vhalf, Fv, 0, NI, s));
        for (int c = 0; c < 3 && F > NI; ++c)
            hipLaunchKernelGGL(k_copyd, dim3(nblk((F - NI) * G * N)), dim3(256), 0, s,
                               vbc + ((int64_t)c * F + NI) * G * N, Fv + ((int64_t)c * F + NI) * G * N,
                               (F - NI) * G * N);
        // step 5
        STDG_HIP(run_rhs_pressure(m, Fv, dt, bp, s));
        STDG_HIP(hipStreamSynchronize(s));
        const auto tg0 = std::chrono::steady_clock::now();
        if (k == 0 && opts->rec_b)
            hipLaunchKernelGGL(k_copyd, dim3(nblk(nP)), dim3(256), 0, s, bp, opts->rec_b, nP);
        // Krylov start of solve k from that solve's history (k = 0: the new
        // pressure p^{n+1,1}, whose unknown is its correction to p^{n+1,0})
        double* h0 = hist_at(k, 0);
        double* h1 = hist_at(k, 1);
        const double* base = (k == 0 && !zero_base) ? pk : nullptr;
        if (kg == STDG_KRYLOV_LEARNED && k == 0) {
            double* dd = ls + 3 * nP;
            if (int e2 = model_predict(opts->model, m, h0, h1, bp, dd, s, true)) return e2;
            if (int e2 = learned_guess(h0, h1, dd, dp, guess_w)) return e2;
        } else if (kg == STDG_KRYLOV_PREVIOUS) {
            hipLaunchKernelGGL(k_copyd, dim3(nblk(nP)), dim3(256), 0, s, h0, dp, nP);
            if (base) hipLaunchKernelGGL(k_axpy, dim3(nblk(nP)), dim3(256), 0, s, dp, base, -1.0, nP);
        } else if (kg == STDG_KRYLOV_EXTRAPOLATE || kg == STDG_KRYLOV_LEARNED) {
            hipLaunchKernelGGL(k_copyd, dim3(nblk(nP)), dim3(256), 0, s, h0, dp, nP);
            hipLaunchKernelGGL(k_axpy, dim3(nblk(nP)), dim3(256), 0, s, dp, h0, 1.0, nP);
            hipLaunchKernelGGL(k_axpy, dim3(nblk(nP)), dim3(256), 0, s, dp, h1, -1.0, nP);
            if (base) hipLaunchKernelGGL(k_axpy, dim3(nblk(nP)), dim3(256), 0, s, dp, base, -1.0, nP);
        } else {
            hipLaunchKernelGGL(k_zero, dim3(nblk(nP)), dim3(256), 0, s, dp, nP);
        }
        STDG_HIP(hipGetLastError());
        stdg_solve_report prep;
        STDG_HIP(hipStreamSynchronize(s));
        const double guess_sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - tg0).count();
        e = stdg_pressure_solve(m, bp, dp, &opts->pressure, &prep, s);
        if (e < 0) return e;
        if (e == STDG_NOT_CONVERGED) status = STDG_NOT_CONVERGED;
        piters += prep.inner_iters;
        papplies += prep.applies;
        fused_us_sum += prep.fused_iter_us * prep.inner_iters;
        fused_w += prep.fused_iter_us > 0.0 ? prep.inner_iters : 0;
        psec += prep.seconds + guess_sec;
        pres = std::max(pres, prep.rel_residual);
        if (k == 0) {
            first_iters = prep.inner_iters;
            first_sec = prep.seconds + guess_sec;
            first_res0 = prep.initial_rel_residual;
        }
        // step 6
        STDG_HIP(run_dualgrad(m, dp, dt, wg, s));
        hipLaunchKernelGGL(k_update, dim3(nblk(nD)), dim3(256), 0, s, Fv, wg, vk, F, NI, G, N);
        hipLaunchKernelGGL(k_axpy, dim3(nblk(nP)), dim3(256), 0, s, pk, dp, 1.0, nP);
        if (k == 0 && opts->rec_x)      // pk = p^{n+1,1}
            hipLaunchKernelGGL(k_copyd, dim3(nblk(nP)), dim3(256), 0, s, pk, opts->rec_x, nP);
        if (opts->hist) {
            // push this solve's value into its history
            double* h0 = hist_at(k, 0);
            hipLaunchKernelGGL(k_copyd, dim3(nblk(nP)), dim3(256), 0, s, h0, hist_at(k, 1), nP);
            hipLaunchKernelGGL(k_copyd, dim3(nblk(nP)), dim3(256), 0, s, k == 0 ? pk : dp, h0, nP);
        }
        STDG_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_copyd, dim3(nblk(nD)), dim3(256), 0, s, vk, vhat, nD);
    if (theta == 1.0)
        hipLaunchKernelGGL(k_copyd, dim3(nblk(nP)), dim3(256), 0, s, pk, p, nP);
    else    // p^{n+1} = (pi - (1 - theta) p^n) / theta
        hipLaunchKernelGGL(k_theta_end, dim3(nblk(nP)), dim3(256), 0, s, pk, p, theta, nP);
    if (int e = stdg_main_from_dual(m, vk, vbar, s)) return e;
    STDG_HIP(hipStreamSynchronize(s));
    if (rep) {
        rep->pressure_iters = piters;
        rep->viscous_iters = viters;
        rep->max_pressure_residual = pres;
        rep->max_viscous_residual = vres;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        rep->pressure_seconds = psec;
        rep->viscous_seconds = vsec;
        rep->pressure_applies = papplies;
        rep->first_pressure_iters = first_iters;
        rep->first_pressure_seconds = first_sec;
        rep->first_initial_residual = first_res0;
        rep->pressure_fused_iter_us = fused_w > 0.0 ? fused_us_sum / fused_w : 0.0;
        rep->guess_weight_network = guess_w;
        rep->status = status;
    }
    return status;
}
