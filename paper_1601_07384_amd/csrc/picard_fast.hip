// Block-row kernels of the Picard step (Sec. 2.6, steps 1, 3, 4, 5 and the
// viscous preconditioner): every output row of N coefficients is a sum of
// small N x N operator blocks times gathered rows.  One thread computes one
// row (entity, component or direction, time node) in registers.  Blocks are
// stored per geometry class (and local face), column-major; elements are
// class-chunked and faces sorted by their blocks' keys, so a wavefront
// usually reads one block: then its columns arrive through scalar loads
// broadcast to all lanes, otherwise each lane reads its own block.

#include "internal.hpp"
#include "kernels.hpp"

namespace stdg {
namespace {

// acc += s * B x with B column-major (column m at Bt + m N)
template <int N>
__device__ __forceinline__ void mv_acc(double (&acc)[N], const double* __restrict__ Bt, const double (&x)[N],
                                       double s) {
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const double xm = s * x[m];
#pragma unroll
        for (int r = 0; r < N; ++r) acc[r] += Bt[m * N + r] * xm;
    }
}

// acc += s * B(key) x, B(key) = base + key * N * N; scalar loads when the
// whole wavefront has the same key
template <int N>
__device__ __forceinline__ void mv_key(double (&acc)[N], const double* __restrict__ base, int64_t key,
                                       const double (&x)[N], double s) {
    const int64_t k0 = __builtin_amdgcn_readfirstlane((int)key);
    if (__all(key == k0)) {
        mv_acc<N>(acc, base + k0 * N * N, x, s);
    } else {
        mv_acc<N>(acc, base + key * N * N, x, s);
    }
}

template <int N>
__device__ __forceinline__ void load_row(double (&x)[N], const double* __restrict__ p) {
#pragma unroll
    for (int m = 0; m < N; ++m) x[m] = p[m];
}

template <int N>
__device__ __forceinline__ void store_row(double* __restrict__ p, const double (&x)[N], double s) {
#pragma unroll
    for (int m = 0; m < N; ++m) p[m] = s * x[m];
}

// dual-grid pressure gradient (the factor of eq. prevpress and eq. A3_mod):
// w[d][j][a] = dt sum_b TW[a][b] (US_{l,d} p_l[b] + UN_{l,d} p_r[b])
template <int N>
__global__ void __launch_bounds__(256) kf_dualgrad(const double* __restrict__ USt, const double* __restrict__ UNt,
                                                   const int32_t* __restrict__ cls, const int64_t* __restrict__ fl,
                                                   const int32_t* __restrict__ flf, const int64_t* __restrict__ fr,
                                                   const double* __restrict__ TW, const double* __restrict__ p,
                                                   double dt, double* __restrict__ w, int64_t F, int G) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * F * G) return;
    const int a = (int)(t % G);
    const int64_t j = (t / G) % F;
    const int d = (int)(t / ((int64_t)G * F));
    const int64_t l = fl[j], rr = fr[j];
    const int64_t key = ((int64_t)cls[l] * 4 + flf[j]) * 3 + d;
    double acc[N], x[N];
#pragma unroll
    for (int r = 0; r < N; ++r) acc[r] = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) x[m] = 0.0;
    for (int b = 0; b < G; ++b) {
        const double tw = TW[a * G + b];
        const double* pl = p + (l * G + b) * N;
#pragma unroll
        for (int m = 0; m < N; ++m) x[m] += tw * pl[m];
    }
    mv_key<N>(acc, USt, key, x, 1.0);
    if (rr >= 0) {
#pragma unroll
        for (int m = 0; m < N; ++m) x[m] = 0.0;
        for (int b = 0; b < G; ++b) {
            const double tw = TW[a * G + b];
            const double* pr = p + (rr * G + b) * N;
#pragma unroll
            for (int m = 0; m < N; ++m) x[m] += tw * pr[m];
        }
        mv_key<N>(acc, UNt, key, x, 1.0);
    }
    store_row<N>(w + ((d * F + j) * G + a) * N, acc, dt);
}

// eq. goback on faces f0 .. f1: out[c][j][a] = GB_l vbar_l[a] + GB_r vbar_r[a]
// (boundary faces: one side, from vbdry)
template <int N>
__global__ void __launch_bounds__(256) kf_goback(const double* __restrict__ GBt, const int32_t* __restrict__ cls,
                                                 const int64_t* __restrict__ fl, const int32_t* __restrict__ flf,
                                                 const int64_t* __restrict__ fr, const int32_t* __restrict__ frf,
                                                 const double* __restrict__ vbar, const double* __restrict__ vbdry,
                                                 double* __restrict__ out, int64_t f0, int64_t f1, int64_t F,
                                                 int64_t E, int G) {
    const int64_t nf = f1 - f0;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * nf * G) return;
    const int a = (int)(t % G);
    const int64_t j = f0 + (t / G) % nf;
    const int c = (int)(t / ((int64_t)G * nf));
    const int64_t l = fl[j], rr = fr[j];
    const double* src = rr >= 0 ? vbar : vbdry;
    double acc[N], x[N];
#pragma unroll
    for (int r = 0; r < N; ++r) acc[r] = 0.0;
    load_row<N>(x, src + ((c * E + l) * G + a) * N);
    mv_key<N>(acc, GBt, (int64_t)cls[l] * 4 + flf[j], x, 1.0);
    if (rr >= 0) {
        load_row<N>(x, vbar + ((c * E + rr) * G + a) * N);
        mv_key<N>(acc, GBt, (int64_t)cls[rr] * 4 + frf[j], x, 1.0);
    }
    store_row<N>(out + ((c * F + j) * G + a) * N, acc, 1.0);
}

// eq. average: vbar[c][i][a] = sum_f A_{i,f} vhat[c][face(i,f)][a]
template <int N>
__global__ void __launch_bounds__(256) kf_average(const double* __restrict__ At, const int32_t* __restrict__ cls,
                                                  const int64_t* __restrict__ tet_face,
                                                  const double* __restrict__ vhat, double* __restrict__ vbar,
                                                  int64_t E, int64_t F, int G) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * E * G) return;
    const int a = (int)(t % G);
    const int64_t i = (t / G) % E;
    const int c = (int)(t / ((int64_t)G * E));
    double acc[N], x[N];
#pragma unroll
    for (int r = 0; r < N; ++r) acc[r] = 0.0;
    for (int f = 0; f < 4; ++f) {
        load_row<N>(x, vhat + ((c * F + tet_face[4 * i + f]) * G + a) * N);
        mv_key<N>(acc, At, (int64_t)cls[i] * 4 + f, x, 1.0);
    }
    store_row<N>(vbar + ((c * E + i) * G + a) * N, acc, 1.0);
}

// pressure right-hand side (eq. A2_mod): b[i][a] = dt W_a sum_{f,d} Q^T_{i,f,d} Fv[d][face][a]
template <int N>
__global__ void __launch_bounds__(256) kf_rhs_pressure(const double* __restrict__ QTt, const int32_t* __restrict__ cls,
                                                       const int64_t* __restrict__ tet_face,
                                                       const double* __restrict__ W, const double* __restrict__ Fv,
                                                       double dt, double* __restrict__ b, int64_t E, int64_t F,
                                                       int G) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= E * G) return;
    const int a = (int)(t % G);
    const int64_t i = t / G;
    double acc[N], x[N];
#pragma unroll
    for (int r = 0; r < N; ++r) acc[r] = 0.0;
    for (int f = 0; f < 4; ++f) {
        const int64_t j = tet_face[4 * i + f];
        for (int d = 0; d < 3; ++d) {
            load_row<N>(x, Fv + ((d * F + j) * G + a) * N);
            mv_key<N>(acc, QTt, ((int64_t)cls[i] * 4 + f) * 3 + d, x, 1.0);
        }
    }
    store_row<N>(b + (i * G + a) * N, acc, dt * W[a]);
}

// viscous right-hand side (eq. A1_mod):
// rhs = M (sum_b g0g1[a][b] vprev_b - T[a][b] lam_b) - ups_a - nu dt W_a sum_{bdry f} BB_f vbc
template <int N>
__global__ void __launch_bounds__(256) kf_visc_rhs(const double* __restrict__ MIt, const double* __restrict__ BBt,
                                                   const int32_t* __restrict__ cls, const int32_t* __restrict__ nbr,
                                                   const int64_t* __restrict__ tet_face,
                                                   const double* __restrict__ g0g1, const double* __restrict__ Tm,
                                                   const double* __restrict__ W, const double* __restrict__ vprev,
                                                   const double* __restrict__ ups, const double* __restrict__ lam,
                                                   const double* __restrict__ vbc, double nu_dt,
                                                   double* __restrict__ rhs, int64_t E, int64_t F, int G) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * E * G) return;
    const int a = (int)(t % G);
    const int64_t i = (t / G) % E;
    const int c = (int)(t / ((int64_t)G * E));
    double acc[N], x[N];
#pragma unroll
    for (int r = 0; r < N; ++r) acc[r] = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) x[m] = 0.0;
    for (int b = 0; b < G; ++b) {
        const double g = g0g1[a * G + b], tm = Tm[a * G + b];
        const double* xp = vprev + ((c * E + i) * G + b) * N;
        const double* xl = lam + ((c * E + i) * G + b) * N;
#pragma unroll
        for (int m = 0; m < N; ++m) x[m] += g * xp[m] - tm * xl[m];
    }
    mv_key<N>(acc, MIt, cls[i], x, 1.0);
    const double* up = ups + ((c * E + i) * G + a) * N;
#pragma unroll
    for (int r = 0; r < N; ++r) acc[r] -= up[r];
    for (int f = 0; f < 4; ++f) {
        // boundary faces only: a wavefront of interior elements skips this
        if (nbr[4 * i + f] >= 0) continue;
        load_row<N>(x, vbc + ((c * F + tet_face[4 * i + f]) * G + a) * N);
        mv_acc<N>(acc, BBt + ((int64_t)cls[i] * 4 + f) * N * N, x, -nu_dt * W[a]);
    }
    store_row<N>(rhs + ((c * E + i) * G + a) * N, acc, 1.0);
}

// y = D^-1 x for the viscous block-Jacobi preconditioner: one thread per
// (component, element) applies the element's NG x NG inverse block (DV
// column-major per class).
template <int NG>
__global__ void __launch_bounds__(256) kf_blockdiag(const double* __restrict__ DV, const int32_t* __restrict__ cls,
                                                    const double* __restrict__ x, double* __restrict__ y, int64_t E) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * E) return;
    const int64_t i = t % E;
    double acc[NG], xv[NG];
#pragma unroll
    for (int r = 0; r < NG; ++r) acc[r] = 0.0;
    load_row<NG>(xv, x + t * NG);
    mv_key<NG>(acc, DV, cls[i], xv, 1.0);
    store_row<NG>(y + t * NG, acc, 1.0);
}

// The same product for meshes whose wavefronts mix classes: one thread per
// (element, row) forms that row for all three components, so each inverse
// entry is read once for the three; neighbouring threads read neighbouring
// rows of the column-major block (per output the same sum in the same order).
template <int NG>
__global__ void __launch_bounds__(256) kf_blockdiag3(const double* __restrict__ DV, const int32_t* __restrict__ cls,
                                                     const double* __restrict__ x, double* __restrict__ y, int64_t E) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= E * NG) return;
    const int64_t i = t / NG;
    const int r = (int)(t - i * NG);
    const double* D = DV + (int64_t)cls[i] * NG * NG + r;
    const double* x0 = x + i * NG;
    const int64_t cs = E * NG;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 8
    for (int m = 0; m < NG; ++m) {
        const double d = D[m * NG];
        a0 += d * x0[m];
        a1 += d * x0[cs + m];
        a2 += d * x0[2 * cs + m];
    }
    double* yo = y + i * NG + r;
    yo[0] = a0;
    yo[cs] = a1;
    yo[2 * cs] = a2;
}

inline unsigned nb(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

template <int N>
struct Launch {
    static hipError_t dualgrad(const stdg_mesh* m, const double* p, double dt, double* w, hipStream_t s) {
        const PicardDevice& d = m->pd;
        const int64_t F = (int64_t)m->faces.size();
        hipLaunchKernelGGL(kf_dualgrad<N>, dim3(nb(3 * F * m->G)), dim3(256), 0, s, d.USt, d.UNt, m->d.cls, d.fl,
                           d.flf, d.fr, d.TW, p, dt, w, F, m->G);
        return hipGetLastError();
    }
    static hipError_t goback(const stdg_mesh* m, const double* vbar, const double* vbdry, double* out, int64_t f0,
                             int64_t f1, hipStream_t s) {
        const PicardDevice& d = m->pd;
        const int64_t F = (int64_t)m->faces.size();
        if (f1 <= f0) return hipSuccess;
        hipLaunchKernelGGL(kf_goback<N>, dim3(nb(3 * (f1 - f0) * m->G)), dim3(256), 0, s, d.GBt, m->d.cls, d.fl,
                           d.flf, d.fr, d.frf, vbar, vbdry, out, f0, f1, F, m->E, m->G);
        return hipGetLastError();
    }
    static hipError_t average(const stdg_mesh* m, const double* vhat, double* vbar, hipStream_t s) {
        const PicardDevice& d = m->pd;
        hipLaunchKernelGGL(kf_average<N>, dim3(nb(3 * m->E * m->G)), dim3(256), 0, s, d.At, m->d.cls, d.tet_face,
                           vhat, vbar, m->E, (int64_t)m->faces.size(), m->G);
        return hipGetLastError();
    }
    static hipError_t rhs_pressure(const stdg_mesh* m, const double* Fv, double dt, double* b, hipStream_t s) {
        const PicardDevice& d = m->pd;
        hipLaunchKernelGGL(kf_rhs_pressure<N>, dim3(nb(m->E * m->G)), dim3(256), 0, s, d.QTt, m->d.cls, d.tet_face,
                           d.W, Fv, dt, b, m->E, (int64_t)m->faces.size(), m->G);
        return hipGetLastError();
    }
    static hipError_t visc_rhs(const stdg_mesh* m, const double* vprev, const double* ups, const double* lam,
                               const double* vbc, double* rhs, hipStream_t s) {
        const PicardDevice& d = m->pd;
        hipLaunchKernelGGL(kf_visc_rhs<N>, dim3(nb(3 * m->E * m->G)), dim3(256), 0, s, d.MIt, d.BBt, m->d.cls,
                           m->d.nbr, d.tet_face, d.g0g1, d.Tm, d.W, vprev, ups, lam, vbc, m->cfg.nu * m->cfg.dt, rhs,
                           m->E, (int64_t)m->faces.size(), m->G);
        return hipGetLastError();
    }
};

template <int NG>
hipError_t blockdiag_ng(const stdg_mesh* m, const double* x, double* y, hipStream_t s) {
    if ((int64_t)m->n_classes * 64 > m->E)
        hipLaunchKernelGGL(kf_blockdiag3<NG>, dim3(nb(m->E * NG)), dim3(256), 0, s, m->pd.DV, m->d.cls, x, y, m->E);
    else
        hipLaunchKernelGGL(kf_blockdiag<NG>, dim3(nb(3 * m->E)), dim3(256), 0, s, m->pd.DV, m->d.cls, x, y, m->E);
    return hipGetLastError();
}


// ------------------------------------------------------------- convection
// Space-time DG convection with the Rusanov flux (eq. convdg), restructured
// for throughput: a wavefront takes 64 consecutive elements (one per lane)
// at one time point t of the rule.  Elements are stored class-chunked, so the
// 64 lanes normally share one geometry class and every table entry (volume
// and face basis values, their gradients, weights, the class Jacobian and
// normals) is the same for the whole wavefront: it is read once through the
// scalar cache and applied by every lane.  A lane holds its element's
// velocity coefficients at time t (3 N values) in registers and, in each of
// two passes over the points, half of the 3 N output sums; the neighbour's
// coefficients across the face in hand are staged in the lane's own LDS
// column.  The per-time-point sums go to tmp[t][3][E][N]
// and kf_conv_combine weights them with the time basis (fixed order).  A
// wavefront that mixes classes (the tail of a mesh with many classes) runs
// the classes present one after the other, the other lanes masked.  With
// MIXED (meshes whose classes hold fewer elements than a wavefront, e.g.
// unstructured ones where every element is its own class) each lane reads
// its own class's tables with vector loads in a single pass.
template <int N, int G, bool MIXED>
__global__ void __launch_bounds__(64) kf_convection(
    const double* __restrict__ vbar, const double* __restrict__ vbc, const int32_t* __restrict__ cls,
    const int32_t* __restrict__ nbr, const int64_t* __restrict__ tet_face, const double* __restrict__ cJinv,
    const double* __restrict__ cdet, const double* __restrict__ cnrm, const double* __restrict__ PHf,
    const double* __restrict__ PHn, const double* __restrict__ FW, const double* __restrict__ PHv,
    const double* __restrict__ dPHv, const double* __restrict__ wv, const double* __restrict__ tw,
    const double* __restrict__ gq, int nqv, int nqf, int qt, double* __restrict__ tmp, int64_t E, int64_t F) {
    constexpr int KH = (N + 1) / 2;              // test functions per pass (two passes)
    __shared__ double xn_s[3 * N * 64];          // [3 N][lane]: neighbour coefficients at t
    const int lane = threadIdx.x;
    const int t = blockIdx.x % qt;
    const int64_t i = (int64_t)(blockIdx.x / qt) * 64 + lane;
    const bool valid = i < E;
    const int c = valid ? cls[i] : -1;
    double gt[G];
#pragma unroll
    for (int b = 0; b < G; ++b) gt[b] = gq[t * G + b];
    const double wt = tw[t];
    // own coefficients at time point t (staged through the lane's LDS column
    // one component at a time, which bounds the loads in flight)
#pragma unroll 1
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
        for (int n = 0; n < N; ++n) {
            double s = 0.0;
            if (valid)
#pragma unroll
                for (int b = 0; b < G; ++b) s += gt[b] * vbar[((cc * E + i) * G + b) * N + n];
            xn_s[(cc * N + n) * 64 + lane] = s;
        }
    double xt[3][N];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
        for (int n = 0; n < N; ++n) xt[cc][n] = xn_s[(cc * N + n) * 64 + lane];
#pragma unroll 1
    for (int k0 = 0; k0 < N; k0 += KH) {
        double o[3][KH];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
#pragma unroll
            for (int kk = 0; kk < KH; ++kk) o[cc][kk] = 0.0;
        for (uint64_t todo = __ballot(valid); todo;) {
            const int cur = MIXED ? c : __builtin_amdgcn_readlane(c, __builtin_ctzll(todo));
            const bool mine = valid && c == cur;
            todo = MIXED ? 0 : todo & ~__ballot(mine);
            if (!mine) continue;
            const double* Ji = cJinv + (int64_t)cur * 9;
            const double det = cdet[cur];
            // volume points: F_cd = v_c v_d pulled back by J^-T, tested with grad phi
#pragma unroll 1
            for (int q = 0; q < nqv; ++q) {
                const double* ph = PHv + (int64_t)q * N;
                double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int n = 0; n < N; ++n) {
                    const double pn = ph[n];
                    v[0] += pn * xt[0][n];
                    v[1] += pn * xt[1][n];
                    v[2] += pn * xt[2][n];
                }
                const double w = wt * wv[q] * det;
                double fl[3][3];
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    const double se = Ji[e * 3 + 0] * v[0] + Ji[e * 3 + 1] * v[1] + Ji[e * 3 + 2] * v[2];
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) fl[cc][e] = w * v[cc] * se;
                }
                const double* dp = dPHv + ((int64_t)q * N + k0) * 3;
#pragma unroll
                for (int kk = 0; kk < KH; ++kk) {
                    if (k0 + kk >= N) break;
                    const double d0 = dp[3 * kk], d1 = dp[3 * kk + 1], d2 = dp[3 * kk + 2];
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) o[cc][kk] -= d0 * fl[cc][0] + d1 * fl[cc][1] + d2 * fl[cc][2];
                }
            }
            // faces: own trace against the neighbour's (or the boundary data)
#pragma unroll 1
            for (int f = 0; f < 4; ++f) {
                // neighbour element k, or the boundary face's prescribed data
                const int64_t k = nbr[4 * i + f];
                const double* xp = k >= 0 ? vbar + k * G * N : vbc + tet_face[4 * i + f] * G * N;
                const int64_t cstr = (k >= 0 ? E : F) * G * N;
#pragma unroll 1
                for (int cc = 0; cc < 3; ++cc)
#pragma unroll
                    for (int n = 0; n < N; ++n) {
                        double s = 0.0;
#pragma unroll
                        for (int b = 0; b < G; ++b) s += gt[b] * xp[cc * cstr + b * N + n];
                        xn_s[(cc * N + n) * 64 + lane] = s;
                    }
                const double* nr = cnrm + (MIXED ? cur * 12 + f * 3 : __builtin_amdgcn_readfirstlane(cur * 12 + f * 3));
                const double n0 = nr[0], n1 = nr[1], n2 = nr[2];
#pragma unroll 1
                for (int q = 0; q < nqf; ++q) {
                    // (wavefront-uniform unless MIXED: the tables are then read
                    // through the scalar cache)
                    const int off = MIXED ? (cur * 4 + f) * nqf + q
                                          : __builtin_amdgcn_readfirstlane((cur * 4 + f) * nqf + q);
                    const double* pf = PHf + (int64_t)off * N;
                    const double* pn = PHn + (int64_t)off * N;
                    // the neighbour's coefficients are re-read from LDS at every
                    // point (an opaque offset keeps the compiler from hoisting
                    // them into registers next to the element's own)
                    int col = lane;
                    asm volatile("" : "+v"(col));
                    const double* xnl = xn_s + col;
                    double vm[3] = {0.0, 0.0, 0.0}, vp[3] = {0.0, 0.0, 0.0};
#pragma unroll
                    for (int n = 0; n < N; ++n) {
                        const double a = pf[n], bq = pn[n];
#pragma unroll
                        for (int cc = 0; cc < 3; ++cc) {
                            vm[cc] += a * xt[cc][n];
                            vp[cc] += bq * xnl[(cc * N + n) * 64];
                        }
                    }
                    const double unm = vm[0] * n0 + vm[1] * n1 + vm[2] * n2;
                    const double unp = vp[0] * n0 + vp[1] * n1 + vp[2] * n2;
                    const double am = sqrt(vm[0] * vm[0] + vm[1] * vm[1] + vm[2] * vm[2]);
                    const double ap = sqrt(vp[0] * vp[0] + vp[1] * vp[1] + vp[2] * vp[2]);
                    const double smax = 2.0 * (am > ap ? am : ap);
                    const double w = wt * FW[off];
                    double fc[3];
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc)
                        fc[cc] = w * (0.5 * (vp[cc] * unp + vm[cc] * unm) - 0.5 * smax * (vp[cc] - vm[cc]));
#pragma unroll
                    for (int kk = 0; kk < KH; ++kk) {
                        if (k0 + kk >= N) break;
                        const double a = pf[k0 + kk];
#pragma unroll
                        for (int cc = 0; cc < 3; ++cc) o[cc][kk] += a * fc[cc];
                    }
                }
            }
        }
        if (valid)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
#pragma unroll
                for (int kk = 0; kk < KH; ++kk)
                    if (k0 + kk < N) tmp[(((int64_t)t * 3 + cc) * E + i) * N + k0 + kk] = o[cc][kk];
    }
}

// ups[c][e][a][k] = dt sum_t gq[t][a] tmp[t][c][e][k]
template <int N, int G>
__global__ void kf_conv_combine(const double* __restrict__ tmp, const double* __restrict__ gq, int qt, double dt,
                                double* __restrict__ ups, int64_t E) {
    const int64_t n = 3 * E * N;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ce = idx / N;
        const int k = (int)(idx - ce * N);
        double acc[G];
#pragma unroll
        for (int a = 0; a < G; ++a) acc[a] = 0.0;
        for (int t = 0; t < qt; ++t) {
            const double v = tmp[(int64_t)t * n + idx];
#pragma unroll
            for (int a = 0; a < G; ++a) acc[a] += gq[t * G + a] * v;
        }
#pragma unroll
        for (int a = 0; a < G; ++a) ups[(ce * G + a) * N + k] = dt * acc[a];
    }
}


template <int N, int G>
hipError_t convection_ng(const stdg_mesh* m, const double* vbar, const double* vbc, double* ups, hipStream_t s) {
    const PicardTables& t = m->pt;
    PicardDevice& d = const_cast<stdg_mesh*>(m)->pd;
    const size_t need = (size_t)t.qt * 3 * m->E * N;
    if (d.conv_len < need) {
        if (d.conv_tmp) (void)hipFree(d.conv_tmp);
        d.conv_tmp = nullptr;
        d.conv_len = 0;
        const hipError_t e = hipMalloc(&d.conv_tmp, need * sizeof(double));
        if (e != hipSuccess) return e;
        d.conv_len = need;
    }
    const unsigned blocks = (unsigned)(((m->E + 63) / 64) * t.qt);
    // per-lane tables once classes average fewer elements than a wavefront
    if ((int64_t)m->n_classes * 64 > m->E)
        hipLaunchKernelGGL((kf_convection<N, G, true>), dim3(blocks), dim3(64), 0, s, vbar, vbc, m->d.cls, m->d.nbr,
                           d.tet_face, d.cJinv, d.cdet, d.cnrm, d.PHf, d.PHn, d.FW, d.PHv, d.dPHv, d.wv, d.tw,
                           d.gq, t.nqv, t.nqf, t.qt, d.conv_tmp, m->E, (int64_t)m->faces.size());
    else
        hipLaunchKernelGGL((kf_convection<N, G, false>), dim3(blocks), dim3(64), 0, s, vbar, vbc, m->d.cls,
                           m->d.nbr, d.tet_face, d.cJinv, d.cdet, d.cnrm, d.PHf, d.PHn, d.FW, d.PHv, d.dPHv, d.wv,
                           d.tw, d.gq, t.nqv, t.nqf, t.qt, d.conv_tmp, m->E, (int64_t)m->faces.size());
    const int64_t n = 3 * m->E * N;
    hipLaunchKernelGGL((kf_conv_combine<N, G>), dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256),
                       0, s, d.conv_tmp, d.gq, t.qt, m->cfg.dt, ups, m->E);
    return hipGetLastError();
}
}  // namespace

#define STDG_FAST_N(CALL)                          \
    switch (m->N) {                                \
        case 4: return Launch<4>::CALL;            \
        case 10: return Launch<10>::CALL;          \
        case 20: return Launch<20>::CALL;          \
        case 35: return Launch<35>::CALL;          \
        default: return hipErrorNotSupported;      \
    }

bool fast_rows_supported(const stdg_mesh* m) { return m->N == 4 || m->N == 10 || m->N == 20 || m->N == 35; }

hipError_t fast_dualgrad(const stdg_mesh* m, const double* p, double dt, double* w, hipStream_t s) {
    STDG_FAST_N(dualgrad(m, p, dt, w, s))
}
hipError_t fast_goback(const stdg_mesh* m, const double* vbar, const double* vbdry, double* out, int64_t f0,
                       int64_t f1, hipStream_t s) {
    STDG_FAST_N(goback(m, vbar, vbdry, out, f0, f1, s))
}
hipError_t fast_average(const stdg_mesh* m, const double* vhat, double* vbar, hipStream_t s) {
    STDG_FAST_N(average(m, vhat, vbar, s))
}
hipError_t fast_rhs_pressure(const stdg_mesh* m, const double* Fv, double dt, double* b, hipStream_t s) {
    STDG_FAST_N(rhs_pressure(m, Fv, dt, b, s))
}
hipError_t fast_visc_rhs(const stdg_mesh* m, const double* vprev, const double* ups, const double* lam,
                         const double* vbc, double* rhs, hipStream_t s) {
    STDG_FAST_N(visc_rhs(m, vprev, ups, lam, vbc, rhs, s))
}
#undef STDG_FAST_N

// convection for p <= 3 (the element's 3 N coefficients and 3 N sums in registers)
hipError_t fast_convection(const stdg_mesh* m, const double* vbar, const double* vbc, double* ups, hipStream_t s) {
#define STDG_CV(n, g) \
    if (m->N == n && m->G == g) return convection_ng<n, g>(m, vbar, vbc, ups, s);
    STDG_CV(4, 1) STDG_CV(4, 2) STDG_CV(4, 3) STDG_CV(4, 4) STDG_CV(4, 5)
    STDG_CV(10, 1) STDG_CV(10, 2) STDG_CV(10, 3) STDG_CV(10, 4) STDG_CV(10, 5)
    STDG_CV(20, 1) STDG_CV(20, 2) STDG_CV(20, 3) STDG_CV(20, 4) STDG_CV(20, 5)
#undef STDG_CV
    return hipErrorNotSupported;
}

// NG = N G up to 40 (p <= 3 with p_gamma <= 1, or p <= 2 with p_gamma <= 3)
hipError_t fast_blockdiag(const stdg_mesh* m, const double* x, double* y, hipStream_t s) {
    switch (m->Nst) {
        case 4: return blockdiag_ng<4>(m, x, y, s);
        case 8: return blockdiag_ng<8>(m, x, y, s);
        case 10: return blockdiag_ng<10>(m, x, y, s);
        case 12: return blockdiag_ng<12>(m, x, y, s);
        case 16: return blockdiag_ng<16>(m, x, y, s);
        case 20: return blockdiag_ng<20>(m, x, y, s);
        case 30: return blockdiag_ng<30>(m, x, y, s);
        case 40: return blockdiag_ng<40>(m, x, y, s);
        default: return hipErrorNotSupported;
    }
}

}  // namespace stdg
