// Quadrature, bases and dense helpers for the host-side block precompute.
#include "fem.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <numeric>

namespace stdg {

real norm(const V3& a) { return std::sqrt(dot(a, a)); }
real det3(const V3& c0, const V3& c1, const V3& c2) { return dot(c0, cross(c1, c2)); }

// Symmetric eigen-decomposition of a small dense matrix by cyclic Jacobi
// rotations.  A (n x n, row-major) is destroyed; eigenvalues in d, the
// eigenvectors in the columns of V.
static void sym_eig(int n, std::vector<real>& A, std::vector<real>& d,
                    std::vector<real>& V) {
    V.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        real off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-40L * tot) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                real apq = A[p * n + q];
                if (apq == 0.0) continue;
                real theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                real t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                real c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {      // A <- A R
                    real akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {      // A <- R^T A
                    real apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {      // V <- V R
                    real vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    d.resize(n);
    for (int i = 0; i < n; ++i) d[i] = A[i * n + i];
}

void gauss_jacobi(int n, real alpha, real beta, std::vector<real>& x,
                  std::vector<real>& w) {
    std::vector<real> J(n * n, 0.0);
    const real ab = alpha + beta;
    for (int k = 0; k < n; ++k) {
        real a;
        if (k == 0) a = (beta - alpha) / (ab + 2.0);
        else a = (beta * beta - alpha * alpha) / ((2 * k + ab) * (2 * k + ab + 2.0));
        J[k * n + k] = a;
        if (k + 1 < n) {
            const real m = k + 1;
            real b = 4.0 * m * (m + alpha) * (m + beta) * (m + ab) /
                       ((2 * m + ab) * (2 * m + ab) * (2 * m + ab + 1.0) * (2 * m + ab - 1.0));
            J[k * n + k + 1] = J[(k + 1) * n + k] = std::sqrt(b);
        }
    }
    std::vector<real> d, V;
    sym_eig(n, J, d, V);
    const real mu0 = std::pow((real)2, ab + 1) * std::tgamma(alpha + 1.0) *
                       std::tgamma(beta + 1.0) / std::tgamma(ab + 2.0);
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        x[i] = d[idx[i]];
        real v0 = V[0 * n + idx[i]];
        w[i] = mu0 * v0 * v0;
    }
}

void gauss_legendre01(int n, std::vector<real>& x, std::vector<real>& w) {
    gauss_jacobi(n, 0.0, 0.0, x, w);
    for (int i = 0; i < n; ++i) {
        x[i] = 0.5 * (x[i] + 1.0);
        w[i] *= 0.5;
    }
}

static void jacobi01(int n, real alpha, std::vector<real>& x, std::vector<real>& w) {
    // weight (1-u)^alpha on [0, 1]
    gauss_jacobi(n, alpha, 0.0, x, w);
    const real s = std::pow((real)2, alpha + 1);
    for (int i = 0; i < n; ++i) {
        x[i] = 0.5 * (x[i] + 1.0);
        w[i] /= s;
    }
}

// The rules depend only on q and cost an eigen-decomposition per direction;
// the block precompute asks for the same few rules for every face of every
// geometry class, so each is built once per process and then copied.
// (std::map entries never move and are never erased, so the references
// handed out stay valid while other threads add rules)
template <typename Build>
static const Rule& cached_rule(std::map<int, Rule>& cache, std::mutex& mu, int q, Build build) {
    {
        std::lock_guard<std::mutex> lk(mu);
        const auto it = cache.find(q);
        if (it != cache.end()) return it->second;
    }
    Rule r = build(q);
    std::lock_guard<std::mutex> lk(mu);
    return cache.emplace(q, std::move(r)).first->second;
}

static Rule build_tet_rule(int q) {
    std::vector<real> xu, wu, xv, wv, xw, ww;
    jacobi01(q, 2.0, xu, wu);
    jacobi01(q, 1.0, xv, wv);
    gauss_legendre01(q, xw, ww);
    Rule r;
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j)
            for (int k = 0; k < q; ++k) {
                real u = xu[i], v = xv[j], s = xw[k];
                r.pts.push_back({u, v * (1.0 - u), s * (1.0 - u) * (1.0 - v)});
                r.w.push_back(wu[i] * wv[j] * ww[k]);
            }
    return r;
}

static Rule build_tri_rule(int q) {
    std::vector<real> xu, wu, xv, wv;
    jacobi01(q, 1.0, xu, wu);
    gauss_legendre01(q, xv, wv);
    Rule r;
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) {
            r.pts.push_back({xu[i], xv[j] * (1.0 - xu[i]), 0.0});
            r.w.push_back(wu[i] * wv[j]);
        }
    return r;
}

const Rule& tet_rule(int q) {
    static std::map<int, Rule> cache;
    static std::mutex mu;
    return cached_rule(cache, mu, q, build_tet_rule);
}

const Rule& tri_rule(int q) {
    static std::map<int, Rule> cache;
    static std::mutex mu;
    return cached_rule(cache, mu, q, build_tri_rule);
}

std::vector<std::array<int, 3>> exponents(int p) {
    std::vector<std::array<int, 3>> e;
    for (int c = 0; c <= p; ++c)
        for (int b = 0; b <= p - c; ++b)
            for (int a = 0; a <= p - c - b; ++a) e.push_back({a, b, c});
    return e;
}

static inline real ipow(real x, int k) {
    real r = 1.0;
    for (int i = 0; i < k; ++i) r *= x;
    return r;
}

NodalBasis::NodalBasis(int p_) : p(p_) {
    ex = exponents(p);
    N = (int)ex.size();
    // VT[r][j] = xi_j^r ; coef = VT^{-1} so that coef * VT = I  (phi_k(xi_j) = delta)
    std::vector<real> VT(N * N);
    for (int j = 0; j < N; ++j) {
        V3 xi = {real(ex[j][0]) / p, real(ex[j][1]) / p, real(ex[j][2]) / p};
        for (int r = 0; r < N; ++r)
            VT[r * N + j] = ipow(xi[0], ex[r][0]) * ipow(xi[1], ex[r][1]) * ipow(xi[2], ex[r][2]);
    }
    // coef[k][r] with sum_r coef[k][r] VT[r][j] = delta_kj  ->  coef = inv(VT)
    lu_inverse(N, VT);
    coef = VT;
}

void NodalBasis::eval(const V3& xi, real* val) const {
    std::vector<real> mono(N);
    for (int r = 0; r < N; ++r)
        mono[r] = ipow(xi[0], ex[r][0]) * ipow(xi[1], ex[r][1]) * ipow(xi[2], ex[r][2]);
    for (int k = 0; k < N; ++k) {
        real s = 0.0;
        for (int r = 0; r < N; ++r) s += coef[k * N + r] * mono[r];
        val[k] = s;
    }
}

void NodalBasis::grad(const V3& xi, real* g) const {
    std::vector<real> dm(3 * N);
    for (int r = 0; r < N; ++r) {
        const auto& e = ex[r];
        dm[3 * r + 0] = e[0] ? e[0] * ipow(xi[0], e[0] - 1) * ipow(xi[1], e[1]) * ipow(xi[2], e[2]) : 0.0;
        dm[3 * r + 1] = e[1] ? e[1] * ipow(xi[0], e[0]) * ipow(xi[1], e[1] - 1) * ipow(xi[2], e[2]) : 0.0;
        dm[3 * r + 2] = e[2] ? e[2] * ipow(xi[0], e[0]) * ipow(xi[1], e[1]) * ipow(xi[2], e[2] - 1) : 0.0;
    }
    for (int k = 0; k < N; ++k)
        for (int d = 0; d < 3; ++d) {
            real s = 0.0;
            for (int r = 0; r < N; ++r) s += coef[k * N + r] * dm[3 * r + d];
            g[3 * k + d] = s;
        }
}

TimeBasis::TimeBasis(int G_) : G(G_) {
    gauss_legendre01(G, nodes, weights);
    std::vector<real> VT(G * G);
    for (int a = 0; a < G; ++a)
        for (int r = 0; r < G; ++r) VT[r * G + a] = ipow(nodes[a], r);
    lu_inverse(G, VT);
    coef = VT;
}

real TimeBasis::eval(int a, real tau) const {
    real s = 0.0;
    for (int r = 0; r < G; ++r) s += coef[a * G + r] * ipow(tau, r);
    return s;
}

real TimeBasis::deriv(int a, real tau) const {
    real s = 0.0;
    for (int r = 1; r < G; ++r) s += coef[a * G + r] * r * ipow(tau, r - 1);
    return s;
}

Affine::Affine(const std::array<V3, 4>& v) {
    v0 = v[0];
    for (int c = 0; c < 3; ++c)
        for (int r = 0; r < 3; ++r) J[r * 3 + c] = v[c + 1][r] - v[0][r];
    det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
          J[2] * (J[3] * J[7] - J[4] * J[6]);
    std::vector<real> A(J, J + 9);
    lu_inverse(3, A);
    for (int i = 0; i < 9; ++i) Jinv[i] = A[i];
}

V3 Affine::to_ref(const V3& x) const {
    V3 d = sub(x, v0);
    return {Jinv[0] * d[0] + Jinv[1] * d[1] + Jinv[2] * d[2],
            Jinv[3] * d[0] + Jinv[4] * d[1] + Jinv[5] * d[2],
            Jinv[6] * d[0] + Jinv[7] * d[1] + Jinv[8] * d[2]};
}

V3 Affine::to_phys(const V3& xi) const {
    return {v0[0] + J[0] * xi[0] + J[1] * xi[1] + J[2] * xi[2],
            v0[1] + J[3] * xi[0] + J[4] * xi[1] + J[5] * xi[2],
            v0[2] + J[6] * xi[0] + J[7] * xi[1] + J[8] * xi[2]};
}

bool lu_inverse(int n, std::vector<real>& A) {
    // Gauss-Jordan elimination with partial pivoting.
    std::vector<real> I(n * n, 0.0);
    for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0.0) return false;
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(A[c * n + k], A[piv * n + k]);
                std::swap(I[c * n + k], I[piv * n + k]);
            }
        real inv = 1.0 / A[c * n + c];
        for (int k = 0; k < n; ++k) {
            A[c * n + k] *= inv;
            I[c * n + k] *= inv;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            real f = A[r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                A[r * n + k] -= f * A[c * n + k];
                I[r * n + k] -= f * I[c * n + k];
            }
        }
    }
    A = I;
    return true;
}

bool cholesky(int n, std::vector<real>& A) {
    for (int j = 0; j < n; ++j) {
        real s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        if (!(s > 0.0)) return false;
        real l = std::sqrt(s);
        A[j * n + j] = l;
        for (int i = j + 1; i < n; ++i) {
            real t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = t / l;
        }
        for (int i = 0; i < j; ++i) A[i * n + j] = 0.0;
    }
    return true;
}

void cholesky_solve(int n, const std::vector<real>& L, real* b, int nrhs, int ldb) {
    for (int c = 0; c < nrhs; ++c) {
        // forward: L y = b
        for (int i = 0; i < n; ++i) {
            real s = b[i * ldb + c];
            for (int k = 0; k < i; ++k) s -= L[i * n + k] * b[k * ldb + c];
            b[i * ldb + c] = s / L[i * n + i];
        }
        // backward: L^T x = y
        for (int i = n - 1; i >= 0; --i) {
            real s = b[i * ldb + c];
            for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * b[k * ldb + c];
            b[i * ldb + c] = s / L[i * n + i];
        }
    }
}

}  // namespace stdg
