// Host-side finite-element machinery of the library: quadrature, bases and
// small dense linear algebra used while precomputing operator blocks.
#pragma once

#include <array>
#include <cstdint>
#include <vector>

namespace stdg {

// The one-time block precompute runs in x87 extended precision: the dual
// mass matrices of the Taylor basis reach condition numbers of 1e9-1e10 at
// p = 4, and 11 extra bits keep the stored FP64 blocks accurate to ~1e-14.
using real = long double;
using V3 = std::array<real, 3>;

inline V3 sub(const V3& a, const V3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
inline V3 add(const V3& a, const V3& b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2]}; }
inline V3 scale(const V3& a, real s) { return {a[0] * s, a[1] * s, a[2] * s}; }
inline real dot(const V3& a, const V3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline V3 cross(const V3& a, const V3& b) {
    return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
real norm(const V3& a);
real det3(const V3& c0, const V3& c1, const V3& c2);  // det of [c0 c1 c2] (columns)

// Gauss-Jacobi rule on [-1, 1] for the weight (1-x)^alpha (1+x)^beta by the
// Golub-Welsch method (eigen-decomposition of the Jacobi matrix).
void gauss_jacobi(int n, real alpha, real beta, std::vector<real>& x,
                  std::vector<real>& w);
// Gauss-Legendre on [0, 1].
void gauss_legendre01(int n, std::vector<real>& x, std::vector<real>& w);

struct Rule {
    std::vector<V3> pts;     // reference coordinates (tet: 3, triangle: first 2)
    std::vector<real> w;   // reference weights
};
// Conical-product (collapsed) rules with q points per direction, exact for
// total degree 2q-1: reference tet {xi >= 0, sum <= 1} (weights sum 1/6) and
// reference triangle {a, b >= 0, a + b <= 1} (weights sum 1/2).
const Rule& tet_rule(int q);
const Rule& tri_rule(int q);

std::vector<std::array<int, 3>> exponents(int p);   // first index fastest

// Nodal Lagrange basis on the reference tet through (j1, j2, j3)/p.
struct NodalBasis {
    int p = 0, N = 0;
    std::vector<std::array<int, 3>> ex;
    std::vector<real> coef;   // coef[k*N + r]: phi_k = sum_r coef * xi^r
    explicit NodalBasis(int p_);
    void eval(const V3& xi, real* val) const;                 // N values
    void grad(const V3& xi, real* g) const;                   // N x 3
};

// Lagrange basis in time through the Gauss-Legendre points of [0, 1].
struct TimeBasis {
    int G = 0;
    std::vector<real> nodes, weights, coef;  // coef[a*G + r]
    explicit TimeBasis(int G_);
    real eval(int a, real tau) const;
    real deriv(int a, real tau) const;
};

// Affine map x = v0 + J xi of a tetrahedron.
struct Affine {
    V3 v0;
    real J[9];      // row-major J[r*3+c], column c = v_{c+1} - v0
    real Jinv[9];
    real det;
    explicit Affine(const std::array<V3, 4>& v);
    V3 to_ref(const V3& x) const;
    V3 to_phys(const V3& xi) const;
};

// Dense helpers (row-major n x n).
bool lu_inverse(int n, std::vector<real>& A);            // in place
bool cholesky(int n, std::vector<real>& A);              // lower factor in place
void cholesky_solve(int n, const std::vector<real>& L, real* b, int nrhs, int ldb);

}  // namespace stdg
