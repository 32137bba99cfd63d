// stdg_mesh_build: primary mesh, face-based dual mesh (Sec. 2.2.1) and the
// precomputed pressure-operator blocks (Sec. 2.4, eq. CS_19; the paper keeps
// every coefficient matrix precomputed, Sec. 2.8).
//
// The pressure operator factors as space x time (the mesh is fixed inside a
// slab and the basis is a tensor product, Sec. 2.3):
//   Q_ij = dt Q^sp_ij (x) W,  D_ij = -Q_ij^T,  M_j = M^sp_j (x) T,
// with W = diag(Gauss-Legendre weights) and T_ab = g_a(1) g_b(1) - int g_a' g_b,
// so  S = -sum_j D_ij M_j^-1 Q_.j = dt^2 S^sp (x) C,  C = W T^-1 W.
// Only the N x N spatial blocks S^sp_ik = sum_d Q^sp_ij,d^T (M^sp_j)^-1 Q^sp_kj,d
// (k = i or the neighbour across face j) are stored, deduplicated over
// elements whose local geometry (own vertices and the four neighbours, in
// local vertex order, relative to local vertex 0) coincides.
#include <omp.h>

#include <algorithm>
#include <tuple>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <unordered_map>

#include "internal.hpp"

namespace stdg {

namespace {

uint64_t hilbert_key(uint32_t X[3], int bits) {
    // Skilling's transpose form of the Hilbert index (AIP Conf. Proc. 707, 2004).
    uint32_t M = 1u << (bits - 1), P, Q, t;
    for (Q = M; Q > 1; Q >>= 1) {
        P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) X[0] ^= P;
            else { t = (X[0] ^ X[i]) & P; X[0] ^= t; X[i] ^= t; }
        }
    }
    for (int i = 1; i < 3; ++i) X[i] ^= X[i - 1];
    t = 0;
    for (Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    uint64_t key = 0;
    for (int b = bits - 1; b >= 0; --b)
        for (int i = 0; i < 3; ++i) key = (key << 1) | ((X[i] >> b) & 1u);
    return key;
}

struct Tri { int64_t a, b, c; bool operator==(const Tri& o) const { return a == o.a && b == o.b && c == o.c; } };
struct TriHash {
    size_t operator()(const Tri& t) const {
        uint64_t h = (uint64_t)t.a * 0x9E3779B97F4A7C15ull;
        h ^= (uint64_t)t.b + 0x7F4A7C159E3779B9ull + (h << 6) + (h >> 2);
        h ^= (uint64_t)t.c + 0x94D049BB133111EBull + (h << 6) + (h >> 2);
        return (size_t)h;
    }
};

}  // namespace

V3 centroid(const std::array<V3, 4>& v) {
    return {(v[0][0] + v[1][0] + v[2][0] + v[3][0]) / 4, (v[0][1] + v[1][1] + v[2][1] + v[3][1]) / 4,
            (v[0][2] + v[1][2] + v[2][2] + v[3][2]) / 4};
}

// Taylor monomials (x - x0)^k / h^|k| (eq. bf_2), exponents first-fastest.
void taylor_eval(const std::vector<std::array<int, 3>>& ex, const V3& x, const V3& x0, real h,
                 real* out) {
    real y[3] = {(x[0] - x0[0]) / h, (x[1] - x0[1]) / h, (x[2] - x0[2]) / h};
    int p = 0;
    for (auto& e : ex) p = std::max(p, e[0] + e[1] + e[2]);
    real pw[3][8];
    for (int d = 0; d < 3; ++d) {
        pw[d][0] = 1.0;
        for (int k = 1; k <= p; ++k) pw[d][k] = pw[d][k - 1] * y[d];
    }
    for (size_t r = 0; r < ex.size(); ++r) out[r] = pw[0][ex[r][0]] * pw[1][ex[r][1]] * pw[2][ex[r][2]];
}

// Dual-element data of one face seen from element t (side 0) and its
// neighbour (side 1): the spatial Q blocks (3 x N x N, rows = dual basis) of
// both sides and the dual mass matrix M^sp_j.
struct DualFaceBlocks {
    std::vector<real> M;          // N x N
    std::vector<real> Q[2];       // 3 x N x N each
};

static void dual_face_blocks(const NodalBasis& phi, int p, const std::array<V3, 4>& Vt, int f,
                             const std::array<V3, 4>& Vk, DualFaceBlocks& out) {
    const int N = phi.N;
    const auto ex = exponents(p);
    V3 P[3];
    for (int k = 0, m = 0; k < 4; ++k)
        if (k != f) P[m++] = Vt[k];
    const V3 bc[2] = {centroid(Vt), centroid(Vk)};
    // dual basis centre: volume centroid of H_j; scale: half its diameter
    real vol[2];
    V3 cen[2];
    for (int s = 0; s < 2; ++s) {
        vol[s] = std::fabs(det3(sub(P[0], bc[s]), sub(P[1], bc[s]), sub(P[2], bc[s]))) / 6.0;
        cen[s] = scale(add(add(P[0], P[1]), add(P[2], bc[s])), 0.25);
    }
    V3 x0 = scale(add(scale(cen[0], vol[0]), scale(cen[1], vol[1])), 1.0 / (vol[0] + vol[1]));
    V3 pts5[5] = {P[0], P[1], P[2], bc[0], bc[1]};
    real h = 0.0;   // half the diameter: scaled coordinates in [-1, 1]
    for (int a = 0; a < 5; ++a)
        for (int b = a + 1; b < 5; ++b) h = std::max(h, 0.5 * norm(sub(pts5[a], pts5[b])));
    V3 nrm = cross(sub(P[1], P[0]), sub(P[2], P[0]));
    nrm = scale(nrm, 1.0 / norm(nrm));
    if (dot(nrm, sub(P[0], bc[0])) < 0) nrm = scale(nrm, -1.0);   // outward of t

    out.M.assign(N * N, 0.0);
    for (int s = 0; s < 2; ++s) out.Q[s].assign(3 * N * N, 0.0);
    const Affine A[2] = {Affine(Vt), Affine(Vk)};
    const int q = p + 1;
    const Rule& tr = tet_rule(q);
    std::vector<real> ps(N), ph(N), gr(3 * N), gx(3 * N);
    for (int s = 0; s < 2; ++s) {
        // sub-tetrahedron T_{i,j}: the face and the element's barycentre
        std::array<V3, 4> sv = {bc[s], P[0], P[1], P[2]};
        Affine sa(sv);
        const real jac = std::fabs(sa.det);
        for (size_t m = 0; m < tr.w.size(); ++m) {
            V3 x = sa.to_phys(tr.pts[m]);
            real w = tr.w[m] * jac;
            taylor_eval(ex, x, x0, h, ps.data());
            V3 xi = A[s].to_ref(x);
            phi.grad(xi, gr.data());
            // physical gradient: J^{-T} grad_xi
            for (int k = 0; k < N; ++k)
                for (int d = 0; d < 3; ++d)
                    gx[3 * k + d] = A[s].Jinv[0 * 3 + d] * gr[3 * k + 0] +
                                    A[s].Jinv[1 * 3 + d] * gr[3 * k + 1] +
                                    A[s].Jinv[2 * 3 + d] * gr[3 * k + 2];
            for (int a = 0; a < N; ++a) {
                const real wa = w * ps[a];
                for (int b = 0; b < N; ++b) out.M[a * N + b] += wa * ps[b];
                for (int d = 0; d < 3; ++d)
                    for (int b = 0; b < N; ++b) out.Q[s][(d * N + a) * N + b] += wa * gx[3 * b + d];
            }
        }
    }
    // face part: - int_Gamma psi phi_i n_ij  (n_ij outward of element i)
    const Rule& fr = tri_rule(q);
    const V3 e1 = sub(P[1], P[0]), e2 = sub(P[2], P[0]);
    const real area2 = norm(cross(e1, e2));
    for (size_t m = 0; m < fr.w.size(); ++m) {
        V3 x = add(P[0], add(scale(e1, fr.pts[m][0]), scale(e2, fr.pts[m][1])));
        real w = fr.w[m] * area2;
        taylor_eval(ex, x, x0, h, ps.data());
        for (int s = 0; s < 2; ++s) {
            phi.eval(A[s].to_ref(x), ph.data());
            const real sg = (s == 0) ? 1.0 : -1.0;
            for (int a = 0; a < N; ++a)
                for (int d = 0; d < 3; ++d) {
                    const real c = w * ps[a] * sg * nrm[d];
                    for (int b = 0; b < N; ++b) out.Q[s][(d * N + a) * N + b] -= c * ph[b];
                }
        }
    }
}

// ---- curved (isoparametric) elements, Sec. 2.8 -------------------------
// Element i is the image of the reference tetrahedron under
// x_i(xi) = sum_k X_ik phi_k(xi) (the degree-p nodal basis through its N
// nodes).  The sub-tetrahedron T_ij is the image under x_i of the reference
// sub-tetrahedron spanned by the reference face and the reference
// barycentre; the face is the image of the reference face, met by both
// elements at equal barycentric coordinates of its three vertices.  All
// integrals run in reference coordinates (dx = |det J| dxi, grad_x =
// J^-T grad_xi, n dS = t_u x t_v du dv); the integrands are then
// polynomials in xi of degree at most 2p^2 + 3(p-1) (volume) and
// p^2 + 3p - 2 (face), which the collapsed rules below integrate exactly.

static const V3 kRefVert[4] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

// Position and Jacobian (J[r*3+c] = dx_r/dxi_c) of the isoparametric map
// with nodes X at xi; val (N) and grad (N x 3) receive the nodal basis there.
static void iso_point(const NodalBasis& phi, const V3* X, const V3& xi, real* val, real* grad, V3& x,
                      real J[9]) {
    phi.eval(xi, val);
    phi.grad(xi, grad);
    x = {0, 0, 0};
    for (int i = 0; i < 9; ++i) J[i] = 0;
    for (int k = 0; k < phi.N; ++k)
        for (int r = 0; r < 3; ++r) {
            x[r] += X[k][r] * val[k];
            for (int c = 0; c < 3; ++c) J[r * 3 + c] += X[k][r] * grad[3 * k + c];
        }
}

// x and J of the map with nodes X from the basis values and gradients at a point
static void iso_from(int N, const V3* X, const real* val, const real* grad, V3& x, real J[9]) {
    x = {0, 0, 0};
    for (int i = 0; i < 9; ++i) J[i] = 0;
    for (int k = 0; k < N; ++k)
        for (int r = 0; r < 3; ++r) {
            x[r] += X[k][r] * val[k];
            for (int c = 0; c < 3; ++c) J[r * 3 + c] += X[k][r] * grad[3 * k + c];
        }
}

// The volume rule of the reference sub-tetrahedron of local face g (the
// reference barycentre and the face's vertices in ascending order), with the
// nodal basis and its reference gradients at its points: the same for every
// curved element, so built once per degree and face.
struct SubTetRule {
    std::vector<V3> xi;
    std::vector<real> w, val, grad;   // w includes the sub-tetrahedron's volume factor
};
static const SubTetRule& subtet_rule(const NodalBasis& phi, int g) {
    static std::mutex mu;
    static std::map<std::pair<int, int>, SubTetRule> cache;
    const std::pair<int, int> key(phi.p, g);
    {
        std::lock_guard<std::mutex> lk(mu);
        const auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    const int p = phi.p, N = phi.N;
    const Rule& tr = tet_rule(p * p + (3 * p - 1) / 2);      // exact for degree 2p^2 + 3p - 3
    std::array<V3, 4> sv;
    sv[0] = {0.25L, 0.25L, 0.25L};
    for (int k = 0, n = 1; k < 4; ++k)
        if (k != g) sv[n++] = kRefVert[k];
    const Affine sa(sv);
    SubTetRule r;
    const size_t nq = tr.w.size();
    r.xi.resize(nq);
    r.w.resize(nq);
    r.val.resize(nq * N);
    r.grad.resize(nq * 3 * N);
    for (size_t q = 0; q < nq; ++q) {
        r.xi[q] = sa.to_phys(tr.pts[q]);
        r.w[q] = tr.w[q] * std::fabs(sa.det);
        phi.eval(r.xi[q], r.val.data() + q * N);
        phi.grad(r.xi[q], r.grad.data() + q * 3 * N);
    }
    std::lock_guard<std::mutex> lk(mu);
    return cache.emplace(key, std::move(r)).first->second;    // map entries never move
}

static real inv3(const real J[9], real Ji[9]) {
    const real det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                     J[2] * (J[3] * J[7] - J[4] * J[6]);
    Ji[0] = (J[4] * J[8] - J[5] * J[7]) / det;
    Ji[1] = (J[2] * J[7] - J[1] * J[8]) / det;
    Ji[2] = (J[1] * J[5] - J[2] * J[4]) / det;
    Ji[3] = (J[5] * J[6] - J[3] * J[8]) / det;
    Ji[4] = (J[0] * J[8] - J[2] * J[6]) / det;
    Ji[5] = (J[2] * J[3] - J[0] * J[5]) / det;
    Ji[6] = (J[3] * J[7] - J[4] * J[6]) / det;
    Ji[7] = (J[1] * J[6] - J[0] * J[7]) / det;
    Ji[8] = (J[0] * J[4] - J[1] * J[3]) / det;
    return det;
}

// Curved counterpart of dual_face_blocks: Xt, Xk the N nodes of element t
// and of its neighbour across t's local face f (Xk translated by shk next to
// t); kv[i] the neighbour's local vertex at t's i-th face vertex (face
// vertices = t's local vertices other than f, ascending).  Returns -2 when the
// two elements do not share the curved face, -3 when the map of either
// element folds (det J at a quadrature point of its sub-tetrahedron has the
// opposite sign of det J at the element's barycentre, or vanishes).
static int curved_face_blocks(const NodalBasis& phi, int p, const V3* Xt, int f, const V3* Xk, const V3& shk,
                              const int kv[3], DualFaceBlocks& out) {
    const int N = phi.N;
    const auto ex = exponents(p);
    const V3 bref = {0.25L, 0.25L, 0.25L};
    int lv[3];
    for (int k = 0, n = 0; k < 4; ++k)
        if (k != f) lv[n++] = k;
    V3 ref[2][3];
    for (int i = 0; i < 3; ++i) {
        ref[0][i] = kRefVert[lv[i]];
        ref[1][i] = kRefVert[kv[i]];
    }
    const V3* X[2] = {Xt, Xk};
    const V3 sh[2] = {{0, 0, 0}, shk};
    std::vector<real> val(N), grad(3 * N), ps(N), gx(3 * N), ph[2] = {std::vector<real>(N), std::vector<real>(N)};
    real J[9], Ji[9];
    auto map = [&](int s, const V3& xi, V3& x) {
        iso_point(phi, X[s], xi, val.data(), grad.data(), x, J);
        x = add(x, sh[s]);
    };
    // dual basis centre and scale as on straight faces, with the element
    // barycentres replaced by their images
    V3 P[3], bc[2];
    for (int i = 0; i < 3; ++i) map(0, ref[0][i], P[i]);
    for (int s = 0; s < 2; ++s) map(s, bref, bc[s]);
    real vol[2];
    V3 cen[2];
    for (int s = 0; s < 2; ++s) {
        vol[s] = std::fabs(det3(sub(P[0], bc[s]), sub(P[1], bc[s]), sub(P[2], bc[s]))) / 6.0;
        cen[s] = scale(add(add(P[0], P[1]), add(P[2], bc[s])), 0.25);
    }
    const V3 x0 = scale(add(scale(cen[0], vol[0]), scale(cen[1], vol[1])), 1.0 / (vol[0] + vol[1]));
    const V3 pts5[5] = {P[0], P[1], P[2], bc[0], bc[1]};
    real h = 0.0;
    for (int a = 0; a < 5; ++a)
        for (int b = a + 1; b < 5; ++b) h = std::max(h, 0.5 * norm(sub(pts5[a], pts5[b])));

    out.M.assign(N * N, 0.0);
    for (int s = 0; s < 2; ++s) out.Q[s].assign(3 * N * N, 0.0);
    const int gk = 6 - kv[0] - kv[1] - kv[2];                  // the neighbour's local face
    for (int s = 0; s < 2; ++s) {
        const SubTetRule& tr = subtet_rule(phi, s == 0 ? f : gk);
        V3 xb;
        map(s, bref, xb);
        const real det_b = inv3(J, Ji);                          // orientation of the element
        for (size_t q = 0; q < tr.w.size(); ++q) {
            V3 x;
            const real* gq = tr.grad.data() + q * 3 * N;
            iso_from(N, X[s], tr.val.data() + q * N, gq, x, J);
            x = add(x, sh[s]);
            const real dj = inv3(J, Ji);
            if (!(dj * det_b > 1e-12L * det_b * det_b)) return -3;
            const real w = tr.w[q] * std::fabs(dj);
            taylor_eval(ex, x, x0, h, ps.data());
            for (int k = 0; k < N; ++k)          // J^-T grad_xi
                for (int d = 0; d < 3; ++d)
                    gx[3 * k + d] = Ji[0 * 3 + d] * gq[3 * k + 0] + Ji[1 * 3 + d] * gq[3 * k + 1] +
                                    Ji[2 * 3 + d] * gq[3 * k + 2];
            for (int a = 0; a < N; ++a) {
                const real wa = w * ps[a];
                for (int b = 0; b < N; ++b) out.M[a * N + b] += wa * ps[b];
                for (int d = 0; d < 3; ++d)
                    for (int b = 0; b < N; ++b) out.Q[s][(d * N + a) * N + b] += wa * gx[3 * b + d];
            }
        }
    }
    // face part: - int_Gamma psi phi_i n_ij dS, n dS = +-(t_u x t_v) du dv
    const V3 e1 = sub(ref[0][1], ref[0][0]), e2 = sub(ref[0][2], ref[0][0]);
    V3 nref = cross(e1, e2);                                   // reference normal out of t
    if (dot(nref, sub(ref[0][0], kRefVert[f])) < 0) nref = scale(nref, -1.0);
    const Rule& fr = tri_rule(p * (p + 3) / 2);               // exact for degree p^2 + 3p - 2
    for (size_t q = 0; q < fr.w.size(); ++q) {
        const real lam[3] = {1 - fr.pts[q][0] - fr.pts[q][1], fr.pts[q][0], fr.pts[q][1]};
        V3 xi[2] = {{0, 0, 0}, {0, 0, 0}};
        for (int s = 0; s < 2; ++s)
            for (int i = 0; i < 3; ++i) xi[s] = add(xi[s], scale(ref[s][i], lam[i]));
        V3 x, x1;
        map(1, xi[1], x1);
        std::copy(val.begin(), val.end(), ph[1].begin());
        map(0, xi[0], x);
        std::copy(val.begin(), val.end(), ph[0].begin());
        if (norm(sub(x, x1)) > 1e-9 * h) return -2;
        inv3(J, Ji);
        V3 tu, tv;
        for (int r = 0; r < 3; ++r) {
            tu[r] = J[r * 3 + 0] * e1[0] + J[r * 3 + 1] * e1[1] + J[r * 3 + 2] * e1[2];
            tv[r] = J[r * 3 + 0] * e2[0] + J[r * 3 + 1] * e2[1] + J[r * 3 + 2] * e2[2];
        }
        V3 A = cross(tu, tv);
        V3 ng;                                                 // J^-T n_ref points out of t
        for (int d = 0; d < 3; ++d) ng[d] = Ji[0 * 3 + d] * nref[0] + Ji[1 * 3 + d] * nref[1] + Ji[2 * 3 + d] * nref[2];
        if (dot(A, ng) < 0) A = scale(A, -1.0);
        taylor_eval(ex, x, x0, h, ps.data());
        for (int s = 0; s < 2; ++s) {
            const real sg = (s == 0) ? 1.0 : -1.0;
            for (int a = 0; a < N; ++a)
                for (int d = 0; d < 3; ++d) {
                    const real c = fr.w[q] * ps[a] * sg * A[d];
                    for (int b = 0; b < N; ++b) out.Q[s][(d * N + a) * N + b] -= c * ph[s][b];
                }
        }
    }
    return 0;
}

// Five dt^2-scaled spatial blocks of element t: [0] diagonal, [1+f] coupling
// to the neighbour across local face f (zero on a boundary face).
static int element_blocks(const stdg_mesh* m, int64_t t, const NodalBasis& phi, double* Bout) {
    const int N = m->N;
    std::vector<real> Bv(5 * N * N, 0.0L);
    real* B = Bv.data();
    const real dt2 = m->cfg.dt * m->cfg.dt;
    DualFaceBlocks fb;
    std::vector<real> Z(3 * N * N);
    for (int f = 0; f < 4; ++f) {
        const int64_t k = m->nbr[t * 4 + f];
        if (k < 0) continue;
        const V3 sh = neighbour_shift(m, t, f);
        std::array<V3, 4> Vk = m->vert[k];
        for (auto& v : Vk) v = add(v, sh);
        if (m->curved && (m->bent[t] || m->bent[k])) {
            int kv[3];
            for (int a = 0, n = 0; a < 4; ++a) {
                if (a == f) continue;
                int best = 0;
                for (int b = 1; b < 4; ++b)
                    if (norm(sub(Vk[b], m->vert[t][a])) < norm(sub(Vk[best], m->vert[t][a]))) best = b;
                kv[n++] = best;
            }
            const int r = curved_face_blocks(phi, m->p, m->geo.data() + t * N, f, m->geo.data() + k * N, sh, kv, fb);
            if (r != 0) return r;
        } else {
            dual_face_blocks(phi, m->p, m->vert[t], f, Vk, fb);
        }
        std::vector<real> L = fb.M;
        if (!cholesky(N, L)) return -1;
        for (int s = 0; s < 2; ++s) {
            // Z = M^-1 Q_s (per component)
            std::copy(fb.Q[s].begin(), fb.Q[s].end(), Z.begin());
            for (int d = 0; d < 3; ++d) cholesky_solve(N, L, Z.data() + d * N * N, N, N);
            real* dst = B + (s == 0 ? 0 : (1 + f)) * N * N;
            for (int d = 0; d < 3; ++d)
                for (int a = 0; a < N; ++a)
                    for (int c = 0; c < N; ++c) {
                        const real qa = fb.Q[0][(d * N + c) * N + a];   // (Q_t^T)_{a c}
                        if (qa == 0.0) continue;
                        for (int b = 0; b < N; ++b) dst[a * N + b] += qa * Z[(d * N + c) * N + b];
                    }
        }
    }
    for (int i = 0; i < 5 * N * N; ++i) Bout[i] = (double)(B[i] * dt2);
    return 0;
}

static void time_factor(int G, std::vector<double>& Cout) {
    TimeBasis tb(G);
    std::vector<real> T(G * G), W(G);
    std::vector<real> xq, wq;
    gauss_legendre01(G + 1, xq, wq);
    for (int a = 0; a < G; ++a) {
        W[a] = tb.weights[a];
        for (int b = 0; b < G; ++b) {
            real s = 0.0;
            for (size_t m = 0; m < xq.size(); ++m) s += wq[m] * tb.deriv(a, xq[m]) * tb.eval(b, xq[m]);
            T[a * G + b] = tb.eval(a, 1.0) * tb.eval(b, 1.0) - s;
        }
    }
    lu_inverse(G, T);
    Cout.assign(G * G, 0.0);
    for (int a = 0; a < G; ++a)
        for (int b = 0; b < G; ++b) Cout[a * G + b] = (double)(W[a] * T[a * G + b] * W[b]);
}

int build_topology(stdg_mesh* m, const double* xyz, int64_t n_vert, const int64_t* tets,
                   const std::vector<int64_t>* order) {
    const int64_t E = m->E;
    const stdg_config& cfg = m->cfg;
    for (int64_t i = 0; i < 4 * E; ++i)
        if (tets[i] < 0 || tets[i] >= n_vert) { set_error("vertex index out of range"); return STDG_ERR_ARG; }
    // bounding box and element renumbering along a Hilbert curve
    V3 lo = {1e300, 1e300, 1e300}, hi = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < n_vert; ++v)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], (real)xyz[3 * v + d]);
            hi[d] = std::max(hi[d], (real)xyz[3 * v + d]);
        }
    const real diag = norm(sub(hi, lo));
    m->perm.resize(E);
    std::iota(m->perm.begin(), m->perm.end(), 0);
    if (order) {
        m->perm = *order;
    } else if (cfg.reorder) {
        std::vector<uint64_t> key(E);
        const int bits = 16;
        const double span = (1u << bits) - 1;
        for (int64_t t = 0; t < E; ++t) {
            V3 c = {0, 0, 0};
            for (int k = 0; k < 4; ++k)
                for (int d = 0; d < 3; ++d) c[d] += 0.25 * xyz[3 * tets[4 * t + k] + d];
            uint32_t X[3];
            for (int d = 0; d < 3; ++d) {
                double ext = hi[d] - lo[d];
                double u = ext > 0 ? (c[d] - lo[d]) / ext : 0.0;
                X[d] = (uint32_t)std::llround(std::min(1.0, std::max(0.0, u)) * span);
            }
            key[t] = hilbert_key(X, bits);
        }
        std::stable_sort(m->perm.begin(), m->perm.end(),
                         [&](int64_t a, int64_t b) { return key[a] < key[b]; });
    }
    m->iperm.resize(E);
    for (int64_t t = 0; t < E; ++t) m->iperm[m->perm[t]] = t;
    m->vert.resize(E);
    real min_edge = 1e300;
    for (int64_t t = 0; t < E; ++t) {
        const int64_t* tv = tets + 4 * m->perm[t];
        for (int k = 0; k < 4; ++k) {
            m->vert[t][k] = {xyz[3 * tv[k]], xyz[3 * tv[k] + 1], xyz[3 * tv[k] + 2]};
        }
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b) min_edge = std::min(min_edge, norm(sub(m->vert[t][a], m->vert[t][b])));
    }
    for (int64_t t = 0; t < E; ++t) {
        const auto& v = m->vert[t];
        double det = det3(sub(v[1], v[0]), sub(v[2], v[0]), sub(v[3], v[0]));
        if (!(std::fabs(det) > 1e-10 * min_edge * min_edge * min_edge)) {
            set_error("degenerate (flat) element " + std::to_string(m->perm[t]));
            return STDG_ERR_MESH;
        }
    }
    // canonical vertex ids (periodic images identified)
    std::vector<int64_t> canon(n_vert);
    if (cfg.periodic) {
        V3 L;
        for (int d = 0; d < 3; ++d) L[d] = cfg.box_hi[d] - cfg.box_lo[d];
        const double tol = 1e-9 * std::max({L[0], L[1], L[2]});
        std::map<std::array<int64_t, 3>, int64_t> ids;
        for (int64_t v = 0; v < n_vert; ++v) {
            std::array<int64_t, 3> q;
            for (int d = 0; d < 3; ++d) {
                double y = std::fmod(xyz[3 * v + d] - cfg.box_lo[d], L[d]);
                if (y < 0) y += L[d];
                if (std::fabs(y - L[d]) < tol) y = 0.0;
                q[d] = std::llround(y / tol);
            }
            auto it = ids.find(q);
            if (it == ids.end()) it = ids.emplace(q, (int64_t)ids.size()).first;
            canon[v] = it->second;
        }
    } else {
        std::iota(canon.begin(), canon.end(), 0);
    }
    // faces
    std::unordered_map<Tri, std::vector<std::pair<int64_t, int>>, TriHash> table;
    table.reserve(4 * E);
    for (int64_t t = 0; t < E; ++t) {
        const int64_t* tv = tets + 4 * m->perm[t];
        for (int f = 0; f < 4; ++f) {
            int64_t c[3];
            for (int k = 0, n = 0; k < 4; ++k)
                if (k != f) c[n++] = canon[tv[k]];
            std::sort(c, c + 3);
            table[{c[0], c[1], c[2]}].push_back({t, f});
        }
    }
    std::vector<Face> inner, bdry;
    for (auto& kv : table) {
        auto& l = kv.second;
        if (l.size() > 2) { set_error("non-manifold face"); return STDG_ERR_MESH; }
        std::sort(l.begin(), l.end());
        Face F;
        F.left = l[0].first; F.lf = l[0].second;
        F.shift = {0, 0, 0};
        if (l.size() == 2) {
            F.right = l[1].first; F.rf = l[1].second;
            if (cfg.periodic) {
                const int64_t* tl = tets + 4 * m->perm[F.left];
                const int64_t* tr = tets + 4 * m->perm[F.right];
                int64_t a = tl[F.lf == 0 ? 1 : 0];
                for (int k = 0; k < 4; ++k)
                    if (k != F.rf && canon[tr[k]] == canon[a]) {
                        for (int d = 0; d < 3; ++d) F.shift[d] = xyz[3 * a + d] - xyz[3 * tr[k] + d];
                    }
            }
            inner.push_back(F);
        } else {
            if (cfg.periodic) { set_error("unmatched periodic face"); return STDG_ERR_MESH; }
            F.right = -1; F.rf = -1;
            bdry.push_back(F);
        }
    }
    auto byl = [](const Face& a, const Face& b) { return a.left != b.left ? a.left < b.left : a.lf < b.lf; };
    std::sort(inner.begin(), inner.end(), byl);
    std::sort(bdry.begin(), bdry.end(), byl);
    m->n_interior = (int64_t)inner.size();
    m->faces = inner;
    m->faces.insert(m->faces.end(), bdry.begin(), bdry.end());
    m->nbr.assign(4 * E, -1);
    m->tet_face.assign(4 * E, -1);
    for (int64_t j = 0; j < (int64_t)m->faces.size(); ++j) {
        const Face& F = m->faces[j];
        m->tet_face[4 * F.left + F.lf] = j;
        if (F.right >= 0) {
            m->tet_face[4 * F.right + F.rf] = j;
            m->nbr[4 * F.left + F.lf] = (int32_t)F.right;
            m->nbr[4 * F.right + F.rf] = (int32_t)F.left;
        }
    }
    (void)diag;
    return STDG_OK;
}

// Translation that brings the neighbour across local face f next to t.
V3 neighbour_shift(const stdg_mesh* m, int64_t t, int f) {
    const Face& F = m->faces[m->tet_face[t * 4 + f]];
    if (F.left == t && F.lf == f) return F.shift;          // neighbour is the right element
    return scale(F.shift, -1.0);                           // neighbour is the left element
}

// Class of every element: elements whose own vertices and whose four
// neighbours (in local vertex order, relative to local vertex 0, periodic
// neighbours translated) coincide share their operator blocks.  rep[c] is
// the first element of class c.
int assign_classes(stdg_mesh* m, std::vector<int64_t>& rep) {
    const int64_t E = m->E;
    real hmin = 1e300;
    for (int64_t t = 0; t < E; ++t)
        for (int a = 1; a < 4; ++a) hmin = std::min(hmin, norm(sub(m->vert[t][a], m->vert[t][0])));
    const real quantum = 1e-7 * hmin;
    std::map<std::vector<int64_t>, int> classes;
    rep.clear();
    m->cls.resize(E);
    auto touches_bent = [&](int64_t t) {
        if (!m->curved) return false;
        if (m->bent[t]) return true;
        for (int f = 0; f < 4; ++f)
            if (m->nbr[4 * t + f] >= 0 && m->bent[m->nbr[4 * t + f]]) return true;
        return false;
    };
    for (int64_t t = 0; t < E; ++t) {
        std::vector<int64_t> key;
        key.reserve(3 * 3 + 4 * 13);
        if (touches_bent(t)) {
            // a curved element or a neighbour of one: its blocks are its own
            key = {INT64_MAX, t};
            auto it = classes.emplace(std::move(key), (int)rep.size()).first;
            rep.push_back(t);
            m->cls[t] = it->second;
            continue;
        }
        const V3 v0 = m->vert[t][0];
        for (int a = 1; a < 4; ++a)
            for (int d = 0; d < 3; ++d) key.push_back(std::llround((m->vert[t][a][d] - v0[d]) / quantum));
        for (int f = 0; f < 4; ++f) {
            const int64_t k = m->nbr[4 * t + f];
            if (k < 0) { key.push_back(INT64_MIN); continue; }
            key.push_back(f);
            const V3 sh = neighbour_shift(m, t, f);
            for (int a = 0; a < 4; ++a)
                for (int d = 0; d < 3; ++d)
                    key.push_back(std::llround((m->vert[k][a][d] + sh[d] - v0[d]) / quantum));
        }
        auto it = classes.find(key);
        if (it == classes.end()) {
            it = classes.emplace(std::move(key), (int)rep.size()).first;
            rep.push_back(t);
        }
        m->cls[t] = it->second;
    }
    m->n_classes = (int)rep.size();
    return STDG_OK;
}

// Element order for the operator kernels: the elements of each class in
// Hilbert order, dealt out in chunks of 64 (one wavefront) round-robin over
// the classes, so that every full wavefront holds a single class and the
// chunks of all classes advance through space together; the partial
// remainder of each class goes to the end so full chunks stay aligned.
// Order faces by the classes and local faces of their two elements (interior
// faces first, then boundary faces), then by the left element.  Face
// operators are stored per (class of the left element, its local face), so
// consecutive faces share operator blocks and a wavefront of face threads
// usually reads one block set.
void sort_faces_by_class(stdg_mesh* m) {
    auto key = [&](const Face& F) {
        const int64_t cl = m->cls[F.left], cr = F.right >= 0 ? m->cls[F.right] : -1;
        return std::make_tuple(cl, F.lf, cr, F.rf, F.left);
    };
    const int64_t NI = m->n_interior;
    std::sort(m->faces.begin(), m->faces.begin() + NI,
              [&](const Face& a, const Face& b) { return key(a) < key(b); });
    std::sort(m->faces.begin() + NI, m->faces.end(), [&](const Face& a, const Face& b) { return key(a) < key(b); });
    for (int64_t j = 0; j < (int64_t)m->faces.size(); ++j) {
        const Face& F = m->faces[j];
        m->tet_face[4 * F.left + F.lf] = j;
        if (F.right >= 0) m->tet_face[4 * F.right + F.rf] = j;
    }
}

std::vector<int64_t> class_chunk_order(const stdg_mesh* m) {
    const int W = 64;
    std::vector<std::vector<int64_t>> lists(m->n_classes);
    for (int64_t t = 0; t < m->E; ++t) lists[m->cls[t]].push_back(m->perm[t]);
    std::vector<int64_t> order;
    order.reserve(m->E);
    std::vector<size_t> pos(m->n_classes, 0);
    bool more = true;
    while (more) {
        more = false;
        for (int c = 0; c < m->n_classes; ++c)
            if (pos[c] + W <= lists[c].size()) {
                order.insert(order.end(), lists[c].begin() + pos[c], lists[c].begin() + pos[c] + W);
                pos[c] += W;
                more = true;
            }
    }
    for (int c = 0; c < m->n_classes; ++c)
        order.insert(order.end(), lists[c].begin() + pos[c], lists[c].end());
    return order;
}

// Nodes of curved elements (input order [n_tet][N][3]) into internal order;
// the vertex nodes must be the vertices, and an element is bent when some
// node lies off the affine image of its reference position.
int set_geometry(stdg_mesh* m, const double* nodes) {
    const int N = m->N, p = m->p;
    const int64_t E = m->E;
    const auto ex = exponents(p);
    int vnode[4] = {0, 0, 0, 0};
    for (int k = 0; k < N; ++k) {
        if (ex[k][0] == p) vnode[1] = k;
        if (ex[k][1] == p) vnode[2] = k;
        if (ex[k][2] == p) vnode[3] = k;
    }
    m->geo.resize((size_t)E * N);
    m->bent.assign(E, 0);
    int64_t bad = -1, nbent = 0;
    for (int64_t t = 0; t < E; ++t) {
        const double* src = nodes + (size_t)m->perm[t] * N * 3;
        V3* X = m->geo.data() + (size_t)t * N;
        for (int k = 0; k < N; ++k) X[k] = {src[3 * k], src[3 * k + 1], src[3 * k + 2]};
        const auto& v = m->vert[t];
        real size = 0;
        for (int a = 1; a < 4; ++a) size = std::max(size, norm(sub(v[a], v[0])));
        for (int a = 0; a < 4; ++a)
            if (norm(sub(X[vnode[a]], v[a])) > 1e-12 * size) bad = m->perm[t];
        for (int k = 0; k < N && !m->bent[t]; ++k) {
            V3 y = v[0];
            for (int a = 1; a < 4; ++a) y = add(y, scale(sub(v[a], v[0]), (real)ex[k][a - 1] / p));
            if (norm(sub(X[k], y)) > 1e-12 * size) m->bent[t] = 1;
        }
        nbent += m->bent[t];
    }
    if (bad >= 0) {
        set_error("element " + std::to_string(bad) + ": vertex nodes do not match the vertices");
        return STDG_ERR_MESH;
    }
    m->curved = nbent > 0;
    if (!m->curved) {
        m->geo.clear();
        m->bent.clear();
    }
    return STDG_OK;
}

int build_blocks(stdg_mesh* m, const std::vector<int64_t>& rep) {
    const int N = m->N;
    m->blocks.assign((size_t)m->n_classes * 5 * N * N, 0.0);
    const NodalBasis phi(m->p);
    int bad = 0, open = 0, fold = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad, open, fold)
    for (int c = 0; c < m->n_classes; ++c) {
        const int r = element_blocks(m, rep[c], phi, m->blocks.data() + (size_t)c * 5 * N * N);
        bad += r == -1;
        open += r == -2;
        fold += r == -3;
    }
    if (open) { set_error("curved elements do not share their common face (non-conforming nodes)"); return STDG_ERR_MESH; }
    if (fold) { set_error("curved element folds (det J changes sign inside it)"); return STDG_ERR_MESH; }
    if (bad) { set_error("dual mass matrix not positive definite (degenerate dual element)"); return STDG_ERR_MESH; }
    time_factor(m->G, m->Ctime);
    return STDG_OK;
}

}  // namespace stdg
