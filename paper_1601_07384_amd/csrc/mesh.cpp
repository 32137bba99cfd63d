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
        dual_face_blocks(phi, m->p, m->vert[t], f, Vk, fb);
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
    for (int64_t t = 0; t < E; ++t) {
        std::vector<int64_t> key;
        key.reserve(3 * 3 + 4 * 13);
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

int build_blocks(stdg_mesh* m, const std::vector<int64_t>& rep) {
    const int N = m->N;
    m->blocks.assign((size_t)m->n_classes * 5 * N * N, 0.0);
    const NodalBasis phi(m->p);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int c = 0; c < m->n_classes; ++c)
        if (element_blocks(m, rep[c], phi, m->blocks.data() + (size_t)c * 5 * N * N) != 0) bad++;
    if (bad) { set_error("dual mass matrix not positive definite (degenerate dual element)"); return STDG_ERR_MESH; }
    time_factor(m->G, m->Ctime);
    return STDG_OK;
}

}  // namespace stdg
