// Host precompute of the Picard-step tables (Sec. 2.5-2.6), per element class
// and local face, in extended precision.  With the tensor-product space-time
// basis every matrix of the step factors as (spatial) x (time):
//   average   M_i^-1 M_ij          = (Mi^-1 Mij)^sp (x) I          (eq. average)
//   goback    Mbar_j^-1 M_ij^T     = (Mj^-1 Mij^T)^sp (x) I        (eq. goback)
//   gradient  M_j^-1 Q_ij          = dt (Mj^-1 Qij)^sp (x) T^-1 W  (eqs. prevpress, A3_mod)
//   rhs       -D_ij = Q_ij^T       = dt (Qij^T)^sp (x) W           (eq. A2_mod)
//   viscous   -nu D Mbar^-1 Q      = nu dt (Q^T Mj^-1 Q)^sp (x) W  (eq. A1_mod)
//   masses    Mbar_i = Mi (x) T,  Mbar_i^- = Mi (x) g(0) g(1)^T
// so only N x N spatial blocks and G x G time matrices are stored.
//
// Boundary (Dirichlet) faces: the dual element is the single sub-tetrahedron;
// its gradient block keeps the volume part only (no jump against the wall) and
// is used for Lambda alone; BB = sum_d n_d Qd^T Mj^-1 K, K = int_Gamma psi psi,
// carries the Dirichlet data into the viscous right-hand side.
//
// Convection tables (eq. convdg): element Jacobians, outward normals, and for
// each face the values of the element's own and of the neighbour's basis
// (boundary: of the boundary dual basis) at the points of the face rule,
// q = ceil((3p+2)/2) collapsed Gauss-Jacobi points per direction on the face
// with its vertices sorted lexicographically by coordinates (the same points
// seen from both sides); the volume rule is exact for degree 3p - 1.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace stdg {

namespace {

struct FaceData {
    std::vector<real> M, Mij, Q[2], Qvol, K;   // dual mass, mixed mass (own side), gradients
    V3 x0, n;
    real h = 0;
};

// Dual element of local face f of an element with vertices Vt; Vk = the
// neighbour's vertices (translated next to t) or nullptr on a boundary face.
void face_data(const NodalBasis& phi, int p, const std::array<V3, 4>& Vt, int f,
               const std::array<V3, 4>* Vk, FaceData& o) {
    const int N = phi.N;
    const auto ex = exponents(p);
    const int ns = Vk ? 2 : 1;
    V3 P[3];
    for (int k = 0, m = 0; k < 4; ++k)
        if (k != f) P[m++] = Vt[k];
    V3 bc[2] = {centroid(Vt), Vk ? centroid(*Vk) : V3{0, 0, 0}};
    real vol[2] = {0, 0};
    V3 cen[2];
    for (int s = 0; s < ns; ++s) {
        vol[s] = std::fabs(det3(sub(P[0], bc[s]), sub(P[1], bc[s]), sub(P[2], bc[s]))) / 6;
        cen[s] = scale(add(add(P[0], P[1]), add(P[2], bc[s])), 0.25L);
    }
    o.x0 = ns == 2 ? scale(add(scale(cen[0], vol[0]), scale(cen[1], vol[1])), 1 / (vol[0] + vol[1])) : cen[0];
    std::vector<V3> pts = {P[0], P[1], P[2], bc[0]};
    if (ns == 2) pts.push_back(bc[1]);
    o.h = 0;
    for (size_t a = 0; a < pts.size(); ++a)
        for (size_t b = a + 1; b < pts.size(); ++b) o.h = std::max(o.h, 0.5L * norm(sub(pts[a], pts[b])));
    o.n = cross(sub(P[1], P[0]), sub(P[2], P[0]));
    o.n = scale(o.n, 1 / norm(o.n));
    if (dot(o.n, sub(P[0], bc[0])) < 0) o.n = scale(o.n, -1);
    o.M.assign(N * N, 0);
    o.Mij.assign(N * N, 0);
    o.K.assign(N * N, 0);
    for (int s = 0; s < 2; ++s) o.Q[s].assign(3 * N * N, 0);
    const Affine A0(Vt);
    const Affine A1(Vk ? *Vk : Vt);
    const Affine* A[2] = {&A0, &A1};
    const int q = p + 1;
    const Rule& tr = tet_rule(q);
    std::vector<real> ps(N), ph(N), gr(3 * N), gx(3 * N);
    for (int s = 0; s < ns; ++s) {
        std::array<V3, 4> sv = {bc[s], P[0], P[1], P[2]};
        Affine sa(sv);
        const real jac = std::fabs(sa.det);
        for (size_t m = 0; m < tr.w.size(); ++m) {
            V3 x = sa.to_phys(tr.pts[m]);
            const real w = tr.w[m] * jac;
            taylor_eval(ex, x, o.x0, o.h, ps.data());
            V3 xi = A[s]->to_ref(x);
            phi.eval(xi, ph.data());
            phi.grad(xi, gr.data());
            for (int k = 0; k < N; ++k)
                for (int d = 0; d < 3; ++d)
                    gx[3 * k + d] = A[s]->Jinv[0 * 3 + d] * gr[3 * k + 0] + A[s]->Jinv[1 * 3 + d] * gr[3 * k + 1] +
                                    A[s]->Jinv[2 * 3 + d] * gr[3 * k + 2];
            for (int a = 0; a < N; ++a) {
                const real wa = w * ps[a];
                for (int b = 0; b < N; ++b) o.M[a * N + b] += wa * ps[b];
                for (int d = 0; d < 3; ++d)
                    for (int b = 0; b < N; ++b) o.Q[s][(d * N + a) * N + b] += wa * gx[3 * b + d];
                if (s == 0)
                    for (int b = 0; b < N; ++b) o.Mij[b * N + a] += wa * ph[b];   // rows phi, cols psi
            }
        }
    }
    o.Qvol = o.Q[0];
    const Rule& fr = tri_rule(q);
    const V3 e1 = sub(P[1], P[0]), e2 = sub(P[2], P[0]);
    const real area2 = norm(cross(e1, e2));
    for (size_t m = 0; m < fr.w.size(); ++m) {
        V3 x = add(P[0], add(scale(e1, fr.pts[m][0]), scale(e2, fr.pts[m][1])));
        const real w = fr.w[m] * area2;
        taylor_eval(ex, x, o.x0, o.h, ps.data());
        for (int a = 0; a < N; ++a)
            for (int b = 0; b < N; ++b) o.K[a * N + b] += w * ps[a] * ps[b];
        for (int s = 0; s < ns; ++s) {
            phi.eval(A[s]->to_ref(x), ph.data());
            const real sg = (s == 0) ? 1 : -1;
            for (int a = 0; a < N; ++a)
                for (int d = 0; d < 3; ++d) {
                    const real c = w * ps[a] * sg * o.n[d];
                    for (int b = 0; b < N; ++b) o.Q[s][(d * N + a) * N + b] -= c * ph[b];
                }
        }
    }
}

void matmul(int n, const real* A, const real* B, real* C) {   // C = A B (n x n)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            real s = 0;
            for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
            C[i * n + j] = s;
        }
}

void solve_spd(int n, const std::vector<real>& M, real* B, int nrhs) {   // B <- M^-1 B (n x nrhs)
    std::vector<real> L = M;
    cholesky(n, L);
    cholesky_solve(n, L, B, nrhs, nrhs);
}

void store(std::vector<double>& dst, size_t off, const real* src, size_t n) {
    for (size_t i = 0; i < n; ++i) dst[off + i] = (double)src[i];
}

}  // namespace

int build_picard_tables(stdg_mesh* m, const std::vector<int64_t>& rep) {
    const int N = m->N, G = m->G, C = m->n_classes, p = m->p;
    PicardTables& t = m->pt;
    const size_t NN = (size_t)N * N;
    t.A.assign((size_t)C * 4 * NN, 0);
    t.GB.assign((size_t)C * 4 * NN, 0);
    t.QT.assign((size_t)C * 4 * 3 * NN, 0);
    t.US.assign((size_t)C * 4 * 3 * NN, 0);
    t.UN.assign((size_t)C * 4 * 3 * NN, 0);
    t.BB.assign((size_t)C * 4 * NN, 0);
    t.SV.assign((size_t)C * 5 * NN, 0);
    t.MI.assign((size_t)C * NN, 0);
    t.qs = (3 * p + 3) / 2;
    t.qt = (3 * (G - 1) + 3) / 2;
    t.qv = (3 * p + 1) / 2;                      // collapsed rule exact for degree 3p - 1
    t.nqf = t.qs * t.qs;
    t.nqv = t.qv * t.qv * t.qv;
    t.cJinv.assign((size_t)C * 9, 0);
    t.cdet.assign(C, 0);
    t.cnrm.assign((size_t)C * 12, 0);
    t.PHf.assign((size_t)C * 4 * t.nqf * N, 0);
    t.PHn.assign((size_t)C * 4 * t.nqf * N, 0);
    t.FW.assign((size_t)C * 4 * t.nqf, 0);
    const NodalBasis phi(p);
    // reference volume rule and tables
    {
        const Rule& vr = tet_rule(t.qv);
        t.PHv.assign((size_t)t.nqv * N, 0);
        t.dPHv.assign((size_t)t.nqv * N * 3, 0);
        t.wv.assign(t.nqv, 0);
        std::vector<real> v(N), g(3 * N);
        for (int q = 0; q < t.nqv; ++q) {
            phi.eval(vr.pts[q], v.data());
            phi.grad(vr.pts[q], g.data());
            store(t.PHv, (size_t)q * N, v.data(), N);
            store(t.dPHv, (size_t)q * N * 3, g.data(), 3 * N);
            t.wv[q] = (double)vr.w[q];
        }
    }
    const Rule& fr = tri_rule(t.qs);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int c = 0; c < C; ++c) {
        const int64_t e = rep[c];
        const auto& Vt = m->vert[e];
        const Affine At(Vt);
        std::vector<real> Mi(NN, 0), tmp(NN), tmp3(3 * NN), SV0(NN, 0), SVk(NN);
        {   // element mass
            const Rule& tr = tet_rule(p + 1);
            std::vector<real> ph(N);
            const real jac = std::fabs(At.det);
            for (size_t q = 0; q < tr.w.size(); ++q) {
                phi.eval(tr.pts[q], ph.data());
                for (int a = 0; a < N; ++a)
                    for (int b = 0; b < N; ++b) Mi[a * N + b] += tr.w[q] * jac * ph[a] * ph[b];
            }
        }
        store(t.MI, (size_t)c * NN, Mi.data(), NN);
        for (int k = 0; k < 9; ++k) t.cJinv[(size_t)c * 9 + k] = (double)At.Jinv[k];
        t.cdet[c] = (double)std::fabs(At.det);
        for (int f = 0; f < 4; ++f) {
            const int64_t k = m->nbr[4 * e + f];
            std::array<V3, 4> Vk;
            if (k >= 0) {
                const V3 sh = neighbour_shift(m, e, f);
                Vk = m->vert[k];
                for (auto& v : Vk) v = add(v, sh);
            }
            FaceData fd;
            face_data(phi, p, Vt, f, k >= 0 ? &Vk : nullptr, fd);
            const size_t o1 = ((size_t)c * 4 + f) * NN, o3 = ((size_t)c * 4 + f) * 3 * NN;
            // average: Mi^-1 Mij
            tmp = fd.Mij;
            solve_spd(N, Mi, tmp.data(), N);
            store(t.A, o1, tmp.data(), NN);
            // goback: Mj^-1 Mij^T
            for (int a = 0; a < N; ++a)
                for (int b = 0; b < N; ++b) tmp[a * N + b] = fd.Mij[b * N + a];
            solve_spd(N, fd.M, tmp.data(), N);
            store(t.GB, o1, tmp.data(), NN);
            for (int d = 0; d < 3; ++d) {
                // Q^T (rows phi, cols psi)
                for (int a = 0; a < N; ++a)
                    for (int b = 0; b < N; ++b) tmp3[(d * N + a) * N + b] = fd.Q[0][(d * N + b) * N + a];
            }
            store(t.QT, o3, tmp3.data(), 3 * NN);
            // dual-grid gradients Mj^-1 Q (self: full, or volume part on a boundary face)
            std::vector<real> Zs = (k >= 0) ? fd.Q[0] : fd.Qvol, Zn = fd.Q[1];
            for (int d = 0; d < 3; ++d) {
                solve_spd(N, fd.M, Zs.data() + d * NN, N);
                if (k >= 0) solve_spd(N, fd.M, Zn.data() + d * NN, N);
            }
            store(t.US, o3, Zs.data(), 3 * NN);
            if (k >= 0) store(t.UN, o3, Zn.data(), 3 * NN);
            // viscous stiffness: Q^T Mj^-1 Q (all faces into the diagonal block)
            std::vector<real> Zf = fd.Q[0];
            for (int d = 0; d < 3; ++d) solve_spd(N, fd.M, Zf.data() + d * NN, N);
            std::fill(SVk.begin(), SVk.end(), 0);
            for (int d = 0; d < 3; ++d)
                for (int a = 0; a < N; ++a)
                    for (int cc = 0; cc < N; ++cc) {
                        const real qa = fd.Q[0][(d * N + cc) * N + a];
                        for (int b = 0; b < N; ++b) {
                            SV0[a * N + b] += qa * Zf[(d * N + cc) * N + b];
                            if (k >= 0) SVk[a * N + b] += qa * Zn[(d * N + cc) * N + b];
                        }
                    }
            if (k >= 0) store(t.SV, ((size_t)c * 5 + 1 + f) * NN, SVk.data(), NN);
            if (k < 0) {   // BB = sum_d n_d Qd^T Mj^-1 K
                std::vector<real> MK = fd.K;
                solve_spd(N, fd.M, MK.data(), N);
                std::fill(tmp.begin(), tmp.end(), 0);
                for (int d = 0; d < 3; ++d)
                    for (int a = 0; a < N; ++a)
                        for (int cc = 0; cc < N; ++cc) {
                            const real qa = fd.Q[0][(d * N + cc) * N + a] * fd.n[d];
                            for (int b = 0; b < N; ++b) tmp[a * N + b] += qa * MK[cc * N + b];
                        }
                store(t.BB, o1, tmp.data(), NN);
            }
            // convection: face points (vertices sorted lexicographically)
            V3 P[3];
            for (int kk = 0, mm = 0; kk < 4; ++kk)
                if (kk != f) P[mm++] = Vt[kk];
            std::sort(P, P + 3, [](const V3& a, const V3& b) {
                return a[0] != b[0] ? a[0] < b[0] : (a[1] != b[1] ? a[1] < b[1] : a[2] < b[2]);
            });
            const V3 e1 = sub(P[1], P[0]), e2 = sub(P[2], P[0]);
            const real area2 = norm(cross(e1, e2));
            for (int d = 0; d < 3; ++d) t.cnrm[(size_t)c * 12 + f * 3 + d] = (double)fd.n[d];
            const Affine Ak(k >= 0 ? Vk : Vt);
            const auto ex = exponents(p);
            std::vector<real> v(N);
            for (int q = 0; q < t.nqf; ++q) {
                V3 x = add(P[0], add(scale(e1, fr.pts[q][0]), scale(e2, fr.pts[q][1])));
                t.FW[((size_t)c * 4 + f) * t.nqf + q] = (double)(fr.w[q] * area2);
                phi.eval(At.to_ref(x), v.data());
                store(t.PHf, (((size_t)c * 4 + f) * t.nqf + q) * N, v.data(), N);
                if (k >= 0) phi.eval(Ak.to_ref(x), v.data());
                else taylor_eval(ex, x, fd.x0, fd.h, v.data());
                store(t.PHn, (((size_t)c * 4 + f) * t.nqf + q) * N, v.data(), N);
            }
        }
        store(t.SV, (size_t)c * 5 * NN, SV0.data(), NN);
    }
    if (bad) { set_error("Picard tables failed"); return STDG_ERR_MESH; }
    // time matrices
    TimeBasis tb(G);
    std::vector<real> xq, wq;
    gauss_legendre01(G + 1, xq, wq);
    std::vector<real> T(G * G), Ti, Wd(G);
    t.Tm.assign(G * G, 0); t.TW.assign(G * G, 0); t.W.assign(G, 0); t.g0g1.assign(G * G, 0); t.g1.assign(G, 0);
    for (int a = 0; a < G; ++a) {
        Wd[a] = tb.weights[a];
        t.W[a] = (double)Wd[a];
        t.g1[a] = (double)tb.eval(a, 1);
        for (int b = 0; b < G; ++b) {
            real s = 0;
            for (size_t q = 0; q < xq.size(); ++q) s += wq[q] * tb.deriv(a, xq[q]) * tb.eval(b, xq[q]);
            T[a * G + b] = tb.eval(a, 1) * tb.eval(b, 1) - s;
            t.g0g1[a * G + b] = (double)(tb.eval(a, 0) * tb.eval(b, 1));
        }
    }
    for (int i = 0; i < G * G; ++i) t.Tm[i] = (double)T[i];
    Ti = T;
    lu_inverse(G, Ti);
    for (int a = 0; a < G; ++a)
        for (int b = 0; b < G; ++b) t.TW[a * G + b] = (double)(Ti[a * G + b] * Wd[b]);
    // inverse of the viscous diagonal block D = MI (x) T + nu dt SV0 (x) W per class
    {
        const int NG = N * G;
        const real nudt = (real)m->cfg.nu * (real)m->cfg.dt;
        t.DV.assign((size_t)C * NG * NG, 0);
        int badv = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : badv)
        for (int c = 0; c < C; ++c) {
            std::vector<real> D((size_t)NG * NG, 0);
            for (int a = 0; a < G; ++a)
                for (int r = 0; r < N; ++r)
                    for (int b = 0; b < G; ++b)
                        for (int mm = 0; mm < N; ++mm) {
                            real v = (real)t.MI[(size_t)c * NN + r * N + mm] * T[a * G + b];
                            if (a == b) v += nudt * (real)t.SV[(size_t)c * 5 * NN + r * N + mm] * Wd[a];
                            D[(size_t)(a * N + r) * NG + b * N + mm] = v;
                        }
            if (!lu_inverse(NG, D)) { badv++; continue; }
            for (int row = 0; row < NG; ++row)
                for (int col = 0; col < NG; ++col)
                    t.DV[(size_t)c * NG * NG + (size_t)col * NG + row] = (double)D[(size_t)row * NG + col];
        }
        if (badv) { set_error("singular viscous diagonal block"); return STDG_ERR_MESH; }
    }
    // convection time rule
    std::vector<real> tq, tw;
    gauss_legendre01(t.qt, tq, tw);
    t.tq.assign(t.qt, 0); t.tw.assign(t.qt, 0); t.gq.assign((size_t)t.qt * G, 0);
    for (int q = 0; q < t.qt; ++q) {
        t.tq[q] = (double)tq[q];
        t.tw[q] = (double)tw[q];
        for (int b = 0; b < G; ++b) t.gq[(size_t)q * G + b] = (double)tb.eval(b, tq[q]);
    }
    return STDG_OK;
}

}  // namespace stdg
