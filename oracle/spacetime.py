"""Literal space-time matrices of the staggered DG scheme (test infrastructure only).

Everything is integrated over the space-time control volumes themselves
(space rule x time rule, dt = Delta t dtau) with the space-time basis
functions phi~ = phi(x) gamma(tau) and psi~ = psi(x) gamma(tau) of Sec. 2.3;
no tensor-product factorisation is used.  A space-time index is
a * N + k (time node a, spatial function k).

Per interior face j (dual element H_j = T_{l,j} u T_{r,j}, Sec. 2.2.1):
  M_j^+, M_j^o, M_j = M_j^+ - M_j^o          eq. MD_2, MD_2_2 and Sec. 2.4
  Mbar_j = int_{H_j^st} psi~ psi~            eq. mj
  Q_{i,j}  (3 components)                    eq. MD_6 with sigma of eq. SD_1
  D_{i,j}  (3 components)                    eq. MD_3
  M_{i,j} = int_{T_ij^st} phi~ psi~          eq. vis3
Per element i:
  M_i = int_{T_i^st} phi~ phi~               eq. vis3
  Mbar_i^+, Mbar_i^-, Mbar_i^o               eq. vis11
Boundary faces have the single sub-tetrahedron as dual element.

Dual basis (eq. bf_2): x0 = volume centroid of H_j, h = half the largest
distance between two vertices of H_j (the paper leaves both open; with half
the diameter the scaled coordinates lie in [-1, 1], which keeps the degree-4
dual mass matrices an order of magnitude better conditioned than the full
diameter does).
"""

import numpy as np

from .basis import NodalBasis, TaylorBasis, TimeBasis, TetMap, nodal_phys
from .linalg import REAL, asreal, norm
from .quadrature import simplex_rule, triangle_rule_3d, gauss_legendre_01


def st_outer(sv, tv):
    """Space-time basis values from spatial (m, N) and time (t, G) values.

    Returns (m, t, G*N) with index a*N + k.
    """
    m, N = sv.shape
    t, G = tv.shape
    return (tv[None, :, :, None] * sv[:, None, None, :]).reshape(m, t, G * N)


class SpaceTimeOperators:
    """Literal space-time matrices for one mesh, degree (p, p_gamma), step dt."""

    def __init__(self, mesh, p, p_gamma, dt):
        self.mesh = mesh
        self.p = p
        self.G = p_gamma + 1
        self.dt = REAL(dt)
        self.phi = NodalBasis(p)
        self.N = self.phi.N
        self.Nst = self.N * self.G
        self.tb = TimeBasis(self.G)
        # exact for the space degree 2p and time degree 2 p_gamma integrands
        self.s_space = p
        self.tau, self.wtau = gauss_legendre_01(self.G + 1)
        self._face_cache = {}
        self._tet_cache = {}

    # ------------------------------------------------------------------
    def dual_basis(self, j):
        """Taylor basis of face j's dual element (in the left element's frame)."""
        mesh = self.mesh
        subs = [mesh.subtet(j, 0)]
        if mesh.right[j] >= 0:
            subs.append(mesh.subtet(j, 1))
        vols = np.array([TetMap(s).volume() for s in subs])
        cents = np.array([s.mean(axis=0) for s in subs])
        x0 = (vols[:, None] * cents).sum(axis=0) / vols.sum()
        pts = np.vstack([asreal(mesh.face_vertices(j))] + [s[3:4] for s in subs])
        h = REAL(0.5) * max(norm(a - b) for a in pts for b in pts)
        return TaylorBasis(self.p, x0, h)

    def face(self, j):
        """Dictionary of the literal space-time matrices of face j."""
        if j in self._face_cache:
            return self._face_cache[j]
        mesh = self.mesh
        dt = self.dt
        psi = self.dual_basis(j)
        n_j = mesh.normal(j)                        # from left to right
        P = mesh.face_vertices(j)
        sides = [0] + ([1] if mesh.right[j] >= 0 else [])
        tv = self.tb.eval(self.tau)                 # (t, G)
        td = self.tb.deriv(self.tau)
        t1 = self.tb.eval(1.0)                      # (1, G)
        out = {"sides": sides, "psi": psi, "normal": n_j}
        Nst = self.Nst
        Mplus = np.zeros((Nst, Nst), dtype=REAL)
        Mcirc = np.zeros((Nst, Nst), dtype=REAL)
        Mbar = np.zeros((Nst, Nst), dtype=REAL)
        fq, fw = triangle_rule_3d(P, self.s_space)
        for s in sides:
            i = mesh.left[j] if s == 0 else mesh.right[j]
            sigma = 1.0 if s == 0 else -1.0         # eq. SD_1: +1 left, -1 right
            tmap = TetMap(mesh.side_vertices(j, s))
            xq, wq = simplex_rule(mesh.subtet(j, s), self.s_space)
            ps = psi.eval(xq)                       # (m, N)
            ph, gph = nodal_phys(self.phi, tmap, xq)
            PS = st_outer(ps, tv)                   # (m, t, Nst)
            PH = st_outer(ph, tv)
            W = wq[:, None] * self.wtau[None, :] * dt          # dx dt
            # mass matrices over the sub-tetrahedron, accumulated over H_j
            PS1 = st_outer(ps, t1)[:, 0, :]
            Mplus += np.einsum("m,mk,ml->kl", wq, PS1, PS1)
            dPS = st_outer(ps, td) / dt             # d/dt psi~
            Mcirc += np.einsum("mt,mtk,mtl->kl", W, dPS, PS)
            Mbar += np.einsum("mt,mtk,mtl->kl", W, PS, PS)
            Mij = np.einsum("mt,mtk,mtl->kl", W, PH, PS)       # phi~ x psi~
            # volume parts of Q and D
            Q = np.zeros((3, Nst, Nst), dtype=REAL)
            D = np.zeros((3, Nst, Nst), dtype=REAL)
            for d in range(3):
                GPH = st_outer(gph[:, :, d], tv)
                Q[d] += np.einsum("mt,mtk,mtl->kl", W, PS, GPH)
                D[d] -= np.einsum("mt,mtk,mtl->kl", W, GPH, PS)
            # face parts on Gamma_j^st
            fps = psi.eval(fq)
            fph, _ = nodal_phys(self.phi, tmap, fq)
            FPS = st_outer(fps, tv)
            FPH = st_outer(fph, tv)
            FW = fw[:, None] * self.wtau[None, :] * dt
            n_ij = sigma * n_j                      # outward normal of T_i
            face_psph = np.einsum("mt,mtk,mtl->kl", FW, FPS, FPH)
            out[("Qvol", s)] = Q.copy()             # volume part only
            for d in range(3):
                Q[d] -= face_psph * sigma * n_j[d]
                D[d] += face_psph.T * n_ij[d]
            out[("Q", s)] = Q
            out[("D", s)] = D
            out[("Mij", s)] = Mij
            out[("elem", s)] = i
        out["Mplus"] = Mplus
        out["Mcirc"] = Mcirc
        out["M"] = Mplus - Mcirc
        out["Mbar"] = Mbar
        self._face_cache[j] = out
        return out

    def tet(self, i):
        """Element matrices M_i, Mbar_i^+, Mbar_i^-, Mbar_i^o of eq. vis3/vis11."""
        if i in self._tet_cache:
            return self._tet_cache[i]
        v = self.mesh.tet_vertices(i)
        tmap = TetMap(v)
        xq, wq = simplex_rule(v, self.s_space)
        ph, _ = nodal_phys(self.phi, tmap, xq)
        tv = self.tb.eval(self.tau)
        td = self.tb.deriv(self.tau)
        t0 = self.tb.eval(0.0)
        t1 = self.tb.eval(1.0)
        PH = st_outer(ph, tv)
        W = wq[:, None] * self.wtau[None, :] * self.dt
        Mi = np.einsum("mt,mtk,mtl->kl", W, PH, PH)
        P1 = st_outer(ph, t1)[:, 0, :]
        P0 = st_outer(ph, t0)[:, 0, :]
        Mp = np.einsum("m,mk,ml->kl", wq, P1, P1)
        Mm = np.einsum("m,mk,ml->kl", wq, P0, P1)   # test at t^n, trial at end of slab n
        dPH = st_outer(ph, td) / self.dt
        Mo = np.einsum("mt,mtk,mtl->kl", W, dPH, PH)
        out = {"M": Mi, "Mbar_plus": Mp, "Mbar_minus": Mm, "Mbar_o": Mo,
               "Mbar": Mp - Mo}
        self._tet_cache[i] = out
        return out
