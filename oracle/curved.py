"""Curved isoparametric elements of Sec. 2.8 (test infrastructure only).

Reading of Sec. 2.8 (the paper describes the construction in words only):

* Element i is the image of the reference tetrahedron under the
  isoparametric map x_i(xi) = sum_k X_ik phi_k(xi), with phi the degree-p
  nodal basis of the pressure (eq. bf_1) and X_ik the element's N nodes.
  Its basis functions are phi_k(xi(x)); physical gradients are
  J^-T grad_xi phi with J = dx/dxi.
* The sub-tetrahedron T_ij of the dual element H_j = T_lj u T_rj is the image
  under x_i of the straight reference sub-tetrahedron spanned by the
  reference face and the reference barycentre, so the curved sub-tetrahedra
  of an element tile it exactly; the face Gamma_j is the image of the
  reference face, the same surface from both sides (the face nodes are
  shared), met at equal barycentric coordinates of the face's vertices.
* The dual (Taylor) basis stays a polynomial basis in physical coordinates
  (eq. bf_2), centred and scaled as on straight faces with the element
  barycentres replaced by their images x_i(1/4, 1/4, 1/4); S does not depend
  on that choice.

Every integral is taken in reference coordinates: dx = |det J| dxi, and on
the face n dS = (t_u x t_v) du dv with t_u, t_v the images of the reference
face edges, oriented out of the left element.  In this form each integrand
is a polynomial in xi (det J and the cofactor matrix det J J^-T are
polynomials), of degree at most 2 p^2 + 3 (p - 1) (the dual mass matrix), so
Grundmann-Moeller rules of that degree integrate them exactly.

Only the pressure system is provided (the matrices M_j, Q_ij, D_ij of
eqs. MD_2, MD_3, MD_6 that ``pressure.apply_S`` and ``pressure.assemble_S``
use), as the same literal space-time integrals as ``spacetime.py``.
"""

import numpy as np

from .basis import NodalBasis, TaylorBasis, nodal_points
from .linalg import REAL, asreal, det3, inv, norm
from .mesh import Mesh
from .quadrature import grundmann_moeller, simplex_rule
from .spacetime import SpaceTimeOperators, st_outer

REF_VERTS = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=REAL)
REF_BARY = np.full(3, REAL(1) / 4)


def exact_orders(p):
    """Grundmann-Moeller s (exact for degree 2s+1) for volume and face integrands.

    Volume: the dual mass integrand psi psi |det J| has degree 2p^2 + 3(p-1),
    the highest of the volume integrands.  Face: psi phi (t_u x t_v) has degree
    p^2 + p + 2(p-1).
    """
    dv = 2 * p * p + 3 * (p - 1)
    df = p * p + p + 2 * (p - 1)
    return max(0, (dv) // 2), max(0, (df) // 2)


class IsoMesh(Mesh):
    """Mesh whose elements carry N isoparametric nodes each (E, N, 3)."""

    def __init__(self, X, tets, nodes, p, periodic=False, box_lo=(0, 0, 0), box_hi=(1, 1, 1)):
        super().__init__(X, tets, periodic, box_lo, box_hi)
        self.p = p
        self.basis = NodalBasis(p)
        self.nodes = asreal(nodes)
        if self.nodes.shape != (self.E, self.basis.N, 3):
            raise ValueError("nodes must be (E, N, 3)")
        # the nodes at the reference vertices are the element's vertices
        ref = nodal_points(p)
        for v in range(4):
            k = int(np.argmin(np.abs(ref - REF_VERTS[v]).sum(axis=1)))
            if np.abs(self.nodes[:, k, :] - asreal(self.X[self.tets[:, v]])).max() > 1e-12:
                raise ValueError("vertex nodes do not match the vertices")

    def x(self, t, xi):
        """Physical points (m, 3) of element t at reference points xi (m, 3)."""
        return self.basis.eval(xi) @ self.nodes[t]

    def jac(self, t, xi):
        """J (m, 3, 3) with J[m, r, c] = d x_r / d xi_c."""
        g = self.basis.grad_ref(xi)                          # (m, N, 3)
        return np.einsum("kr,mkc->mrc", self.nodes[t], g)

    def face_ref_vertices(self, j, side):
        """Reference coordinates (3, 3) of face j's vertices in element l(j)
        (side 0) or r(j) (side 1), in the same vertex order for both sides."""
        canon = self._canon
        lt, lf = self.left[j], self.left_face[j]
        lverts = [k for k in range(4) if k != lf]
        if side == 0:
            return REF_VERTS[lverts]
        rt = self.right[j]
        rlocal = [int(np.nonzero(canon[self.tets[rt]] == canon[self.tets[lt, k]])[0][0]) for k in lverts]
        return REF_VERTS[rlocal]

    @property
    def _canon(self):
        if not hasattr(self, "_canon_cache"):
            self._canon_cache = self._canonical_vertex()
        return self._canon_cache


def _mat_inv_batch(J):
    return np.stack([inv(Jm) for Jm in J])


class CurvedSpaceTimeOperators(SpaceTimeOperators):
    """Literal space-time pressure matrices on an ``IsoMesh``."""

    def __init__(self, mesh, p, p_gamma, dt):
        if mesh.p != p:
            raise ValueError("isoparametric: the node degree is the pressure degree")
        super().__init__(mesh, p, p_gamma, dt)
        self.s_vol, self.s_face = exact_orders(p)

    def _side_shift(self, j, side):
        return np.zeros(3, dtype=REAL) if side == 0 else asreal(self.mesh.offset[j])

    def dual_basis(self, j):
        """Taylor basis of face j's dual element, centred as on straight faces
        with the barycentres replaced by their images."""
        mesh = self.mesh
        P = asreal(mesh.face_vertices(j))
        sides = [0] + ([1] if mesh.right[j] >= 0 else [])
        bc, vols, cents = [], [], []
        for s in sides:
            i = mesh.left[j] if s == 0 else mesh.right[j]
            b = mesh.x(i, REF_BARY[None, :])[0] + self._side_shift(j, s)
            sub = np.vstack([P, b[None, :]])
            vols.append(abs(det3((sub[1:] - sub[0]).T)) / 6)
            cents.append(sub.mean(axis=0))
            bc.append(b)
        vols = np.array(vols, dtype=REAL)
        x0 = (vols[:, None] * np.array(cents, dtype=REAL)).sum(axis=0) / vols.sum()
        pts = [P[0], P[1], P[2]] + bc
        h = REAL(0.5) * max(norm(a - b) for a in pts for b in pts)
        return TaylorBasis(self.p, x0, h)

    def face(self, j):
        """The literal space-time pressure matrices of face j (curved)."""
        if j in self._face_cache:
            return self._face_cache[j]
        mesh = self.mesh
        dt = self.dt
        psi = self.dual_basis(j)
        sides = [0] + ([1] if mesh.right[j] >= 0 else [])
        tv = self.tb.eval(self.tau)
        td = self.tb.deriv(self.tau)
        t1 = self.tb.eval(1.0)
        Nst = self.Nst
        out = {"sides": sides, "psi": psi}
        Mplus = np.zeros((Nst, Nst), dtype=REAL)
        Mcirc = np.zeros((Nst, Nst), dtype=REAL)
        Mbar = np.zeros((Nst, Nst), dtype=REAL)
        refs = {s: mesh.face_ref_vertices(j, s) for s in sides}
        elem = {s: (mesh.left[j] if s == 0 else mesh.right[j]) for s in sides}

        # face rule on the reference face of the left element; the same
        # barycentric coordinates give the point in the right element
        uv, fw = grundmann_moeller(2, self.s_face)
        lam = np.stack([1 - uv[:, 0] - uv[:, 1], uv[:, 0], uv[:, 1]], axis=1)
        fxi = {s: lam @ refs[s] for s in sides}
        fx = mesh.x(elem[0], fxi[0])
        if 1 in sides:
            other = mesh.x(elem[1], fxi[1]) + self._side_shift(j, 1)
            if np.abs(other - fx).max() > 1e-9 * (1 + np.abs(fx).max()):
                raise ValueError(f"face {j}: the two elements do not share the curved face")
        J0 = mesh.jac(elem[0], fxi[0])
        tu = J0 @ (refs[0][1] - refs[0][0])
        tv_ = J0 @ (refs[0][2] - refs[0][0])
        area = np.stack([tu[:, 1] * tv_[:, 2] - tu[:, 2] * tv_[:, 1],
                         tu[:, 2] * tv_[:, 0] - tu[:, 0] * tv_[:, 2],
                         tu[:, 0] * tv_[:, 1] - tu[:, 1] * tv_[:, 0]], axis=1)
        # outward of the left element: along J^-T n_ref (n_ref away from the
        # opposite vertex), which is outward whatever the sign of det J
        lf = mesh.left_face[j]
        e1, e2 = refs[0][1] - refs[0][0], refs[0][2] - refs[0][0]
        nref = np.array([e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                         e1[0] * e2[1] - e1[1] * e2[0]], dtype=REAL)
        if nref @ (refs[0][0] - REF_VERTS[lf]) < 0:
            nref = -nref
        Jit = np.transpose(_mat_inv_batch(J0), (0, 2, 1))
        sgn = np.sign(np.einsum("md,md->m", area, Jit @ nref))
        area = area * sgn[:, None]                          # n dS / (du dv), outward of l(j)
        fps = psi.eval(fx)
        FPS = st_outer(fps, tv)
        FWt = fw[:, None] * self.wtau[None, :] * dt

        for s in sides:
            i = elem[s]
            sigma = REAL(1) if s == 0 else REAL(-1)         # eq. SD_1
            sub = np.vstack([refs[s], REF_BARY[None, :]])
            xi, w = simplex_rule(sub, self.s_vol)           # reference sub-tetrahedron
            J = mesh.jac(i, xi)
            dJ = np.array([det3(Jm) for Jm in J])
            Jinv = _mat_inv_batch(J)
            wq = w * np.abs(dJ)
            x = mesh.x(i, xi) + self._side_shift(j, s)
            ps = psi.eval(x)
            ph = self.phi.eval(xi)
            gph = np.einsum("mcr,mkc->mkr", Jinv, self.phi.grad_ref(xi))   # J^-T grad_xi
            PS = st_outer(ps, tv)
            PH = st_outer(ph, tv)
            W = wq[:, None] * self.wtau[None, :] * dt
            PS1 = st_outer(ps, t1)[:, 0, :]
            Mplus += np.einsum("m,mk,ml->kl", wq, PS1, PS1)
            dPS = st_outer(ps, td) / dt
            Mcirc += np.einsum("mt,mtk,mtl->kl", W, dPS, PS)
            Mbar += np.einsum("mt,mtk,mtl->kl", W, PS, PS)
            Q = np.zeros((3, Nst, Nst), dtype=REAL)
            D = np.zeros((3, Nst, Nst), dtype=REAL)
            for d in range(3):
                GPH = st_outer(gph[:, :, d], tv)
                Q[d] += np.einsum("mt,mtk,mtl->kl", W, PS, GPH)
                D[d] -= np.einsum("mt,mtk,mtl->kl", W, GPH, PS)
            FPH = st_outer(self.phi.eval(fxi[s]), tv)
            out[("Qvol", s)] = Q.copy()
            for d in range(3):
                face_d = np.einsum("mt,mtk,mtl->kl", FWt * area[:, d:d + 1], FPS, FPH)
                Q[d] -= face_d * sigma
                D[d] += face_d.T * sigma
            out[("Q", s)] = Q
            out[("D", s)] = D
            out[("elem", s)] = i
        out["Mplus"] = Mplus
        out["Mcirc"] = Mcirc
        out["M"] = Mplus - Mcirc
        out["Mbar"] = Mbar
        self._face_cache[j] = out
        return out

    def tet(self, i):
        raise NotImplementedError("curved elements: only the pressure system is provided")
