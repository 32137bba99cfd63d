"""Oracle Picard pressure-correction time step (Sec. 2.6; test infrastructure only).

One time step of the staggered space-time DG scheme, steps 0-6 of Sec. 2.6,
with the literal space-time matrices of ``spacetime.py``:

 0. guess: dual velocity = previous slab's value at its end (tau = 1) at every
    time node; pressure p^{n+1,0} = 0.
 1. average the dual velocity to the main grid (eq. average) and form the
    previous-iteration pressure contribution Lambda (eq. prevpress).
 2. convective terms on the main grid, space-time DG with the Rusanov flux
    (eq. convdg).
 3. viscous system on the main grid (eq. A1_mod), one solve per component.
 4. project back to the dual grid (eq. goback).
 5. pressure-correction system (eq. A2_mod), anchored.
 6. velocity update (eq. A3_mod).
Steps 1-6 run n_pic times (the paper uses p_gamma + 1).

Readings where the final text is silent (the boundary terms appear only in
commented-out text):
 * Dirichlet faces: the boundary dual element is the single sub-tetrahedron;
   its velocity is prescribed as the projection (goback map with one side) of
   the nodal Dirichlet data g of its element, it has no momentum equation and
   no pressure coupling, its D_ij term enters the pressure right-hand side.
 * In the viscous stress the boundary jump uses g: the boundary face adds
   Q_ij^T Mbar_j^-1 Q_ij to the viscous diagonal and nu D_ij Mbar_j^-1 Ghat_j,
   Ghat_j = int psi~ g n_ij, to the right-hand side, g = the boundary dual
   velocity on the face.
 * Lambda on a Dirichlet face uses the element's own pressure gradient on the
   boundary sub-tetrahedron, M_j^-1 int_{T_ij} psi~ grad p_i (no jump
   against the wall), so Lambda approximates grad p up to the boundary.
 * Lambda is formed from the current Picard pressure p^{n+1,k} at every
   iteration (zero when the guess p^{n+1,0} is zero).
 * Rusanov ghost state on a Dirichlet face: the boundary dual velocity.
 * Mbar_i^- acts on the previous slab's averaged velocity (test at t^n of the
   new slab, trial at the end of the previous slab).
Vectors: dual velocity (F, 3, Nst), main velocity (E, 3, Nst), pressure
(E, Nst); faces and elements in the oracle mesh's numbering.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import linalg
from .basis import TetMap, nodal_phys
from .pressure import assemble_S, solve_anchored
from .quadrature import (convection_orders, face_rule_points, gauss_legendre_01,
                         simplex_rule)
from .spacetime import st_outer

R = linalg.REAL


def _elem_faces(mesh, i):
    return [int(mesh.tet_faces[i, f]) for f in range(4)]


def _side(F, i):
    return 0 if F[("elem", 0)] == i else 1


def time_end_value(ops, v):
    """Value at tau = 1 of a slab (..., Nst) broadcast to all time nodes."""
    G, N = ops.G, ops.N
    g1 = ops.tb.eval(1.0)[0]
    v = linalg.asreal(v).reshape(v.shape[:-1] + (G, N))
    end = np.einsum("a,...an->...n", g1, v)
    return np.repeat(end[..., None, :], G, axis=-2).reshape(v.shape[:-2] + (G * N,))


def goback(ops, vbar, j):
    """Eq. goback for face j: Mbar_j^-1 sum_sides M_ij^T vbar_i  (3, Nst)."""
    F = ops.face(j)
    rhs = sum(F[("Mij", s)].T @ linalg.asreal(vbar[F[("elem", s)]]).T for s in F["sides"])
    return linalg.solve(F["Mbar"], rhs).T


def average(ops, vhat):
    """Eq. average: vbar_i = M_i^-1 sum_{j in S_i} M_ij vhat_j  (E, 3, Nst)."""
    mesh = ops.mesh
    out = np.zeros((mesh.E, 3, ops.Nst), dtype=R)
    for i in range(mesh.E):
        acc = np.zeros((ops.Nst, 3), dtype=R)
        for j in _elem_faces(mesh, i):
            F = ops.face(j)
            acc += F[("Mij", _side(F, i))] @ linalg.asreal(vhat[j]).T
        out[i] = linalg.solve(ops.tet(i)["M"], acc).T
    return out


def prev_pressure(ops, p):
    """Eq. prevpress: Lambda_i = M_i^-1 sum_j M_ij M_j^-1 (Q_rj p_r + Q_lj p_l)."""
    mesh = ops.mesh
    out = np.zeros((mesh.E, 3, ops.Nst), dtype=R)
    for i in range(mesh.E):
        acc = np.zeros((ops.Nst, 3), dtype=R)
        for j in _elem_faces(mesh, i):
            F = ops.face(j)
            if mesh.right[j] < 0:
                g = np.einsum("dkl,l->dk", F[("Qvol", 0)], linalg.asreal(p[i]))
            else:
                g = sum(np.einsum("dkl,l->dk", F[("Q", s)], linalg.asreal(p[F[("elem", s)]]))
                        for s in (0, 1))
            w = linalg.solve(F["M"], g.T)                  # (Nst, 3)
            acc += F[("Mij", _side(F, i))] @ w
        out[i] = linalg.solve(ops.tet(i)["M"], acc).T
    return out


def neighbour_vertices(mesh, i, f):
    """Vertices of the element across local face f of i, translated next to i."""
    k, j = mesh.neighbour(i, f)
    if k < 0:
        return None
    if mesh.left[j] == i:
        return mesh.tet_vertices(k, mesh.offset[j])
    return mesh.tet_vertices(k, -mesh.offset[j])


def convection(ops, vbar, vhat_bc):
    """Eq. convdg: Upsilon_i = oint phi~ F^RS . n - int grad phi~ : (v (x) v).

    vbar: (E, 3, Nst) main velocity; vhat_bc: dict face -> (3, Nst) boundary
    dual velocity (Rusanov ghost state on Dirichlet faces).  Returns (E, 3, Nst).
    """
    mesh = ops.mesh
    p, G, N = ops.p, ops.G, ops.N
    qs, qt = convection_orders(p, G - 1)
    tau, wtau = gauss_legendre_01(qt)
    tv = ops.tb.eval(tau)                                   # (t, G)
    dt = ops.dt
    out = np.zeros((mesh.E, 3, ops.Nst), dtype=R)
    s_vol = max(0, (3 * p - 1) // 2)                        # exact for degree 3p - 1
    for i in range(mesh.E):
        v = mesh.tet_vertices(i)
        tm = TetMap(v)
        V = linalg.asreal(vbar[i]).reshape(3, G, N)
        # volume term
        xq, wq = simplex_rule(v, s_vol)
        ph, gph = nodal_phys(ops.phi, tm, xq)               # (m, N), (m, N, 3)
        vel = np.einsum("mn,cgn,tg->mtc", ph, V, tv)        # (m, t, 3)
        Fc = vel[..., :, None] * vel[..., None, :]          # (m, t, c, d)
        W = wq[:, None] * wtau[None, :] * dt
        for c in range(3):
            for d in range(3):
                GPH = st_outer(gph[:, :, d], tv)             # (m, t, Nst)
                out[i, c] -= np.einsum("mt,mtk,mt->k", W, GPH, Fc[..., c, d])
        # face terms
        for f in range(4):
            P = v[[k for k in range(4) if k != f]]
            fq, fw = face_rule_points(P, qs)
            fq, fw = linalg.asreal(fq), linalg.asreal(fw)
            n = linalg.cross(linalg.asreal(P[1]) - P[0], linalg.asreal(P[2]) - P[0])
            n /= linalg.norm(n)
            if n @ (linalg.asreal(P[0]) - linalg.asreal(v).mean(axis=0)) < 0:
                n = -n
            fph, _ = nodal_phys(ops.phi, tm, fq)
            vm = np.einsum("mn,cgn,tg->mtc", fph, V, tv)
            k, j = mesh.neighbour(i, f)
            if k >= 0:
                vk = neighbour_vertices(mesh, i, f)
                kph, _ = nodal_phys(ops.phi, TetMap(vk), fq)
                Vk = linalg.asreal(vbar[k]).reshape(3, G, N)
                vp = np.einsum("mn,cgn,tg->mtc", kph, Vk, tv)
            else:
                psi = ops.face(j)["psi"].eval(fq)           # boundary dual basis
                Vb = linalg.asreal(vhat_bc[j]).reshape(3, G, N)
                vp = np.einsum("mn,cgn,tg->mtc", psi, Vb, tv)
            un_m = vm @ n
            un_p = vp @ n
            smax = 2 * np.maximum(np.sqrt((vm * vm).sum(-1)), np.sqrt((vp * vp).sum(-1)))
            flux = 0.5 * (vp * un_p[..., None] + vm * un_m[..., None]) \
                - 0.5 * smax[..., None] * (vp - vm)         # (m, t, 3)
            FPH = st_outer(fph, tv)
            FW = fw[:, None] * wtau[None, :] * dt
            out[i] += np.einsum("mt,mtk,mtc->ck", FW, FPH, flux)
    return out


def viscous_matrix(ops, nu):
    """Matrix of eq. A1_mod: Mbar_i - nu sum_j D_ij Mbar_j^-1 Q_{.,j}, all faces."""
    mesh = ops.mesh
    Nst = ops.Nst
    rows, cols, vals = [], [], []

    def put(i, k, blk):
        r, c = np.meshgrid(np.arange(Nst) + i * Nst, np.arange(Nst) + k * Nst, indexing="ij")
        rows.append(r.ravel()); cols.append(c.ravel()); vals.append(blk.ravel().astype(np.float64))
    for i in range(mesh.E):
        put(i, i, ops.tet(i)["Mbar"])
    for j in range(mesh.F):
        F = ops.face(j)
        Minv = linalg.inv(F["Mbar"])
        for s in F["sides"]:
            for t in F["sides"]:
                blk = -nu * np.einsum("dkm,dmn->kn", np.einsum("dkl,lm->dkm", F[("D", s)], Minv), F[("Q", t)])
                put(F[("elem", s)], F[("elem", t)], blk)
    n = mesh.E * Nst
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def _face_psi_mass(ops, j):
    """int over Gamma_j^st of psi~ psi~ times the outward normal of its element."""
    mesh = ops.mesh
    F = ops.face(j)
    from .quadrature import triangle_rule_3d
    P = mesh.face_vertices(j)
    fq, fw = triangle_rule_3d(P, ops.s_space)
    tv = ops.tb.eval(ops.tau)
    PS = st_outer(F["psi"].eval(fq), tv)
    FW = fw[:, None] * ops.wtau[None, :] * ops.dt
    return np.einsum("mt,mtk,mtl->kl", FW, PS, PS), F["normal"]


def picard_step(ops, vhat_prev, vbar_prev, g_nodal, nu, n_pic, anchor_elem=0, anchor_node=0,
                p_init=None, theta=1.0, p_prev=None):
    """One time step.  Returns (vhat, vbar_new, p, diagnostics).

    p_init: pressure guess p^{n+1,0} (E, Nst); zero (the paper's choice) when
    None, or e.g. the previous slab's pressure (the paper's alternative).

    theta: implicitness of the pressure for p_gamma = 0 (Sec. 2.7, eqs.
    CS_15_theta and CS_16_theta): the momentum equation carries
    theta p^{n+1} + (1 - theta) p^n, p^n = p_prev.  In this pressure-correction
    form that pressure enters Lambda, the correction system becomes
    theta S dp = b, and the dual velocity is corrected by theta M^-1 Q dp.
    theta = 1 is the scheme of Sec. 2.6."""
    if theta != 1.0:
        if ops.G != 1:
            raise ValueError("the theta-method is defined for p_gamma = 0")
        if p_prev is None:
            raise ValueError("theta < 1 needs the previous pressure p_prev")
    mesh = ops.mesh
    E, Fn, Nst = mesh.E, mesh.F, ops.Nst
    bfaces = [j for j in range(Fn) if mesh.right[j] < 0]
    ifaces = [j for j in range(Fn) if mesh.right[j] >= 0]
    # step 0
    vhat = time_end_value(ops, linalg.asreal(vhat_prev))
    vhat_bc = {j: goback(ops, g_nodal, j) for j in bfaces}
    for j in bfaces:
        vhat[j] = vhat_bc[j]
    p = np.zeros((E, Nst), dtype=R) if p_init is None else linalg.asreal(p_init).copy()
    S = assemble_S(ops)
    Av = viscous_matrix(ops, nu).tocsc()
    Av_lu = spla.splu(Av)
    bnd_term = np.zeros((E, 3, Nst), dtype=R)
    for j in bfaces:
        F = ops.face(j)
        i = F[("elem", 0)]
        K, n = _face_psi_mass(ops, j)          # n: outward normal of element i
        Minv = linalg.inv(F["Mbar"])
        for c in range(3):
            Ghat = np.stack([K @ vhat_bc[j][c] * n[d] for d in range(3)])     # (3, Nst)
            bnd_term[i, c] += nu * np.einsum("dkl,lm,dm->k", F[("D", 0)], Minv, Ghat)
    Mb_minus = [ops.tet(i)["Mbar_minus"] for i in range(E)]
    Mb = [ops.tet(i)["Mbar"] for i in range(E)]
    vbar_prev = linalg.asreal(vbar_prev)
    diag = {"solves": []}
    for k in range(n_pic):
        # step 1
        vbar_k = average(ops, vhat)
        p_mom = p if theta == 1.0 else theta * p + (1.0 - theta) * linalg.asreal(p_prev)
        lam = prev_pressure(ops, p_mom)
        # step 2
        ups = convection(ops, vbar_k, vhat_bc)
        # step 3
        rhs = np.zeros((E, 3, Nst), dtype=R)
        for i in range(E):
            for c in range(3):
                rhs[i, c] = Mb_minus[i] @ vbar_prev[i, c] - ups[i, c] - Mb[i] @ lam[i, c]
        rhs += bnd_term
        vbar_half = np.zeros((E, 3, Nst), dtype=R)
        for c in range(3):
            vbar_half[:, c] = Av_lu.solve(rhs[:, c].astype(np.float64).ravel()).reshape(E, Nst)
        # step 4
        Fv = np.zeros((Fn, 3, Nst), dtype=R)
        for j in ifaces:
            Fv[j] = goback(ops, vbar_half, j)
        for j in bfaces:
            Fv[j] = vhat_bc[j]
        # step 5: b_i = -sum_{j in S_i} D_ij Fv_j
        b = np.zeros((E, Nst), dtype=R)
        for j in range(Fn):
            F = ops.face(j)
            for s in F["sides"]:
                b[F[("elem", s)]] -= np.einsum("dkl,dl->k", F[("D", s)], Fv[j])
        dp = solve_anchored(ops, theta * S, b.astype(np.float64).ravel(), anchor_elem, anchor_node)
        dp = linalg.asreal(dp).reshape(E, Nst)
        diag["solves"].append({"b": b.astype(np.float64), "dp": dp.astype(np.float64)})
        # step 6
        for j in ifaces:
            F = ops.face(j)
            g = sum(np.einsum("dkl,l->dk", F[("Q", s)], dp[F[("elem", s)]]) for s in (0, 1))
            vhat[j] = Fv[j] - theta * linalg.solve(F["M"], g.T).T
        for j in bfaces:
            vhat[j] = vhat_bc[j]
        p = p + dp
    vbar_new = average(ops, vhat)
    return (vhat.astype(np.float64), vbar_new.astype(np.float64), p.astype(np.float64), diag)


def initial_state(ops, vbar0):
    """Dual velocity of the initial slab: goback of the nodal initial field
    (one-sided on boundary faces).  Returns (F, 3, Nst)."""
    return np.stack([goback(ops, vbar0, j) for j in range(ops.mesh.F)]).astype(np.float64)


def divergence(ops, vhat):
    """sum_{j in S_i} D_ij vhat_j per element (eq. CS_15)  (E, Nst)."""
    mesh = ops.mesh
    out = np.zeros((mesh.E, ops.Nst), dtype=R)
    for j in range(mesh.F):
        F = ops.face(j)
        for s in F["sides"]:
            out[F[("elem", s)]] += np.einsum("dkl,dl->k", F[("D", s)], linalg.asreal(vhat[j]))
    return out.astype(np.float64)
