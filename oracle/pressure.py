"""Oracle pressure Schur operator and anchored solve (test infrastructure only).

The paper's pressure system (eq. CS_19) is
    sum_j D_ij M_j^-1 Q_ij p_i + sum_j D_ij M_j^-1 Q_{P(i,j),j} p_{P(i,j)} = rhs_i
over the interior faces j of element i.  Because D_ij = -Q_ij^T, that matrix is
minus a positive semi-definite one when p_gamma = 0, while Corollaries 1-2 call
the system matrix positive semi-definite; the oracle (and the library) work with
    S = -(sum_j D_ij M_j^-1 Q_{.,j}),
so S p = -sum_j D_ij Fv_j has the same solution as the paper's equation.

The pressure is fixed at one point (Sec. 3.3 and the abstract: pressure
specified in at least one point): the anchored system replaces the rows and
columns of the anchor element's node 0, at every time node, by the identity
with zero right-hand side.  Vectors are [element][time node][spatial node]
flattened, in the mesh's input element numbering.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import linalg


def interior_faces(mesh):
    return [j for j in range(mesh.F) if mesh.right[j] >= 0]


def apply_S(ops, x, elements=None):
    """y = S x (eq. CS_19, sign as above).

    x: (E, Nst).  If `elements` is given only those rows are computed (the
    other rows of the result are left at zero).
    """
    mesh = ops.mesh
    x = linalg.asreal(x).reshape(mesh.E, ops.Nst)
    y = np.zeros_like(x)
    if elements is None:
        faces = interior_faces(mesh)
        want = None
    else:
        want = set(int(e) for e in elements)
        faces = sorted({int(mesh.tet_faces[e, f]) for e in want for f in range(4)})
        faces = [j for j in faces if mesh.right[j] >= 0]
    for j in faces:
        F = ops.face(j)
        # momentum-equation velocity response to the pressure on both sides
        g = sum(np.einsum("dkl,l->dk", F[("Q", s)], x[F[("elem", s)]]) for s in (0, 1))
        w = linalg.solve(F["M"], g.T).T             # M_j^-1 per component
        for s in (0, 1):
            i = F[("elem", s)]
            if want is not None and i not in want:
                continue
            y[i] -= np.einsum("dkl,dl->k", F[("D", s)], w)
    return y.astype(np.float64)


def assemble_S(ops):
    """Sparse S (E*Nst square)."""
    mesh = ops.mesh
    Nst = ops.Nst
    rows, cols, vals = [], [], []
    for j in interior_faces(mesh):
        F = ops.face(j)
        Minv = linalg.inv(F["M"])
        for s in (0, 1):
            for t in (0, 1):
                blk = -np.einsum("dkm,dmn->kn", np.einsum("dkl,lm->dkm", F[("D", s)], Minv), F[("Q", t)])
                i, k = F[("elem", s)], F[("elem", t)]
                r, c = np.meshgrid(np.arange(Nst) + i * Nst, np.arange(Nst) + k * Nst,
                                   indexing="ij")
                rows.append(r.ravel()); cols.append(c.ravel())
                vals.append(blk.ravel().astype(np.float64))
    n = mesh.E * Nst
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def anchor_indices(ops, anchor_elem=0, anchor_node=0):
    """Flat indices of the anchored unknowns (one per time node)."""
    return np.array([anchor_elem * ops.Nst + a * ops.N + anchor_node for a in range(ops.G)])


def anchored_system(S, b, idx):
    """Rows and columns idx replaced by the identity, right-hand side zero."""
    S = sp.lil_matrix(S)
    for k in idx:
        S[k, :] = 0.0
        S[:, k] = 0.0
        S[k, k] = 1.0
    b = np.array(b, dtype=np.float64).ravel()
    b[idx] = 0.0
    return S.tocsr(), b


def solve_anchored(ops, S, b, anchor_elem=0, anchor_node=0):
    """The unique solution of the anchored pressure system (sparse direct)."""
    idx = anchor_indices(ops, anchor_elem, anchor_node)
    Sa, ba = anchored_system(S, b, idx)
    return spla.spsolve(Sa.tocsc(), ba)


def anchored_residual(ops, x, b, y_of_x, anchor_elem=0, anchor_node=0):
    """||b_a - S_a x|| / ||b_a|| given y = S x (x with x_anchor = 0)."""
    idx = anchor_indices(ops, anchor_elem, anchor_node)
    r = np.array(b, dtype=np.float64).ravel() - np.asarray(y_of_x).ravel()
    r[idx] = 0.0 - np.asarray(x).ravel()[idx]
    bb = np.array(b, dtype=np.float64).ravel()
    bb[idx] = 0.0
    return np.linalg.norm(r) / np.linalg.norm(bb)
