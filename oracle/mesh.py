"""Oracle primary mesh and face-based dual mesh (Sec. 2.2.1; test infrastructure only).

For every face Gamma_j the oracle records its left and right elements
l(j) < r(j) (the paper lets the assignment be arbitrary), the local face index
in each (local face f is the face opposite local vertex f), the unit normal
n_j from left to right, and for periodic pairs the translation that brings the
right element next to the left one.  Boundary faces have r(j) = -1.  The dual
element H_j of an interior face is the union of the sub-tetrahedra
T_{l(j),j} and T_{r(j),j}, each spanned by the face and the barycentre of its
element; a boundary face's dual element is the single sub-tetrahedron.
"""

import numpy as np

from .linalg import asreal, cross, norm


class Mesh:
    def __init__(self, X, tets, periodic=False, box_lo=(0, 0, 0), box_hi=(1, 1, 1)):
        self.X = np.asarray(X, dtype=np.float64)
        self.tets = np.asarray(tets, dtype=np.int64)
        self.E = self.tets.shape[0]
        self.periodic = periodic
        self.box_lo = np.asarray(box_lo, dtype=np.float64)
        self.box_hi = np.asarray(box_hi, dtype=np.float64)
        self._build_faces()

    def _canonical_vertex(self):
        """Map each vertex to a representative of its periodic image class."""
        if not self.periodic:
            return np.arange(self.X.shape[0])
        L = self.box_hi - self.box_lo
        tol = 1e-9 * L.max()
        y = np.mod(self.X - self.box_lo, L)
        y[np.abs(y - L) < tol] = 0.0
        key = np.round(y / tol).astype(np.int64)
        _, inv = np.unique(key, axis=0, return_inverse=True)
        return inv.ravel()

    def _build_faces(self):
        E = self.E
        canon = self._canonical_vertex()
        table = {}
        for t in range(E):
            for f in range(4):
                vs = [self.tets[t, k] for k in range(4) if k != f]
                key = tuple(sorted(canon[v] for v in vs))
                table.setdefault(key, []).append((t, f))
        left, right, lf, rf = [], [], [], []
        for key, lst in table.items():
            if len(lst) == 1:
                (t, f), = lst
                left.append(t); lf.append(f); right.append(-1); rf.append(-1)
            elif len(lst) == 2:
                (a, fa), (b, fb) = sorted(lst)
                left.append(a); lf.append(fa); right.append(b); rf.append(fb)
            else:
                raise ValueError("non-manifold face")
        order = np.lexsort((np.asarray(lf), np.asarray(left)))
        self.left = np.asarray(left)[order]
        self.right = np.asarray(right)[order]
        self.left_face = np.asarray(lf)[order]
        self.right_face = np.asarray(rf)[order]
        self.F = self.left.size
        self.tet_faces = -np.ones((E, 4), dtype=np.int64)
        for j in range(self.F):
            self.tet_faces[self.left[j], self.left_face[j]] = j
            if self.right[j] >= 0:
                self.tet_faces[self.right[j], self.right_face[j]] = j
        self.offset = np.zeros((self.F, 3))
        for j in range(self.F):
            r = self.right[j]
            if r < 0 or not self.periodic:
                continue
            # the right element's copy of a face vertex, moved onto the left's
            lv = [self.tets[self.left[j], k] for k in range(4) if k != self.left_face[j]]
            rv = [self.tets[r, k] for k in range(4) if k != self.right_face[j]]
            a = lv[0]
            b = [v for v in rv if canon[v] == canon[a]][0]
            self.offset[j] = self.X[a] - self.X[b]
        if self.periodic and np.any(self.right < 0):
            raise ValueError("unmatched periodic face")

    # ----- geometry -------------------------------------------------------
    def tet_vertices(self, t, shift=None):
        v = self.X[self.tets[t]].copy()
        if shift is not None:
            v += shift
        return v

    def face_vertices(self, j):
        """Face vertices (3, 3) in the left element's frame."""
        t, f = self.left[j], self.left_face[j]
        return self.X[[self.tets[t, k] for k in range(4) if k != f]]

    def side_vertices(self, j, side):
        """Vertices (4, 3) of the left (side 0) or right (side 1) element,
        the right one translated into the left one's frame."""
        if side == 0:
            return self.tet_vertices(self.left[j])
        return self.tet_vertices(self.right[j], self.offset[j])

    def normal(self, j):
        """Unit normal of face j pointing out of the left element."""
        P = asreal(self.face_vertices(j))
        n = cross(P[1] - P[0], P[2] - P[0])
        n /= norm(n)
        c = asreal(self.tet_vertices(self.left[j])).mean(axis=0)
        if n @ (P[0] - c) < 0:
            n = -n
        return n

    def subtet(self, j, side):
        """Sub-tetrahedron T_{i,j} (4, 3): the face and the element's barycentre."""
        P = asreal(self.face_vertices(j))
        bary = asreal(self.side_vertices(j, side)).mean(axis=0)
        return np.vstack([P, bary[None, :]])

    def neighbour(self, t, f):
        """(neighbour element, face id) across local face f of t (-1 if boundary)."""
        j = self.tet_faces[t, f]
        if self.left[j] == t and self.left_face[j] == f:
            return self.right[j], j
        return self.left[j], j
