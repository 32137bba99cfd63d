"""Curved (isoparametric) meshes: a smooth deformation of a straight mesh.

A curved element is given by the physical positions of its N spatial nodes
(the equispaced reference points (j1, j2, j3)/p in the layout order of
``node_coordinates``).  These helpers deform a straight Kuhn mesh by a map F,
returning the deformed vertices F(X) and the deformed nodes F(x_k) of every
element; neighbouring elements share the images of their shared face nodes,
so the curved faces match from both sides.

Maps (eps = amplitude, all smooth and invertible for |eps| < 0.1):

* ``"periodic"``: F_d(x) = x_d + eps sin(2 pi x_d) cos(2 pi x_{d+1}) on the
  unit cube; it keeps every boundary plane in place and commutes with the
  unit translations, so periodic pairing still holds.
* ``"bulge"``: F(x) = x + eps sin(pi y) sin(pi z) (x, 0, 0): the face x = 1
  of the unit cube bulges out, every other face stays flat.
* ``"quadratic"``: F(x) = (x + a x^2, y + b y z, z + c x y) with
  (a, b, c) = eps * (1, 0.5, -0.7); a polynomial of degree 2, which degree
  p >= 2 isoparametric elements reproduce exactly.
"""

import numpy as np

from .nodes import node_coordinates


def deform(x, kind, eps):
    """F(x) for points x (..., 3)."""
    x = np.asarray(x, dtype=np.float64)
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    if kind == "periodic":
        tp = 2.0 * np.pi
        return np.stack([X + eps * np.sin(tp * X) * np.cos(tp * Y),
                         Y + eps * np.sin(tp * Y) * np.cos(tp * Z),
                         Z + eps * np.sin(tp * Z) * np.cos(tp * X)], axis=-1)
    if kind == "bulge":
        b = eps * np.sin(np.pi * Y) * np.sin(np.pi * Z)
        return np.stack([X + b * X, Y, Z], axis=-1)
    if kind == "quadratic":
        a, b, c = eps * 1.0, eps * 0.5, eps * -0.7
        return np.stack([X + a * X * X, Y + b * Y * Z, Z + c * X * Y], axis=-1)
    raise ValueError(kind)


def curved_mesh(X, tets, p, kind="periodic", eps=0.04):
    """(F(X), nodes (E, N, 3)) of the deformed mesh with degree-p elements."""
    return deform(X, kind, eps), deform(node_coordinates(X, tets, p), kind, eps)
