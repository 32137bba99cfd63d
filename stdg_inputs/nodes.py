"""Where nodal coefficients live: the layout of pressure and main-grid vectors."""

import numpy as np


def n_spatial(p):
    """Number of spatial basis functions of degree p on a tetrahedron."""
    return (p + 1) * (p + 2) * (p + 3) // 6


def node_reference_points(p):
    """(N, 3) reference coordinates (j1, j2, j3)/p, j1 fastest then j2, j3."""
    pts = []
    for j3 in range(p + 1):
        for j2 in range(p + 1 - j3):
            for j1 in range(p + 1 - j3 - j2):
                pts.append((j1, j2, j3))
    pts = np.asarray(pts, dtype=np.float64)
    return pts / p if p > 0 else pts


def node_coordinates(X, tets, p):
    """(E, N, 3) physical coordinates of every tet's spatial nodes."""
    ref = node_reference_points(p)
    v = X[tets]                                # (E, 4, 3)
    J = v[:, 1:, :] - v[:, :1, :]              # rows: v1-v0, v2-v0, v3-v0
    return v[:, None, 0, :] + np.einsum("nk,ekd->end", ref, J)


def time_nodes(G):
    """Gauss-Legendre points of [0, 1] in ascending order (G of them)."""
    x, _ = np.polynomial.legendre.leggauss(G)
    return 0.5 * (x + 1.0)
