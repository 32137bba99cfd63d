"""Structured tetrahedral meshes: n^3 hexahedra, each split into 6 tetrahedra.

The split is the Kuhn (Freudenthal) one: for every permutation s of the three
axes, the tetrahedron {v0, v0+h e_s0, v0+h(e_s0+e_s1), v0+h(1,1,1)}.  The
paper's own regular meshes have 6 n^3 elements (Tables 1 and 2 of Sec. 3.2).
"""

import numpy as np

# Axis permutations in a fixed order; the tetrahedron type of a tet is its
# position in this list.
KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def hex_count_for(n_tets):
    """Return n such that 6 n^3 == n_tets (raises if there is none)."""
    n = int(round((n_tets / 6) ** (1.0 / 3.0)))
    if 6 * n ** 3 != n_tets:
        raise ValueError(f"{n_tets} is not 6 n^3")
    return n


def kuhn_mesh(n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), jitter=0.0, seed=0):
    """Return (X, tets) for the box [lo, hi] cut into n^3 hexahedra x 6 tets.

    X    : (V, 3) float64, V = (n+1)^3, vertex (i, j, k) has index
           i + (n+1) (j + (n+1) k).
    tets : (6 n^3, 4) int64; hexahedra in lexicographic (k, j, i) order, the
           6 tets of a hexahedron in ``KUHN_PERMS`` order.
    jitter moves every interior vertex by a seeded uniform offset in
    [-jitter h, jitter h]^3 (boundary vertices stay put so the box and any
    periodic pairing are unchanged).
    """
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    m = n + 1
    g = [np.linspace(lo[d], hi[d], m) for d in range(3)]
    kk, jj, ii = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    X = np.stack([g[0][ii.ravel()], g[1][jj.ravel()], g[2][kk.ravel()]], axis=1)
    if jitter:
        h = (hi - lo) / n
        rng = np.random.default_rng(seed)
        off = rng.uniform(-jitter, jitter, size=X.shape) * h
        interior = ((ii > 0) & (ii < n) & (jj > 0) & (jj < n) & (kk > 0) & (kk < n)).ravel()
        X[interior] += off[interior]

    def vid(i, j, k):
        return i + m * (j + m * k)

    tets = np.empty((6 * n ** 3, 4), dtype=np.int64)
    t = 0
    for k in range(n):
        for j in range(n):
            for i in range(n):
                base = np.array([i, j, k])
                for s in KUHN_PERMS:
                    c = base.copy()
                    verts = [vid(*c)]
                    for d in range(3):
                        c[s[d]] += 1
                        verts.append(vid(*c))
                    tets[t] = verts
                    t += 1
    return X, tets
