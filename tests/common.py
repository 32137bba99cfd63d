"""Shared test helpers: build matching oracle and library meshes for a case."""

import numpy as np

from stdg_inputs import kuhn_mesh


def case_mesh(n, jitter=0.0, seed=3):
    return kuhn_mesh(n, jitter=jitter, seed=seed)


def to_internal(v_input, perm):
    """Input-order rows -> internal-order rows."""
    return np.asarray(v_input)[perm]


def to_input(v_internal, perm):
    out = np.empty_like(v_internal)
    out[perm] = v_internal
    return out


def blocks_apply(mesh, x_int):
    """Apply the library's exported host tables in numpy (test of the tables)."""
    B, cls, nbr, C = mesh.blocks()
    E, G, N = mesh.E, mesh.G, mesh.N
    X = np.asarray(x_int).reshape(E, G, N)
    Y = np.zeros_like(X)
    for i in range(E):
        acc = np.zeros((N, G))
        for k in range(5):
            t = i if k == 0 else nbr[i, k - 1]
            if t < 0:
                continue
            acc += B[cls[i], k] @ X[t].T
        Y[i] = (acc @ C.T).T
    return Y.reshape(E, -1)
