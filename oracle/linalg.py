"""Extended-precision helpers of the oracle (test infrastructure only).

The oracle evaluates every matrix of the scheme in numpy.longdouble (x87
80-bit, 64-bit mantissa): at p = 4 the dual mass matrices of the Taylor basis
of eq. bf_2 have condition numbers near 1e10, which costs FP64 evaluations
about ten digits.  numpy.linalg has no longdouble routines, so the few dense
operations needed are written out here.
"""

import numpy as np

REAL = np.longdouble


def asreal(a):
    return np.asarray(a, dtype=REAL)


def solve(A, B):
    """Solve A X = B by Gauss-Jordan elimination with partial pivoting."""
    A = asreal(A).copy()
    B = asreal(B).copy()
    vec = B.ndim == 1
    if vec:
        B = B[:, None]
    n = A.shape[0]
    for c in range(n):
        piv = c + int(np.argmax(np.abs(A[c:, c])))
        if A[piv, c] == 0:
            raise np.linalg.LinAlgError("singular matrix")
        if piv != c:
            A[[c, piv]] = A[[piv, c]]
            B[[c, piv]] = B[[piv, c]]
        inv = REAL(1) / A[c, c]
        A[c] *= inv
        B[c] *= inv
        f = A[:, c].copy()
        f[c] = 0
        A -= np.outer(f, A[c])
        B -= np.outer(f, B[c])
    return B[:, 0] if vec else B


def inv(A):
    A = asreal(A)
    return solve(A, np.eye(A.shape[0], dtype=REAL))


def det3(J):
    """Determinant of a 3 x 3 matrix."""
    J = asreal(J)
    return (J[0, 0] * (J[1, 1] * J[2, 2] - J[1, 2] * J[2, 1])
            - J[0, 1] * (J[1, 0] * J[2, 2] - J[1, 2] * J[2, 0])
            + J[0, 2] * (J[1, 0] * J[2, 1] - J[1, 1] * J[2, 0]))


def norm(v):
    v = asreal(v)
    return np.sqrt(np.sum(v * v))


def cross(a, b):
    a, b = asreal(a), asreal(b)
    return np.array([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]], dtype=REAL)
