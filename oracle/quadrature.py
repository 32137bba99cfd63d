"""Oracle quadrature rules (test infrastructure only).

* ``grundmann_moeller(n, s)``: the Grundmann-Moeller rule on the unit
  n-simplex, exact for polynomials of degree 2s+1 (A. Grundmann and
  H. M. Moeller, SIAM J. Numer. Anal. 15 (1978) 282-290).  All polynomial
  integrals of the scheme (mass, gradient and face matrices of Sec. 2.4-2.5)
  are integrated exactly with it.
* ``gauss_legendre_01(m)``: Gauss-Legendre on [0, 1] (time integrals; the time
  basis of Sec. 2.3 interpolates at these points).
* ``collapsed_triangle_rule(q)``: the face rule fixed for the non-polynomial
  Rusanov term of eq. convdg (the paper does not say which rule it uses):
  q Gauss-Jacobi(1,0) points in the collapsed direction times q Gauss-Legendre
  points, on the reference triangle {a, b >= 0, a + b <= 1}.
"""

import itertools
import math

import numpy as np
from scipy.special import roots_jacobi

from .linalg import REAL, asreal, cross, det3, norm


def _compositions(total, parts):
    """All tuples of `parts` non-negative integers summing to `total`."""
    for cut in itertools.combinations(range(total + parts - 1), parts - 1):
        prev = -1
        out = []
        for c in cut:
            out.append(c - prev - 1)
            prev = c
        out.append(total + parts - 1 - prev - 1)
        yield tuple(out)


def grundmann_moeller(n, s):
    """Points (m, n) and weights (m,) on {x >= 0, sum x <= 1} in R^n.

    Degree of exactness 2s+1; weights sum to the simplex volume 1/n!.
    Computed in numpy.longdouble (weights from exact integer ratios).
    """
    d = 2 * s + 1
    pts, wts = [], []
    for i in range(s + 1):
        num = ((-1) ** i) * (d + n - 2 * i) ** d
        den = 4 ** s * math.factorial(i) * math.factorial(d + n - i)
        w = REAL(num) / REAL(den)
        for beta in _compositions(s - i, n + 1):
            bary = [REAL(2 * b + 1) / REAL(d + n - 2 * i) for b in beta]
            pts.append(bary[1:])
            wts.append(w)
    return np.asarray(pts, dtype=REAL), np.asarray(wts, dtype=REAL)


def simplex_rule(vertices, s):
    """Grundmann-Moeller rule mapped onto the simplex with the given vertices.

    vertices: (n+1, n) array.  Returns physical points (m, n) and weights (m,)
    that already include the volume factor |det J|.
    """
    vertices = asreal(vertices)
    n = vertices.shape[1]
    ref, w = grundmann_moeller(n, s)
    J = (vertices[1:] - vertices[0]).T           # columns: edges from vertex 0
    pts = vertices[0] + ref @ J.T
    dj = det3(J) if n == 3 else J[0, 0] * J[1, 1] - J[0, 1] * J[1, 0]
    return pts, w * abs(dj)


def triangle_rule_3d(P, s):
    """Grundmann-Moeller rule on a triangle P (3, 3) embedded in R^3."""
    P = asreal(P)
    ref, w = grundmann_moeller(2, s)
    e1, e2 = P[1] - P[0], P[2] - P[0]
    pts = P[0] + np.outer(ref[:, 0], e1) + np.outer(ref[:, 1], e2)
    return pts, w * norm(cross(e1, e2))


def _legendre(n, x):
    """P_n(x) and P_n'(x) by the three-term recurrence."""
    p0, p1 = np.ones_like(x), x
    if n == 0:
        return p0, np.zeros_like(x)
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    dp = n * (x * p1 - p0) / (x * x - 1)
    return p1, dp


def gauss_legendre_01(m):
    """Gauss-Legendre nodes and weights on [0, 1] (longdouble: the float64
    nodes are refined by Newton steps on P_m)."""
    x0, _ = np.polynomial.legendre.leggauss(m)
    x = asreal(x0)
    for _ in range(4):
        p, dp = _legendre(m, x)
        x = x - p / dp
    _, dp = _legendre(m, x)
    w = REAL(2) / ((1 - x * x) * dp * dp)
    return REAL(0.5) * (x + 1), REAL(0.5) * w


def collapsed_triangle_rule(q):
    """Reference-triangle rule (q*q points (a, b), weights summing to 1/2).

    a runs over the Gauss-Jacobi points for the weight (1-a) on [0, 1], b =
    v (1 - a) with v the Gauss-Legendre points of [0, 1]; point (i, j) has
    index i*q + j.
    """
    xa, wa = roots_jacobi(q, 1.0, 0.0)          # weight (1-x) on [-1, 1]
    a = 0.5 * (xa + 1.0)
    wa = wa / 4.0                               # (1-x) dx = 4 (1-a) da
    v, wv = gauss_legendre_01(q)
    pts = np.array([(a[i], v[j] * (1.0 - a[i])) for i in range(q) for j in range(q)])
    wts = np.array([wa[i] * wv[j] for i in range(q) for j in range(q)])
    return pts, wts


def face_rule_points(P, q):
    """The Rusanov face rule on the physical triangle P (3, 3).

    The three vertices are first sorted lexicographically by (x, y, z) so the
    point set does not depend on which element looks at the face (and is the
    same, up to the translation, on both sides of a periodic face).  Returns
    points (q*q, 3) and weights including the area factor.
    """
    P = np.asarray(P, dtype=np.float64)
    order = sorted(range(3), key=lambda k: tuple(P[k]))
    P = P[order]
    ref, w = collapsed_triangle_rule(q)
    e1, e2 = P[1] - P[0], P[2] - P[0]
    pts = P[0] + np.outer(ref[:, 0], e1) + np.outer(ref[:, 1], e2)
    return pts, w * np.linalg.norm(np.cross(e1, e2))


def convection_orders(p, p_gamma):
    """Points per direction (space, time) of the Rusanov-term rules.

    Space: ceil((3p+2)/2) so the polynomial part (degree 3p) is exact;
    time: ceil((3 p_gamma + 2)/2) Gauss-Legendre points.
    """
    return (3 * p + 3) // 2, (3 * p_gamma + 3) // 2
