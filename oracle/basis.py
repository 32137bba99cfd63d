"""Oracle basis functions (test infrastructure only).

* Nodal Lagrange basis on the reference tetrahedron (Sec. 2.3, eq. bf_1): the
  coefficients alpha_kr of phi_k = sum_r alpha_kr xi^r solve
  alpha_kr xi_j^r = delta_kj at the equispaced nodes (j1, j2, j3)/p.
* Taylor modal basis on a dual element (eq. bf_2):
  psi_k(x) = prod_d (x_d - x0_d)^{k_d} / h^{|k|}, |k| <= p.
* Time basis: Lagrange polynomials through the Gauss-Legendre points of
  [0, 1] (Sec. 2.3), with their derivatives.

Monomial exponents are enumerated with the first exponent fastest, then the
second, then the third; the same enumeration orders the nodes and the Taylor
functions.
"""

import numpy as np

from .linalg import REAL, asreal, det3, inv
from .quadrature import gauss_legendre_01


def exponents(p):
    """(N, 3) integer exponents r with |r| <= p, first index fastest."""
    out = []
    for r3 in range(p + 1):
        for r2 in range(p + 1 - r3):
            for r1 in range(p + 1 - r3 - r2):
                out.append((r1, r2, r3))
    return np.asarray(out, dtype=np.int64)


def nodal_points(p):
    """(N, 3) reference nodes (j1, j2, j3)/p."""
    e = exponents(p).astype(REAL)
    return e / REAL(p) if p > 0 else e


def _monomials(pts, ex):
    """(m, N) values of x^r at points (m, 3)."""
    return np.prod(pts[:, None, :] ** ex[None, :, :], axis=2)


def _monomial_grads(pts, ex):
    """(m, N, 3) gradients of x^r."""
    m, N = pts.shape[0], ex.shape[0]
    g = np.zeros((m, N, 3), dtype=pts.dtype)
    for d in range(3):
        ed = ex.copy()
        coef = ed[:, d].astype(np.float64)
        ed[:, d] = np.maximum(ed[:, d] - 1, 0)
        g[:, :, d] = coef[None, :] * _monomials(pts, ed)
    return g


def nodal_coefficients(p):
    """alpha (N, N) with phi_k(xi) = sum_r alpha[k, r] xi^r."""
    ex = exponents(p)
    V = _monomials(nodal_points(p), ex)          # V[j, r] = xi_j^r
    # alpha V^T = I
    return inv(V.T)


class NodalBasis:
    """Nodal Lagrange basis of degree p on the reference tetrahedron."""

    def __init__(self, p):
        self.p = p
        self.ex = exponents(p)
        self.N = self.ex.shape[0]
        self.alpha = nodal_coefficients(p)

    def eval(self, xi):
        """Values (m, N) at reference points xi (m, 3)."""
        return _monomials(np.atleast_2d(asreal(xi)), self.ex) @ self.alpha.T

    def grad_ref(self, xi):
        """Reference gradients (m, N, 3)."""
        g = _monomial_grads(np.atleast_2d(asreal(xi)), self.ex)   # (m, R, 3)
        return np.einsum("kr,mrd->mkd", self.alpha, g)


class TetMap:
    """Affine map of a tetrahedron with vertices v (4, 3) (Sec. 2.3)."""

    def __init__(self, v):
        self.v = asreal(v)
        self.J = (self.v[1:] - self.v[0]).T          # x = v0 + J xi
        self.Jinv = inv(self.J)
        self.detJ = det3(self.J)

    def to_ref(self, x):
        return (np.atleast_2d(asreal(x)) - self.v[0]) @ self.Jinv.T

    def to_phys(self, xi):
        return self.v[0] + np.atleast_2d(xi) @ self.J.T

    def volume(self):
        return abs(self.detJ) / 6.0


def nodal_phys(basis, tmap, x):
    """Values (m, N) and physical gradients (m, N, 3) of a tet's nodal basis."""
    xi = tmap.to_ref(x)
    val = basis.eval(xi)
    gref = basis.grad_ref(xi)
    # grad_x phi = J^{-T} grad_xi phi
    grad = np.einsum("ed,mkd->mke", tmap.Jinv.T, gref)
    return val, grad


class TaylorBasis:
    """Taylor modal basis psi_k = (x-x0)^k / h^|k| of eq. bf_2."""

    def __init__(self, p, x0, h):
        self.p = p
        self.ex = exponents(p)
        self.N = self.ex.shape[0]
        self.x0 = asreal(x0)
        self.h = REAL(h)

    def eval(self, x):
        y = (np.atleast_2d(asreal(x)) - self.x0) / self.h
        return _monomials(y, self.ex)


class TimeBasis:
    """Lagrange basis through the G Gauss-Legendre points of [0, 1]."""

    def __init__(self, G):
        self.G = G
        self.nodes, self.weights = gauss_legendre_01(G)
        V = np.vander(self.nodes, G, increasing=True)   # V[a, r] = tau_a^r
        self.coef = inv(V).T                             # gamma_a = sum_r coef[a, r] tau^r

    def eval(self, tau):
        tau = np.atleast_1d(asreal(tau))
        P = np.vander(tau, self.G, increasing=True)
        return P @ self.coef.T                           # (m, G)

    def deriv(self, tau):
        tau = np.atleast_1d(asreal(tau))
        G = self.G
        D = np.zeros((tau.size, G), dtype=REAL)
        for r in range(1, G):
            D[:, r] = r * tau ** (r - 1)
        return D @ self.coef.T
