"""Precision pin of the FP64 oracle at p = 4 (the degree of the 175-DoF case).

One interior dual element of a Kuhn mesh is evaluated in 40-digit arithmetic
(mpmath) by an independent route: the Lagrange basis in Silvester's product
form on barycentric coordinates (the closed-form solution of the interpolation
conditions of eq. bf_1), a Grundmann-Moeller rule built in mpmath, a Taylor
dual basis centred at a face vertex with unit scale (any P_p basis gives the
same operator), and exact vertex coordinates.  The oracle's FP64 blocks
-D_ij M_j^-1 Q_kj (eq. CS_19) must agree to 3e-13 relative (the FP64 evaluation of the same blocks is off by up to 2e-10 on face 47).
"""

import itertools

import numpy as np
import pytest

from stdg_inputs import kuhn_mesh
from oracle.basis import exponents
from oracle.linalg import inv
from oracle.mesh import Mesh
from oracle.spacetime import SpaceTimeOperators

mp = pytest.importorskip("mpmath")


def _compositions(total, parts):
    for cut in itertools.combinations(range(total + parts - 1), parts - 1):
        prev, out = -1, []
        for c in cut:
            out.append(c - prev - 1)
            prev = c
        out.append(total + parts - 2 - prev)
        yield tuple(out)


def _gm_mp(n, s):
    d = 2 * s + 1
    pts, w = [], []
    for i in range(s + 1):
        wi = mp.mpf(-1) ** i * mp.mpf(2) ** (-2 * s) * mp.mpf(d + n - 2 * i) ** d \
            / (mp.factorial(i) * mp.factorial(d + n - i))
        for beta in _compositions(s - i, n + 1):
            pts.append([mp.mpf(2 * b + 1) / (d + n - 2 * i) for b in beta])
            w.append(wi)
    return pts, w


def _silvester(p, ex, lam):
    """Values and barycentric derivatives of the equispaced Lagrange basis."""
    vals, dls = [], []
    for e in ex:
        idx = [p - sum(e), e[0], e[1], e[2]]
        L, dL = [], []
        for c in range(4):
            v, dv = mp.mpf(1), mp.mpf(0)
            for m in range(idx[c]):
                f = (p * lam[c] - m) / (m + 1)
                dv = dv * f + v * mp.mpf(p) / (m + 1)
                v = v * f
            L.append(v)
            dL.append(dv)
        vals.append(L[0] * L[1] * L[2] * L[3])
        dls.append((L, dL))
    return vals, dls


def _block_mp(mesh, j, p):
    mp.mp.dps = 40
    ex = [tuple(int(c) for c in e) for e in exponents(p)]
    N = len(ex)

    def q(v):  # Kuhn n=2 coordinates are multiples of 1/2: exact
        return [mp.mpf(int(round(c * 2))) / 2 for c in v]
    P = [q(v) for v in mesh.face_vertices(j)]
    V = [[q(v) for v in mesh.side_vertices(j, s)] for s in (0, 1)]
    bary = [[sum(v[k][d] for k in range(4)) / 4 for d in range(3)] for v in V]
    e1 = [P[1][d] - P[0][d] for d in range(3)]
    e2 = [P[2][d] - P[0][d] for d in range(3)]
    cr = [e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]]
    area2 = mp.sqrt(sum(c * c for c in cr))
    nrm = [c / area2 for c in cr]
    if sum(nrm[d] * (P[0][d] - bary[0][d]) for d in range(3)) < 0:
        nrm = [-c for c in nrm]

    def psi(x):
        y = [x[d] - P[0][d] for d in range(3)]
        return [y[0] ** e[0] * y[1] ** e[1] * y[2] ** e[2] for e in ex]

    def phys(v, x):
        J = mp.matrix(3, 3)
        for c in range(3):
            for r in range(3):
                J[r, c] = v[c + 1][r] - v[0][r]
        Ji = J ** -1
        xi = Ji * mp.matrix([x[d] - v[0][d] for d in range(3)])
        lam = [1 - xi[0] - xi[1] - xi[2], xi[0], xi[1], xi[2]]
        vals, dls = _silvester(p, ex, lam)
        grads = []
        for L, dL in dls:
            g = []
            for a in range(3):
                others = mp.mpf(1)
                for k in (1, 2, 3):
                    if k != a + 1:
                        others *= L[k]
                g.append(dL[a + 1] * L[0] * others - dL[0] * L[1] * L[2] * L[3])
            grads.append([sum(Ji[b, c] * g[b] for b in range(3)) for c in range(3)])
        return vals, grads

    p3, w3 = _gm_mp(3, p + 1)
    p2, w2 = _gm_mp(2, p + 1)
    M = mp.matrix(N, N)
    Q = [[mp.matrix(N, N) for _ in range(3)] for _ in range(2)]
    for s in (0, 1):
        sub = [bary[s]] + P
        Js = mp.matrix(3, 3)
        for c in range(3):
            for r in range(3):
                Js[r, c] = sub[c + 1][r] - sub[0][r]
        jac = abs(mp.det(Js))
        for qq, wq in zip(p3, w3):
            x = [sub[0][r] + sum(Js[r, c] * qq[c + 1] for c in range(3)) for r in range(3)]
            ps = psi(x)
            _, grads = phys(V[s], x)
            for a in range(N):
                wa = wq * jac * ps[a]
                for b in range(N):
                    M[a, b] += wa * ps[b]
                    for d in range(3):
                        Q[s][d][a, b] += wa * grads[b][d]
        sg = 1 if s == 0 else -1
        for qq, wq in zip(p2, w2):
            x = [P[0][r] + qq[1] * e1[r] + qq[2] * e2[r] for r in range(3)]
            ps = psi(x)
            vals, _ = phys(V[s], x)
            for a in range(N):
                for b in range(N):
                    c = wq * area2 * ps[a] * vals[b] * sg
                    for d in range(3):
                        Q[s][d][a, b] -= c * nrm[d]
    Mi = M ** -1
    out = []
    for t in (0, 1):
        S = mp.matrix(N, N)
        for d in range(3):
            S += Q[0][d].T * Mi * Q[t][d]
        out.append(np.array(S.tolist(), dtype=float))
    return out


@pytest.mark.slow
@pytest.mark.parametrize("which", ["fourth_interior", "face_47"])
def test_p4_block_matches_40_digit_evaluation(which):
    """Face 47 of the 2^3 x 6 mesh is the worst-conditioned one in FP64."""
    p = 4
    X, T = kuhn_mesh(2)
    mesh = Mesh(X, T)
    j = 47 if which == "face_47" else [k for k in range(mesh.F) if mesh.right[k] >= 0][3]
    assert mesh.right[j] >= 0
    ref00, ref01 = _block_mp(mesh, j, p)
    ops = SpaceTimeOperators(mesh, p, 0, 1.0)
    F = ops.face(j)
    Minv = inv(F["M"])
    s00 = -np.einsum("dkl,lm,dmn->kn", F[("D", 0)], Minv, F[("Q", 0)])
    s01 = -np.einsum("dkl,lm,dmn->kn", F[("D", 0)], Minv, F[("Q", 1)])
    assert np.abs(s00 - ref00).max() <= 3e-13 * np.abs(ref00).max()
    assert np.abs(s01 - ref01).max() <= 3e-13 * np.abs(ref01).max()
