"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed-form
integrals, hand-derived matrices, identities that follow from the paper's
definitions (Sec. 2.4, eqs. MD_3, MD_6, SD_1, CS_19), Corollaries 1-2 of
Sec. 2.7, and Green's formula on polynomial pressures.
"""

import itertools
import math

import numpy as np
import pytest

from stdg_inputs import kuhn_mesh, node_coordinates
from oracle.basis import NodalBasis, TimeBasis, exponents, nodal_points
from oracle.mesh import Mesh
from oracle.pressure import (apply_S, assemble_S, anchor_indices, anchored_system,
                             solve_anchored)
from oracle.quadrature import (grundmann_moeller, collapsed_triangle_rule,
                               simplex_rule)
from oracle.spacetime import SpaceTimeOperators

SQ3 = math.sqrt(3.0)


# ---------------------------------------------------------------- quadrature
@pytest.mark.parametrize("n", [2, 3])
@pytest.mark.parametrize("s", [0, 1, 2, 3, 4])
def test_grundmann_moeller_exact_on_monomials(n, s):
    """int over the unit simplex of x^a = a! / (|a| + n)!  (Dirichlet integral)."""
    pts, w = grundmann_moeller(n, s)
    for a in itertools.product(range(2 * s + 2), repeat=n):
        if sum(a) > 2 * s + 1:
            continue
        exact = np.prod([math.factorial(k) for k in a]) / math.factorial(sum(a) + n)
        got = np.sum(w * np.prod(pts ** np.array(a), axis=1))
        assert abs(got - exact) <= 1e-13 * max(1.0, abs(exact)), (a, got, exact)


@pytest.mark.parametrize("q", [1, 2, 4, 6, 7])
def test_collapsed_triangle_rule_exact(q):
    pts, w = collapsed_triangle_rule(q)
    for a in range(2 * q):
        for b in range(2 * q - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b)
            assert abs(got - exact) <= 1e-14, (a, b)


# ---------------------------------------------------------------- bases
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_nodal_basis_is_kronecker_delta(p):
    """phi_k(xi_j) = delta_kj (eq. bf_1) and the basis reproduces P_p."""
    B = NodalBasis(p)
    assert B.N == (p + 1) * (p + 2) * (p + 3) // 6
    V = B.eval(nodal_points(p))
    assert np.allclose(V, np.eye(B.N), atol=1e-11)
    rng = np.random.default_rng(3)
    pts = rng.random((20, 3)) / 3
    for r in exponents(p)[::3]:
        f_nodes = np.prod(nodal_points(p) ** r, axis=1)
        f_pts = np.prod(pts ** r, axis=1)
        assert np.allclose(B.eval(pts) @ f_nodes, f_pts, atol=1e-11)


def test_time_basis_pgamma1_closed_form():
    """For p_gamma = 1 the Gauss-Legendre Lagrange basis gives, by hand,
    gamma(1) = ((1-sqrt3)/2, (1+sqrt3)/2), gamma' = (-sqrt3, sqrt3), and
    T = gamma(1) gamma(1)^T - int gamma' gamma^T = [[1, (sqrt3-1)/2],
    [-(sqrt3+1)/2, 1]] (the time factor of M_j = M_j^+ - M_j^o, Sec. 2.4)."""
    tb = TimeBasis(2)
    g1 = tb.eval(1.0)[0]
    g0 = tb.eval(0.0)[0]
    assert np.allclose(g1, [(1 - SQ3) / 2, (1 + SQ3) / 2], atol=1e-14)
    assert np.allclose(g0, [(1 + SQ3) / 2, (1 - SQ3) / 2], atol=1e-14)
    assert np.allclose(tb.deriv(0.3)[0], [-SQ3, SQ3], atol=1e-13)


# ---------------------------------------------------------------- helpers
def make_ops(n, p, pg, periodic=False, dt=0.1, jitter=0.0):
    X, T = kuhn_mesh(n, jitter=jitter, seed=7)
    return SpaceTimeOperators(Mesh(X, T, periodic=periodic), p, pg, dt)


T_CLOSED = np.array([[1.0, (SQ3 - 1) / 2], [-(SQ3 + 1) / 2, 1.0]])


def test_D_is_minus_Q_transpose():
    """MD_3 and MD_6 with sigma of SD_1 give D_ij = -Q_ij^T exactly."""
    ops = make_ops(2, 2, 1)
    for j in range(0, ops.mesh.F, 17):
        F = ops.face(j)
        for s in F["sides"]:
            Q, D = F[("Q", s)], F[("D", s)]
            assert np.abs(D + Q.transpose(0, 2, 1)).max() <= 1e-14 * np.abs(Q).max()


def test_spacetime_matrices_factor_as_space_times_time():
    """Literal space-time matrices equal spatial ones times the hand-derived
    time matrices: M_j = M^sp (x) T, Q = (x) W, Mbar_j = (x) W, W = I/2."""
    o1 = make_ops(2, 2, 0)
    o2 = make_ops(2, 2, 1)
    W = 0.5 * np.eye(2)
    for j in (0, 5, 40, 77):
        a, b = o1.face(j), o2.face(j)
        assert np.allclose(b["M"], np.kron(T_CLOSED, a["M"]), rtol=0, atol=1e-13 * abs(a["M"]).max())
        assert np.allclose(b["Mbar"], np.kron(W, a["Mbar"]), rtol=0, atol=1e-13 * abs(a["Mbar"]).max())
        for s in a["sides"]:
            for d in range(3):
                assert np.allclose(b[("Q", s)][d], np.kron(W, a[("Q", s)][d]), rtol=0,
                                   atol=1e-13 * abs(a[("Q", s)]).max())


@pytest.mark.parametrize("periodic,n,p", [(False, 2, 1), (False, 2, 2), (True, 3, 1)])
def test_pressure_operator_symmetric_psd_constant_nullspace(periodic, n, p):
    """Corollaries 1-2 (p_gamma = 0): S symmetric positive semi-definite; with
    Dirichlet velocity or periodic faces its null space is the constants."""
    ops = make_ops(n, p, 0, periodic=periodic)
    S = assemble_S(ops).toarray()
    scale = np.abs(S).max()
    assert np.abs(S - S.T).max() <= 1e-13 * scale
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev.min() >= -1e-12 * ev.max()
    assert np.sum(ev < 1e-10 * ev.max()) == 1
    assert np.abs(S @ np.ones(S.shape[0])).max() <= 1e-13 * scale


def _poly(coef, ex, x):
    return np.sum(coef * np.prod(x[..., None, :] ** ex, axis=-1), axis=-1)


def _laplacian_poly(coef, ex, x):
    out = np.zeros(x.shape[:-1])
    for c, e in zip(coef, ex):
        for d in range(3):
            if e[d] >= 2:
                e2 = e.copy(); e2[d] -= 2
                out += c * e[d] * (e[d] - 1) * np.prod(x ** e2, axis=-1)
    return out


@pytest.mark.parametrize("p,pg", [(2, 0), (3, 0), (2, 1), (1, 0)])
def test_closed_form_on_polynomial_pressure(p, pg):
    """For a global polynomial q in P_p and an element whose four faces are
    interior: the velocity response M_j^-1 (Q_l q + Q_r q) reproduces grad q
    exactly, and summing D_ij over the faces is Green's formula, so
    (S q)_(i,a,k) = -dt^2 c_a int_Ti phi_k Lap(q), with c = 1 for p_gamma = 0
    and c = W T^-1 W 1 = ((3-sqrt3)/12, (3+sqrt3)/12) for p_gamma = 1."""
    dt = 0.1
    ops = make_ops(3, p, pg, dt=dt)
    mesh = ops.mesh
    rng = np.random.default_rng(11)
    ex = exponents(p)
    coef = rng.standard_normal(ex.shape[0])
    xn = node_coordinates(mesh.X, mesh.tets, p)           # (E, N, 3)
    qn = _poly(coef, ex, xn)                               # (E, N)
    x = np.tile(qn, (1, ops.G))
    inner = [e for e in range(mesh.E) if all(mesh.neighbour(e, f)[0] >= 0 for f in range(4))]
    assert len(inner) > 10
    sample = inner[::7]
    y = apply_S(ops, x, elements=sample)
    c = np.array([1.0]) if pg == 0 else np.array([(3 - SQ3) / 12, (3 + SQ3) / 12])
    from oracle.basis import TetMap, nodal_phys
    for e in sample:
        v = mesh.tet_vertices(e)
        xq, wq = simplex_rule(v, p + 1)
        ph, _ = nodal_phys(ops.phi, TetMap(v), xq)
        rhs = -dt * dt * (wq[:, None] * ph * _laplacian_poly(coef, ex, xq)[:, None]).sum(0)
        expect = np.concatenate([ca * rhs for ca in c])
        # natural size of one row: dt^2 |q| h  (int phi Lap q ~ h^3 |q| / h^2)
        scale = max(np.abs(expect).max(), dt * dt * np.abs(qn).max() / 3.0)
        assert np.abs(y[e] - expect).max() <= 1e-9 * scale, (e, y[e], expect)


def test_dual_basis_choice_does_not_change_S():
    """Changing the Taylor centre and scale (eq. bf_2 leaves them open) maps the
    dual basis by an invertible matrix C, Q -> CQ, D -> DC^T, M -> CMC^T, so
    D M^-1 Q is unchanged."""
    ops = make_ops(2, 2, 1)
    x = np.random.default_rng(5).standard_normal((ops.mesh.E, ops.Nst))
    y0 = apply_S(ops, x)
    orig = ops.dual_basis

    def moved(j):
        b = orig(j)
        b.x0 = b.x0 + np.array([0.03, -0.02, 0.05])
        b.h = 0.7 * b.h
        return b
    ops2 = make_ops(2, 2, 1)
    ops2.dual_basis = moved
    y1 = apply_S(ops2, x)
    assert np.abs(y1 - y0).max() <= 1e-11 * np.abs(y0).max()


def test_element_renumbering_is_equivariant():
    """Relabelling elements (which also swaps left/right on faces) permutes S."""
    X, T = kuhn_mesh(2, jitter=0.1, seed=2)
    perm = np.random.default_rng(4).permutation(T.shape[0])
    o1 = SpaceTimeOperators(Mesh(X, T), 2, 0, 0.1)
    o2 = SpaceTimeOperators(Mesh(X, T[perm]), 2, 0, 0.1)
    x = np.random.default_rng(6).standard_normal((T.shape[0], o1.Nst))
    y1 = apply_S(o1, x)
    y2 = apply_S(o2, x[perm])
    assert np.abs(y2 - y1[perm]).max() <= 1e-12 * np.abs(y1).max()


@pytest.mark.parametrize("pg", [0, 1])
def test_anchor_equals_consistent_solve_plus_shift(pg):
    """Anchoring node 0 of element 0 (every time node) is the same as solving the
    consistent singular system S x = b~ (b~_a = -sum_{i != a} b_i per time node)
    and shifting so that x_a = 0."""
    ops = make_ops(2, 1, pg, jitter=0.1)
    S = assemble_S(ops)
    rng = np.random.default_rng(8)
    b = rng.standard_normal(S.shape[0])
    xa = solve_anchored(ops, S, b)
    idx = anchor_indices(ops)
    Sd = S.toarray()
    bt = b.copy()
    N, G = ops.N, ops.G
    for a, k in enumerate(idx):
        sl = [e * ops.Nst + a * N + m for e in range(ops.mesh.E) for m in range(N)]
        bt[k] = 0.0
        bt[k] = -bt[sl].sum()
    xc, *_ = np.linalg.lstsq(Sd, bt, rcond=None)
    for a, k in enumerate(idx):
        sl = [e * ops.Nst + a * N + m for e in range(ops.mesh.E) for m in range(N)]
        xc[sl] -= xc[k]
    assert np.abs(xc - xa).max() <= 1e-9 * np.abs(xa).max()
    # and the anchored residual is zero for the anchored solution
    Sa, ba = anchored_system(S, b, idx)
    assert np.linalg.norm(Sa @ xa - ba) <= 1e-10 * np.linalg.norm(ba)
