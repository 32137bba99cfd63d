"""Pins of the oracle's curved (isoparametric) pressure operator, Sec. 2.8.

Each test checks the curved matrices against something other than their own
formulas:

* straight nodes: the curved construction (integrals in reference
  coordinates through the isoparametric map) reduces to the straight oracle
  (integrals on the physical sub-tetrahedra), a separately pinned code path;
* the total volume of a domain deformed by a quadratic map, which degree-2
  elements reproduce exactly, is the closed-form integral of det grad F;
* Corollaries 1-2 (p_gamma = 0): S symmetric positive semi-definite with the
  constants as null space, on curved periodic and curved Dirichlet meshes;
* Green's formula: isoparametric elements reproduce linear functions, so for
  a global linear pressure the velocity response is its constant gradient
  and the rows of elements whose faces are all interior vanish (the
  divergence theorem on each curved element ties the volume measure, the
  mapped gradients and the curved face normals together);
* a rigid motion of the curved mesh leaves S unchanged.
"""

import math

import numpy as np
import pytest

from stdg_inputs import curved_mesh, kuhn_mesh, node_coordinates
from oracle.curved import CurvedSpaceTimeOperators, IsoMesh
from oracle.mesh import Mesh
from oracle.pressure import apply_S, assemble_S
from oracle.spacetime import SpaceTimeOperators


def curved_ops(n, p, pg, kind, eps, periodic=False, dt=0.1, transform=None):
    X, T = kuhn_mesh(n)
    Xc, nodes = curved_mesh(X, T, p, kind, eps)
    if transform is not None:
        Xc, nodes = transform(Xc), transform(nodes)
    return CurvedSpaceTimeOperators(IsoMesh(Xc, T, nodes, p, periodic=periodic), p, pg, dt)


@pytest.mark.parametrize("n,p,pg,periodic,jitter", [(2, 2, 1, False, 0.1), (3, 2, 0, True, 0.0),
                                                     (2, 1, 0, False, 0.15)])
def test_straight_nodes_reduce_to_straight_operator(n, p, pg, periodic, jitter):
    X, T = kuhn_mesh(n, jitter=jitter, seed=3)
    a = SpaceTimeOperators(Mesh(X, T, periodic=periodic), p, pg, 0.1)
    b = CurvedSpaceTimeOperators(IsoMesh(X, T, node_coordinates(X, T, p), p, periodic=periodic), p, pg, 0.1)
    x = np.random.default_rng(1).standard_normal((T.shape[0], a.Nst))
    ya, yb = apply_S(a, x), apply_S(b, x)
    assert np.abs(ya - yb).max() <= 1e-13 * np.abs(ya).max()


def test_quadratic_map_volume_is_exact():
    """F(x) = (x + a x^2, y + b y z, z + c x y): det grad F =
    (1 + 2 a x)(1 + b z - b c x y), whose integral over the unit cube is
    1 + a + b/2 - b c/4 + a b/2 - a b c/3.  The dual elements
    (with the single sub-tetrahedron of a boundary face) tile the domain, and
    the first Taylor function is 1, so sum_j Mbar_j[0, 0] = dt vol (G = 1)."""
    eps, dt = 0.2, 0.1
    a, b, c = eps * 1.0, eps * 0.5, eps * -0.7
    ops = curved_ops(2, 2, 0, "quadratic", eps, dt=dt)
    vol = sum(ops.face(j)["Mbar"][0, 0] for j in range(ops.mesh.F)) / dt
    exact = 1 + a + b / 2 - b * c / 4 + a * b / 2 - a * b * c / 3
    assert abs(float(vol) - exact) <= 1e-14
    # and the map is not affine: the straight skeleton has a different volume
    straight = SpaceTimeOperators(Mesh(ops.mesh.X, ops.mesh.tets), 2, 0, dt)
    vs = sum(straight.face(j)["Mbar"][0, 0] for j in range(straight.mesh.F)) / dt
    assert abs(float(vs) - exact) > 1e-4


@pytest.mark.parametrize("n,kind,periodic", [(3, "periodic", True), (2, "bulge", False)])
def test_curved_operator_symmetric_psd_constant_nullspace(n, kind, periodic):
    ops = curved_ops(n, 2, 0, kind, 0.04 if periodic else 0.15, periodic=periodic)
    S = assemble_S(ops).toarray()
    scale = np.abs(S).max()
    assert np.abs(S - S.T).max() <= 1e-13 * scale
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev.min() >= -1e-12 * ev.max()
    assert np.sum(ev < 1e-10 * ev.max()) == 1
    assert np.abs(S @ np.ones(S.shape[0])).max() <= 1e-13 * scale


@pytest.mark.parametrize("pg", [0, 1])
def test_linear_pressure_rows_vanish_on_curved_elements(pg):
    """Green's formula (the closed form of the straight pin with Lap q = 0)."""
    p = 2
    ops = curved_ops(3, p, pg, "bulge", 0.15)
    mesh = ops.mesh
    coef = np.array([0.3, -1.1, 0.7])
    qn = np.asarray(mesh.nodes, dtype=np.float64) @ coef + 0.4       # (E, N): exact in the space
    x = np.tile(qn, (1, ops.G))
    inner = [e for e in range(mesh.E) if all(mesh.neighbour(e, f)[0] >= 0 for f in range(4))]
    assert len(inner) > 10
    # the interior elements touch curved elements: their nodes are off the straight positions
    straight = node_coordinates(mesh.X, mesh.tets, p)
    assert max(np.abs(np.asarray(mesh.nodes[e], dtype=np.float64) - straight[e]).max() for e in inner) > 1e-3
    sample = inner[::3]
    y = apply_S(ops, x, elements=sample)
    full = apply_S(ops, np.random.default_rng(2).standard_normal(x.shape), elements=sample)
    scale = np.abs(full[sample]).max() * np.abs(qn).max()
    for e in sample:
        assert np.abs(y[e]).max() <= 1e-12 * scale, (e, np.abs(y[e]).max(), scale)


def test_rigid_motion_leaves_curved_operator_unchanged():
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th), 0.0], [math.sin(th), math.cos(th), 0.0], [0.0, 0.0, 1.0]])
    R = R @ np.array([[1.0, 0.0, 0.0], [0.0, math.cos(0.4), -math.sin(0.4)], [0.0, math.sin(0.4), math.cos(0.4)]])
    shift = np.array([0.3, -1.2, 2.0])
    a = curved_ops(2, 2, 1, "bulge", 0.15)
    b = curved_ops(2, 2, 1, "bulge", 0.15, transform=lambda y: y @ R.T + shift)
    x = np.random.default_rng(4).standard_normal((a.mesh.E, a.Nst))
    ya, yb = apply_S(a, x), apply_S(b, x)
    assert np.abs(ya - yb).max() <= 1e-12 * np.abs(ya).max()
    # the deformation matters: the straight skeleton's operator differs
    s = SpaceTimeOperators(Mesh(a.mesh.X, a.mesh.tets), 2, 1, 0.1)
    assert np.abs(apply_S(s, x) - ya).max() > 1e-3 * np.abs(ya).max()
