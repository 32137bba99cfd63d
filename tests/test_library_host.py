"""CPU tests of the library: exported symbols, host-side tables, error paths.

No device computation runs here: meshes are built with stdg_mesh_build_host.
"""

import ctypes
import os
import re

import numpy as np
import pytest

from common import blocks_apply, case_mesh, to_input
from oracle.mesh import Mesh as OracleMesh
from oracle.pressure import apply_S
from oracle.spacetime import SpaceTimeOperators

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

P = pytest.importorskip("paper_1601_07384_amd")
from paper_1601_07384_amd import _lib  # noqa: E402


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(stdg_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_symbols()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in _lib.SIGNATURES}
    assert names <= bound, names - bound


def test_binding_constants_match_header():
    """Every integer #define of the header that the binding names has the
    header's value, and the binding names all method, precision,
    preconditioner, guess and loss constants."""
    txt = open(os.path.join(ROOT, "include", "stdg.h")).read()
    defs = {k: int(v) for k, v in re.findall(r"#define\s+(STDG_[A-Z0-9_]+)\s+(-?\d+)\b", txt)}
    assert len(defs) >= 15
    for k, v in defs.items():
        if hasattr(_lib, k):
            assert getattr(_lib, k) == v, k
    for prefix in ("STDG_FP", "STDG_PRECOND_", "STDG_KRYLOV_", "STDG_LOSS_"):
        for k in defs:
            if k.startswith(prefix):
                assert hasattr(_lib, k), k
    for k in ("STDG_AUTO", "STDG_CG", "STDG_GMRES", "STDG_CG_TIME", "STDG_BICGSTAB"):
        assert getattr(_lib, k) == defs[k], k


@pytest.mark.parametrize("n,p,pg,periodic,jitter", [
    (2, 2, 0, False, 0.0), (2, 1, 1, False, 0.15), (3, 2, 1, True, 0.0),
    (2, 3, 0, False, 0.1), (2, 2, 2, False, 0.0)])
def test_host_tables_match_oracle(n, p, pg, periodic, jitter):
    """The library's Kronecker-factored blocks reproduce the oracle's literal
    space-time operator (eq. CS_19) to 1e-12 relative."""
    X, T = case_mesh(n, jitter=jitter)
    m = P.Mesh(X, T, p, pg, dt=0.05, periodic=periodic, device=False)
    ops = SpaceTimeOperators(OracleMesh(X, T, periodic=periodic), p, pg, 0.05)
    x = np.random.default_rng(1).standard_normal((m.E, m.Nst))
    yo = apply_S(ops, x)
    perm = m.permutation()
    yp = to_input(blocks_apply(m, x[perm]), perm)
    assert np.abs(yp - yo).max() <= 1e-12 * np.abs(yo).max()


def test_kuhn_classes_and_face_counts():
    """A periodic Kuhn mesh has 6 translation classes; face counts 12 n^3
    (periodic) and 12 n^3 - 6 n^2 interior + 12 n^2 boundary (Dirichlet)."""
    X, T = case_mesh(4)
    per = P.Mesh(X, T, 2, 0, periodic=True, device=False)
    assert per.n_classes == 6
    assert per.n_face == per.n_interior_face == 12 * 64
    dr = P.Mesh(X, T, 2, 0, periodic=False, device=False)
    assert dr.n_interior_face == 12 * 64 - 6 * 16
    assert dr.n_face - dr.n_interior_face == 12 * 16


def test_hilbert_permutation_is_a_permutation():
    X, T = case_mesh(3)
    m = P.Mesh(X, T, 1, 0, device=False)
    perm = m.permutation()
    assert sorted(perm.tolist()) == list(range(T.shape[0]))
    m0 = P.Mesh(X, T, 1, 0, device=False, reorder=False)
    assert (m0.permutation() == np.arange(T.shape[0])).all()


def test_error_paths():
    X, T = case_mesh(2)
    with pytest.raises(P.StdgError) as e:
        P.Mesh(X, T, 0, 0, device=False)
    assert e.value.code == _lib.STDG_ERR_ARG
    with pytest.raises(P.StdgError) as e:
        P.Mesh(X, T, 2, 0, dt=-1.0, device=False)
    assert e.value.code == _lib.STDG_ERR_ARG
    # flat element
    Xf = X.copy()
    T2 = T.copy()
    T2[0, 3] = T2[0, 2]
    with pytest.raises(P.StdgError) as e:
        P.Mesh(Xf, T2, 1, 0, device=False)
    assert e.value.code == _lib.STDG_ERR_MESH
    # non-manifold face: duplicate an element
    T3 = np.vstack([T, T[:1]])
    with pytest.raises(P.StdgError) as e:
        P.Mesh(X, T3, 1, 0, device=False)
    assert e.value.code == _lib.STDG_ERR_MESH
    # unmatched periodic face: a box that does not match the mesh
    with pytest.raises(P.StdgError) as e:
        P.Mesh(X, T, 1, 0, periodic=True, box_hi=(2.0, 1.0, 1.0), device=False)
    assert e.value.code == _lib.STDG_ERR_MESH
    # vertex index out of range
    T4 = T.copy(); T4[1, 1] = 10 ** 6
    with pytest.raises(P.StdgError) as e:
        P.Mesh(X, T4, 1, 0, device=False)
    assert e.value.code == _lib.STDG_ERR_ARG


def test_device_entry_points_reject_host_only_handle():
    X, T = case_mesh(2)
    m = P.Mesh(X, T, 1, 0, device=False)
    lib = _lib.load()
    code = lib.stdg_pressure_apply(m._h, 0, ctypes.c_void_p(8), ctypes.c_void_p(16), None)
    assert code == _lib.STDG_ERR_ARG


@pytest.mark.parametrize("n,p,pg,kind,eps,periodic", [
    (2, 2, 0, "bulge", 0.15, False), (3, 2, 1, "periodic", 0.04, True),
    (2, 2, 1, "quadratic", 0.2, False), (1, 3, 0, "bulge", 0.1, False)])
def test_host_curved_tables_match_oracle(n, p, pg, kind, eps, periodic):
    """Curved isoparametric elements (Sec. 2.8): the library's blocks, from its
    own exact reference-coordinate integration, reproduce the oracle's curved
    space-time operator."""
    from oracle.curved import CurvedSpaceTimeOperators, IsoMesh
    from stdg_inputs import curved_mesh, kuhn_mesh
    X, T = kuhn_mesh(n)
    Xc, nodes = curved_mesh(X, T, p, kind, eps)
    m = P.Mesh(Xc, T, p, pg, dt=0.05, periodic=periodic, device=False, nodes=nodes)
    assert m.n_classes == m.E                      # every element curved
    ops = CurvedSpaceTimeOperators(IsoMesh(Xc, T, nodes, p, periodic=periodic), p, pg, 0.05)
    x = np.random.default_rng(1).standard_normal((m.E, m.Nst))
    yo = apply_S(ops, x)
    perm = m.permutation()
    yp = to_input(blocks_apply(m, x[perm]), perm)
    tol = 1e-12 if p <= 2 else 1e-11              # the oracle's degree-25 rule has alternating weights
    assert np.abs(yp - yo).max() <= tol * np.abs(yo).max()


def test_host_curved_straight_nodes_and_partial_curving():
    """Straight nodes give the straight mesh exactly; curving only the
    elements of one hexahedron gives their blocks and their neighbours' their
    own classes while the rest keep the shared ones."""
    from stdg_inputs import curved_mesh, kuhn_mesh, node_coordinates
    X, T = kuhn_mesh(3)
    p = 2
    a = P.Mesh(X, T, p, 0, dt=0.05, periodic=True, device=False)
    b = P.Mesh(X, T, p, 0, dt=0.05, periodic=True, device=False, nodes=node_coordinates(X, T, p))
    assert b.n_classes == a.n_classes == 6
    for u, v in zip(a.blocks(), b.blocks()):
        assert np.array_equal(u, v)
    nodes = node_coordinates(X, T, p)
    hexa = np.arange(6 * 13, 6 * 14)               # the central hexahedron [1/3, 2/3]^3
    # a smooth displacement that vanishes outside the hexahedron, applied by
    # position so shared nodes move together
    u = np.clip((nodes - 1.0 / 3.0) * 3.0, 0.0, 1.0)
    bump = np.prod(np.sin(np.pi * u), axis=-1, keepdims=True)
    bump[bump < 1e-12] = 0.0                       # sin(pi) is not exactly zero
    nodes = nodes + 0.02 * bump * np.array([1.0, -0.5, 0.3])
    assert np.abs(bump[hexa]).max() > 0.5 and np.abs(np.delete(bump, hexa, axis=0)).max() == 0.0
    c = P.Mesh(X, T, p, 0, dt=0.05, periodic=True, device=False, nodes=nodes)
    assert 6 < c.n_classes < c.E
    from oracle.curved import CurvedSpaceTimeOperators, IsoMesh
    ops = CurvedSpaceTimeOperators(IsoMesh(X, T, nodes, p, periodic=True), p, 0, 0.05)
    x = np.random.default_rng(3).standard_normal((c.E, c.Nst))
    perm = c.permutation()
    yp = to_input(blocks_apply(c, x[perm]), perm)
    sample = sorted(set(hexa.tolist()) | {0, 50, 100, 161})
    yo = apply_S(ops, x, elements=sample)
    assert np.abs(yp[sample] - yo[sample]).max() <= 1e-12 * np.abs(yo[sample]).max()


def test_curved_mesh_errors():
    from stdg_inputs import curved_mesh, kuhn_mesh
    X, T = kuhn_mesh(2)
    Xc, nodes = curved_mesh(X, T, 2, "bulge", 0.1)
    bad = nodes.copy()
    bad[3, 0] += 1e-3                               # a vertex node off its vertex
    with pytest.raises(RuntimeError, match="vertex nodes"):
        P.Mesh(Xc, T, 2, 0, device=False, nodes=bad)
    bad = nodes.copy()
    bad[5, 1] += 1e-2                               # an edge node of one element only
    with pytest.raises(RuntimeError, match="non-conforming"):
        P.Mesh(Xc, T, 2, 0, device=False, nodes=bad)
    with pytest.raises(ValueError):
        P.Mesh(Xc, T, 2, 0, device=False, nodes=nodes[:, :5])
    # an interior edge node pushed through the element (the same for every
    # element sharing the edge): the map folds
    from stdg_inputs import node_coordinates
    X3, T3 = kuhn_mesh(3)
    n3 = node_coordinates(X3, T3, 2)
    centre = np.array([0.5, 0.5, 0.5])
    moved = np.abs(n3 - centre).max(axis=-1) < 1e-12
    assert moved.any()
    n3[moved] += np.array([0.3, 0.3, -0.3])
    with pytest.raises(RuntimeError, match="folds"):
        P.Mesh(X3, T3, 2, 0, device=False, nodes=n3)
