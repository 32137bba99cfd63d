"""Curved isoparametric elements (Sec. 2.8) on the device.

The curved geometry changes only the precomputed blocks (every curved
element and its neighbours get blocks of their own), so these cases run the
class-mixed kernels of the unstructured meshes: the FP64 apply against the
oracle's curved space-time operator, the solves against its anchored direct
solve, and a 24,576-element curved cube (sampled rows, refinement solve).
"""

import time

import numpy as np
import pytest

from common import to_input
from stdg_inputs import curved_mesh, kuhn_mesh
from oracle.curved import CurvedSpaceTimeOperators, IsoMesh
from oracle.pressure import apply_S, assemble_S, solve_anchored

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1601_07384_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def gpu(v, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(v), dtype=dtype, device=DEV)


def build(n, p, pg, kind, eps, periodic, dt):
    X, T = kuhn_mesh(n)
    Xc, nodes = curved_mesh(X, T, p, kind, eps)
    m = P.Mesh(Xc, T, p, pg, dt=dt, periodic=periodic, nodes=nodes)
    return m, (Xc, T, nodes)


def oracle_ops(geo, p, pg, periodic, dt):
    Xc, T, nodes = geo
    return CurvedSpaceTimeOperators(IsoMesh(Xc, T, nodes, p, periodic=periodic), p, pg, dt)


@pytest.mark.parametrize("n,p,pg,kind,eps,periodic", [
    (2, 2, 1, "bulge", 0.15, False), (3, 2, 0, "periodic", 0.04, True), (1, 3, 1, "bulge", 0.1, False),
    (3, 1, 1, "periodic", 0.04, True)])
def test_curved_apply_matches_oracle(n, p, pg, kind, eps, periodic):
    print(f"curved apply n={n} p={p} pg={pg} {kind}", flush=True)
    m, geo = build(n, p, pg, kind, eps, periodic, 0.05)
    ops = oracle_ops(geo, p, pg, periodic, 0.05)
    x = np.random.default_rng(2).standard_normal((m.E, m.Nst))
    yo = apply_S(ops, x)
    perm = m.permutation()
    xg = gpu(x[perm].ravel())
    yg = torch.empty_like(xg)
    m.apply(xg, yg)
    torch.cuda.synchronize()
    y = to_input(yg.cpu().numpy().reshape(m.E, m.Nst), perm)
    tol = 1e-12 if p <= 2 else 1e-11              # the oracle's degree-25 rule at p = 3
    assert np.abs(y - yo).max() <= tol * np.abs(yo).max()


@pytest.mark.parametrize("method,precision", [(P.STDG_CG_TIME, P.STDG_FP32), (P.STDG_GMRES, P.STDG_FP64),
                                              (P.STDG_CG_TIME, P.STDG_FP64)])
def test_curved_solve_matches_oracle(method, precision):
    print(f"curved solve method={method} precision={precision}", flush=True)
    p, pg, dt = 2, 1, 1e-2
    m, geo = build(3, p, pg, "periodic", 0.04, True, dt)
    ops = oracle_ops(geo, p, pg, True, dt)
    S = assemble_S(ops)
    rng = np.random.default_rng(12)
    xt = rng.standard_normal(S.shape[0])
    b = S @ xt + 1e-3 * np.abs(S @ xt).max() * rng.standard_normal(S.shape[0])
    xo = solve_anchored(ops, S, b).reshape(m.E, m.Nst)
    perm = m.permutation()
    bg = gpu(b.reshape(m.E, m.Nst)[perm].ravel())
    xg = torch.zeros_like(bg)
    rep = m.solve(bg, xg, method=method, precision=precision, rtol=1e-12, restart=40)
    assert rep.status == 0, (rep.status, rep.rel_residual)
    assert rep.rel_residual <= 1e-12
    xs = to_input(xg.cpu().numpy().reshape(m.E, m.Nst), perm)
    assert np.abs(xs - xo).max() <= 1e-8 * np.abs(xo).max()


def test_curved_mesh_rejects_picard_step():
    m, _ = build(2, 2, 0, "bulge", 0.1, False, 1e-2)
    vbar = torch.zeros(3 * m.E * m.Nst, dtype=torch.float64, device=DEV)
    vhat = torch.zeros(3 * m.n_face * m.Nst, dtype=torch.float64, device=DEV)
    with pytest.raises(RuntimeError, match="curved"):
        m.dual_from_main(vbar, vhat)


def test_curved_cube_16_sampled_rows_and_refinement_solve():
    """16^3 x 6 = 24,576 curved tets, p = 2, p_gamma = 1, periodic: every
    element its own block set; sampled FP64 rows against the oracle, and the
    FP32-refined time-decoupled CG solve to 1e-10 against FP64 CG."""
    p, pg, dt = 2, 1, 1e-3
    t0 = time.perf_counter()
    m, geo = build(16, p, pg, "periodic", 0.02, True, dt)
    build_s = time.perf_counter() - t0
    assert m.n_classes == m.E
    rng = np.random.default_rng(21)
    x = rng.standard_normal((m.E, m.Nst))
    perm = m.permutation()
    xg = gpu(x[perm].ravel())
    yg = torch.empty_like(xg)
    m.apply(xg, yg)
    torch.cuda.synchronize()
    y = to_input(yg.cpu().numpy().reshape(m.E, m.Nst), perm)
    rows = np.concatenate([rng.choice(m.E, size=8, replace=False), [0, m.E - 1]])
    yo = apply_S(oracle_ops(geo, p, pg, True, dt), x, elements=rows)
    assert np.abs(y[rows] - yo[rows]).max() <= 1e-12 * np.abs(yo[rows]).max()
    b = torch.empty_like(xg)
    m.apply(gpu(rng.standard_normal(m.E * m.Nst)), b)
    out = {}
    for prec in (P.STDG_FP32, P.STDG_FP64):
        xs = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = m.solve(b, xs, method=P.STDG_CG_TIME, precision=prec, rtol=1e-10, inner_rtol=1e-5, max_iter=100000)
        torch.cuda.synchronize()
        out[prec] = (xs, rep, time.perf_counter() - t0)
        assert rep.status == P.STDG_OK and rep.rel_residual <= 1e-10
    err = float((out[P.STDG_FP32][0] - out[P.STDG_FP64][0]).abs().max() / out[P.STDG_FP64][0].abs().max())
    print(f"curved 16^3 p=2 pg=1: build {build_s:.1f} s, FP32 refinement {out[P.STDG_FP32][2] * 1e3:.1f} ms "
          f"({out[P.STDG_FP32][1].inner_iters} inner it), FP64 CG {out[P.STDG_FP64][2] * 1e3:.1f} ms "
          f"({out[P.STDG_FP64][1].inner_iters} it), difference {err:.2e}", flush=True)
    assert err <= 1e-7
