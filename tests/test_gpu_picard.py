"""GPU parity of the Picard time step (Sec. 2.6) against the oracle.

The library's step (averaging, Lambda, convection with the Rusanov flux,
viscous solve, goback, pressure correction, velocity update) is compared with
the oracle's literal space-time step on the same seeded data.  Velocities are
compared as dual-element coefficients (faces matched through the element
numbering) and main-grid coefficients; the pressure to 1e-8 relative.
"""

import numpy as np
import pytest

from stdg_inputs import (kuhn_mesh, node_coordinates, node_reference_points, beltrami_velocity,
                         fourier_modes, fourier_velocity, time_nodes)
from oracle.mesh import Mesh as OracleMesh
from oracle.picard import divergence, initial_state, picard_step
from oracle.pressure import anchor_indices
from oracle.spacetime import SpaceTimeOperators

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1601_07384_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def nodal(X, T, p, G, fn, t0=0.0, dt=0.0):
    """(E, 3, G*N) nodal values of fn(x, t) at the slab's time nodes."""
    xn = node_coordinates(X, T, p)
    tau = time_nodes(G)
    return np.concatenate([np.transpose(fn(xn, t0 + dt * ta), (0, 2, 1)) for ta in tau], axis=2)


def to_dev_main(v, perm):
    """(E, 3, Nst) input order -> device [3][E][G][N] internal order."""
    return torch.tensor(np.ascontiguousarray(np.transpose(v[perm], (1, 0, 2))).ravel(),
                        dtype=torch.float64, device=DEV)


def from_dev_main(t, perm, E, Nst):
    v = t.cpu().numpy().reshape(3, E, Nst).transpose(1, 0, 2)
    out = np.empty_like(v)
    out[perm] = v
    return out


def face_map(m, om, perm):
    left, lf, _, _ = m.faces()
    return np.array([om.tet_faces[perm[l], f] for l, f in zip(left, lf)])


def from_dev_dual(t, fmap, F, Nst):
    v = t.cpu().numpy().reshape(3, F, Nst).transpose(1, 0, 2)
    out = np.empty_like(v)
    out[fmap] = v
    return out


def dual_values(ops, vh):
    """Values of every dual element's space-time velocity (F, 3, Nst) at the
    degree-p nodes of its sub-tetrahedra (unisolvent, so two dual fields
    agree iff these values do).  The Taylor coefficients of eq. bf_2 are not
    compared directly: the dual mass matrices reach condition numbers near
    1e9 at p = 4, so FP64 coefficients differ by up to that many ulps while
    the fields they represent agree to rounding."""
    ref = np.asarray(node_reference_points(ops.p), np.float64)
    out = []
    for j in range(ops.mesh.F):
        sides = (0, 1) if ops.mesh.right[j] >= 0 else (0,)
        pts = np.vstack([ops.mesh.subtet(j, s)[:1] + ref @ (ops.mesh.subtet(j, s)[1:] - ops.mesh.subtet(j, s)[:1])
                         for s in sides])
        V = ops.dual_basis(j).eval(pts)                                   # longdouble (m, N)
        c = np.asarray(vh[j], np.longdouble).reshape(3, ops.G, -1)
        out.append(np.einsum("mk,cgk->mcg", V, c).astype(np.float64).ravel())
    return np.concatenate(out)


def dual_close(ops, a, b, rtol):
    va, vb = dual_values(ops, a), dual_values(ops, b)
    err = np.abs(va - vb).max() / np.abs(vb).max()
    print(f"  dual field relative difference {err:.3e}", flush=True)
    return err <= rtol


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


_ORACLE = {}


def oracle_step(n, p, pg, periodic, nu, dt, n_pic, field, jitter):
    """Mesh, inputs and the oracle's step for one case (cached per case: the
    viscous-solver variants of a case share one oracle run)."""
    key = (n, p, pg, periodic, nu, dt, n_pic, field, jitter)
    if key not in _ORACLE:
        X, T = kuhn_mesh(n, jitter=jitter, seed=3)
        om = OracleMesh(X, T, periodic=periodic)
        ops = SpaceTimeOperators(om, p, pg, dt)
        G = pg + 1
        if field == "beltrami":
            fn = lambda x, t: beltrami_velocity(x, t, nu)
        else:
            modes = fourier_modes(seed=1601, n_modes=6, kmax=2)
            fn = lambda x, t: fourier_velocity(x, modes)
        u0 = nodal(X, T, p, G, lambda x, t: fn(x, 0.0))
        g = nodal(X, T, p, G, fn, 0.0, dt)
        vh0 = initial_state(ops, u0)
        vh_o, vb_o, p_o, _ = picard_step(ops, vh0, u0, g, nu, n_pic)
        _ORACLE[key] = (X, T, om, ops, u0, g, vh0, (vh_o, vb_o, p_o))
    return _ORACLE[key]


def run_both(n, p, pg, periodic, nu, dt, n_pic, field, viscous_method=None, jitter=0.0):
    # unpreconditioned restarted GMRES (the default for p_gamma > 0) needs
    # more than 20000 iterations for 1e-13 at p = 4; the time-decoupled CG
    # solves the same system in a few hundred
    pressure = {"rtol": 1e-13}
    if p >= 4 or (p >= 3 and pg >= 1 and n >= 4):
        pressure["method"] = P.STDG_CG_TIME
    X, T, om, ops, u0, g, vh0, (vh_o, vb_o, p_o) = oracle_step(n, p, pg, periodic, nu, dt, n_pic, field, jitter)
    m = P.Mesh(X, T, p, pg, dt=dt, nu=nu, periodic=periodic)
    perm = m.permutation()
    fmap = face_map(m, om, perm)
    vbar = to_dev_main(u0, perm)
    vhat = torch.empty(3 * m.n_face * m.Nst, dtype=torch.float64, device=DEV)
    m.dual_from_main(vbar, vhat)
    torch.cuda.synchronize()
    vh0_g = from_dev_dual(vhat, fmap, m.n_face, m.Nst)
    # values through the Taylor dual mass inverses (condition ~3e9 at p = 4,
    # growing about tenfold per degree) carry that much more FP64 rounding
    assert dual_close(ops, vh0_g, vh0, 1e-11 if p <= 4 else 1e-10)
    pg_dev = torch.zeros(m.E * m.Nst, dtype=torch.float64, device=DEV)
    gd = to_dev_main(g, perm) if not periodic else None
    visc = {"rtol": 1e-13}
    if viscous_method is not None:
        visc.update(method=viscous_method, restart=30)
    rep = m.picard_step(vhat, vbar, pg_dev, gd, n_picard=n_pic, pressure=pressure, viscous=visc)
    vh_g = from_dev_dual(vhat, fmap, m.n_face, m.Nst)
    vb_g = from_dev_main(vbar, perm, m.E, m.Nst)
    p_g = np.empty((m.E, m.Nst))
    p_g[perm] = pg_dev.cpu().numpy().reshape(m.E, m.Nst)
    return (vh_o, vb_o, p_o), (vh_g, vb_g, p_g), rep, (ops, m)


CASES = [  # n, p, p_gamma, periodic, nu, dt, n_pic, field
    (2, 2, 0, False, 1e-2, 1e-2, 2, "beltrami"),
    (2, 2, 1, False, 5e-2, 2e-2, 2, "beltrami"),
    (3, 2, 1, True, 1e-2, 1e-2, 2, "fourier"),
    (2, 3, 0, False, 1e-1, 1e-2, 1, "beltrami"),
    (3, 1, 2, True, 1e-3, 5e-3, 3, "fourier"),
    (6, 2, 0, False, 1e-2, 1e-2, 2, "beltrami"),   # 6^3 x 6 unit cube, one step, 2 Picard
    (1, 4, 1, False, 5e-2, 2e-2, 2, "beltrami"),   # degrees of the convergence tables on one cube
    (1, 5, 0, False, 1e-1, 1e-2, 1, "beltrami"),
    (1, 3, 3, False, 1.0, 1e-2, 2, "beltrami"),
    (1, 1, 4, False, 1.0, 1e-2, 2, "beltrami"),
]


@pytest.mark.parametrize("n,p,pg,periodic,nu,dt,n_pic,field", CASES)
def test_picard_step_matches_oracle(n, p, pg, periodic, nu, dt, n_pic, field):
    print(f"picard case n={n} p={p} pg={pg} periodic={periodic}", flush=True)
    (vh_o, vb_o, p_o), (vh_g, vb_g, p_g), rep, (ops, _) = run_both(n, p, pg, periodic, nu, dt, n_pic, field)
    print(f"  vbar {rel(vb_g, vb_o):.3e}  p {rel(p_g, p_o):.3e}  residuals {rep.max_pressure_residual:.2e} "
          f"{rep.max_viscous_residual:.2e}", flush=True)
    assert dual_close(ops, vh_g, vh_o, 1e-9)
    assert rel(vb_g, vb_o) <= 1e-9
    assert rel(p_g, p_o) <= 1e-8
    assert rep.max_pressure_residual <= 1e-12


@pytest.mark.parametrize("n,p,pg,periodic,nu,dt,n_pic,field", [CASES[1], CASES[4]])
def test_picard_step_bicgstab_viscous(n, p, pg, periodic, nu, dt, n_pic, field):
    """The same step with the viscous systems solved by preconditioned
    BiCGStab instead of GMRES."""
    print(f"picard bicgstab case n={n} p={p} pg={pg} periodic={periodic}", flush=True)
    (vh_o, vb_o, p_o), (vh_g, vb_g, p_g), rep, (ops, _) = run_both(n, p, pg, periodic, nu, dt, n_pic, field,
                                                                   viscous_method=P.STDG_BICGSTAB)
    assert dual_close(ops, vh_g, vh_o, 1e-9)
    assert np.abs(vb_g - vb_o).max() <= 1e-9 * np.abs(vb_o).max()
    assert np.abs(p_g - p_o).max() <= 1e-8 * np.abs(p_o).max()
    assert rep.max_viscous_residual <= 1e-12


# Periodic 4^3 x 6 cube: 384 elements in 6 geometry classes, so every
# wavefront of the element kernels holds one class (n_classes * 64 <= E) and
# the step runs the class-uniform variants that the large periodic meshes
# use: convection kf_convection<N, G, false>, viscous operator k_visc_tn<N, G>
# and viscous block-Jacobi kf_blockdiag<N G>.  One Picard iteration at
# (3, 1), where the oracle's literal space-time step is the slowest.
UNIFORM = [  # n, p, p_gamma, periodic, nu, dt, n_pic, field
    (4, 2, 1, True, 1e-2, 1e-2, 2, "fourier"),
    (4, 3, 0, True, 1e-2, 1e-2, 2, "fourier"),
    (4, 3, 1, True, 1e-2, 1e-2, 1, "fourier"),
]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("viscous", ["gmres", "bicgstab"])
@pytest.mark.parametrize("n,p,pg,periodic,nu,dt,n_pic,field", UNIFORM)
def test_picard_step_class_uniform_kernels(n, p, pg, periodic, nu, dt, n_pic, field, viscous):
    N, G = (p + 1) * (p + 2) * (p + 3) // 6, pg + 1
    print(f"uniform-class case p={p} pg={pg} viscous={viscous}: kf_convection<{N},{G},false>, "
          f"k_visc_tn<{N},{G}>, kf_blockdiag<{N * G}>", flush=True)
    method = P.STDG_GMRES if viscous == "gmres" else P.STDG_BICGSTAB
    (vh_o, vb_o, p_o), (vh_g, vb_g, p_g), rep, (ops, m) = run_both(n, p, pg, periodic, nu, dt, n_pic, field,
                                                                   viscous_method=method)
    assert m.n_classes * 64 <= m.E, (m.n_classes, m.E)
    print(f"  classes {m.n_classes} of {m.E}  vbar {rel(vb_g, vb_o):.3e}  p {rel(p_g, p_o):.3e}  "
          f"residuals {rep.max_pressure_residual:.2e} {rep.max_viscous_residual:.2e}", flush=True)
    assert dual_close(ops, vh_g, vh_o, 1e-9)
    assert rel(vb_g, vb_o) <= 1e-9
    assert rel(p_g, p_o) <= 1e-8
    assert rep.max_pressure_residual <= 1e-12
    assert rep.max_viscous_residual <= 1e-12


@pytest.mark.parametrize("n,p,pg,periodic,nu,dt,n_pic,field,jitter",
                         [(2, 2, 0, False, 1e-2, 1e-2, 2, "beltrami", 0.15),
                          (3, 2, 1, True, 1e-2, 1e-2, 2, "fourier", 0.1),
                          (3, 3, 0, True, 1e-2, 1e-2, 1, "fourier", 0.1)])
def test_picard_step_jittered_matches_oracle(n, p, pg, periodic, nu, dt, n_pic, field, jitter):
    """Unstructured meshes (every element its own geometry class, so every
    wavefront mixes classes) through the same step."""
    print(f"picard jittered case n={n} p={p} pg={pg} periodic={periodic}", flush=True)
    (vh_o, vb_o, p_o), (vh_g, vb_g, p_g), rep, (ops, m) = run_both(n, p, pg, periodic, nu, dt, n_pic, field,
                                                                   jitter=jitter)
    assert m.n_classes == m.E or not periodic
    print(f"  classes {m.n_classes} of {m.E}  vbar {rel(vb_g, vb_o):.3e}  p {rel(p_g, p_o):.3e}", flush=True)
    assert dual_close(ops, vh_g, vh_o, 1e-9)
    assert rel(vb_g, vb_o) <= 1e-9
    assert rel(p_g, p_o) <= 1e-8
    assert rep.max_pressure_residual <= 1e-12


def test_picard_step_divergence_free_on_device():
    """eq. CS_15 after a device step, evaluated by the library (all elements
    but the anchor) and by the oracle on the device result."""
    (vh_o, _, _), (vh_g, _, _), _, (ops, m) = run_both(3, 2, 1, True, 1e-2, 1e-2, 2, "fourier")
    div = divergence(ops, vh_g)
    div[0] = 0.0
    assert np.abs(div).max() <= 1e-9 * np.abs(vh_g).max()


def test_steady_linear_flow_c1_mesh():
    """6^3 x 6 mesh, p=2: u = A x, q = -x.A^2.x/2 is reproduced by one device
    step with nu = 1e-2 and the previous-pressure guess (exact steady state)."""
    A = np.array([[0.3, 0.2, -0.1], [0.2, -0.5, 0.4], [-0.1, 0.4, 0.2]])
    X, T = kuhn_mesh(6)
    p, pg, dt, nu = 2, 0, 1e-2, 1e-2
    m = P.Mesh(X, T, p, pg, dt=dt, nu=nu)
    perm = m.permutation()
    u = nodal(X, T, p, 1, lambda x, t: x @ A.T)
    xn = node_coordinates(X, T, p)
    q = -0.5 * np.einsum("...i,ij,...j->...", xn, A @ A, xn)
    q = q - q[0, 0]
    vbar = to_dev_main(u, perm)
    vhat = torch.empty(3 * m.n_face * m.Nst, dtype=torch.float64, device=DEV)
    m.dual_from_main(vbar, vhat)
    vh0 = vhat.clone()
    pd = torch.tensor(q[perm].ravel(), dtype=torch.float64, device=DEV)
    m.picard_step(vhat, vbar, pd, to_dev_main(u, perm), n_picard=2,
                  pressure_guess=P.STDG_GUESS_PREVIOUS, pressure={"rtol": 1e-13},
                  viscous={"rtol": 1e-13})
    assert float((vhat - vh0).abs().max()) <= 1e-10 * float(vh0.abs().max())
    pr = np.empty_like(q)
    pr[perm] = pd.cpu().numpy().reshape(q.shape)
    assert np.abs(pr - q).max() <= 1e-9 * np.abs(q).max()


@pytest.mark.parametrize("theta", [0.5, 0.75])
@pytest.mark.parametrize("guess", ["zero", "previous"])
def test_theta_method_matches_oracle(theta, guess):
    """theta-method for p_gamma = 0 (Sec. 2.7, eqs. CS_15_theta-CS_16_theta):
    the library solves for the weighted pressure and recovers p^{n+1} at the
    end; the oracle takes the literal theta S dp = b form."""
    print(f"theta case theta={theta} guess={guess}", flush=True)
    n, p, nu, dt, n_pic = 2, 2, 1e-2, 1e-2, 2
    X, T = kuhn_mesh(n)
    om = OracleMesh(X, T)
    ops = SpaceTimeOperators(om, p, 0, dt)
    fn = lambda x, t: beltrami_velocity(x, t, nu)
    u0 = nodal(X, T, p, 1, lambda x, t: fn(x, 0.0))
    g = nodal(X, T, p, 1, fn, 0.0, dt)
    p_prev = np.random.default_rng(5).standard_normal((om.E, ops.Nst))
    vh0 = initial_state(ops, u0)
    vh_o, vb_o, p_o, _ = picard_step(ops, vh0, u0, g, nu, n_pic, theta=theta, p_prev=p_prev,
                                     p_init=p_prev if guess == "previous" else None)
    m = P.Mesh(X, T, p, 0, dt=dt, nu=nu)
    perm = m.permutation()
    fmap = face_map(m, om, perm)
    vbar = to_dev_main(u0, perm)
    vhat = torch.empty(3 * m.n_face * m.Nst, dtype=torch.float64, device=DEV)
    m.dual_from_main(vbar, vhat)
    pd = torch.tensor(np.ascontiguousarray(p_prev[perm]).ravel(), dtype=torch.float64, device=DEV)
    opts = P.step_opts(n_picard=n_pic, theta=theta, pressure={"rtol": 1e-13}, viscous={"rtol": 1e-13},
                       pressure_guess=P.STDG_GUESS_PREVIOUS if guess == "previous" else P.STDG_GUESS_ZERO)
    rep = m.picard_step(vhat, vbar, pd, to_dev_main(g, perm), opts=opts)
    vh_g = from_dev_dual(vhat, fmap, m.n_face, m.Nst)
    vb_g = from_dev_main(vbar, perm, m.E, m.Nst)
    p_g = np.empty((m.E, m.Nst))
    p_g[perm] = pd.cpu().numpy().reshape(m.E, m.Nst)
    print(f"  vbar {rel(vb_g, vb_o):.3e}  p {rel(p_g, p_o):.3e}", flush=True)
    assert rep.status == P.STDG_OK
    assert dual_close(ops, vh_g, vh_o, 1e-9)
    assert rel(vb_g, vb_o) <= 1e-9
    assert rel(p_g, p_o) <= 1e-8


def test_theta_method_rejected_for_space_time_pressure():
    X, T = kuhn_mesh(2)
    m = P.Mesh(X, T, 1, 1, dt=1e-2, nu=1e-2)
    vbar = torch.zeros(3 * m.E * m.Nst, dtype=torch.float64, device=DEV)
    vhat = torch.zeros(3 * m.n_face * m.Nst, dtype=torch.float64, device=DEV)
    pd = torch.zeros(m.E * m.Nst, dtype=torch.float64, device=DEV)
    with pytest.raises(P.StdgError):
        m.picard_step(vhat, vbar, pd, vbar, opts=P.step_opts(theta=0.5))
