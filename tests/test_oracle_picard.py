"""Pins of the oracle's Picard time step (Sec. 2.6) against closed forms.

* A linear velocity u = A x with A symmetric and trace-free, with pressure
  q = -x.A^2.x/2, is an exact steady Navier-Stokes solution for every nu:
  (u.grad)u = A^2 x = -grad q, Lap u = 0, div u = 0.  Every integrand of the
  scheme is then a polynomial integrated exactly, the Rusanov jump vanishes,
  and one time step must return u and q (up to the anchor constant) to
  round-off: with p^{n+1,0} = 0 when nu = 0 (the first correction recovers q
  exactly), and for any nu when p^{n+1,0} = q.
* Discrete divergence-freeness (eq. CS_15) after a step on every element but
  the anchor.
* Corollaries 3-4: the viscous system is symmetric positive definite for
  p_gamma = 0.
* theta-method (Sec. 2.7, eqs. CS_15_theta-CS_16_theta): with the
  previous pressure p^n = q the same steady linear flow is returned for
  theta = 1/2 and 3/4 (a dropped (1 - theta) p^n term returns q / theta);
  the step stays divergence-free (a correction not scaled by theta breaks
  eq. CS_15_theta); and with pi = theta p + (1 - theta) p^n the step is the
  theta = 1 step in pi started from theta p^{n+1,0} + (1 - theta) p^n.
* Convection of a continuous polynomial field equals int phi~ div(u (x) u)
  (Green's formula; the Rusanov jump is zero), and for piecewise-constant
  states only face terms remain: sum_f int phi (F^RS - F(v_i)).n.
"""

import numpy as np
import pytest

from stdg_inputs import kuhn_mesh, node_coordinates, beltrami_velocity
from oracle.basis import TetMap, nodal_phys
from oracle.mesh import Mesh
from oracle.pressure import anchor_indices
from oracle.picard import (convection, divergence, goback, initial_state, picard_step,
                           viscous_matrix)
from oracle.quadrature import simplex_rule, triangle_rule_3d
from oracle.spacetime import SpaceTimeOperators

A = np.array([[0.3, 0.2, -0.1], [0.2, -0.5, 0.4], [-0.1, 0.4, 0.2]])   # symmetric, trace 0


def _nodal_field(ops, fn):
    """(E, 3, Nst) nodal values of a steady field fn(x) -> (..., 3)."""
    xn = node_coordinates(ops.mesh.X, ops.mesh.tets, ops.p)            # (E, N, 3)
    v = fn(xn)                                                          # (E, N, 3)
    return np.tile(np.transpose(v, (0, 2, 1)), (1, 1, ops.G))


def _nodal_scalar(ops, fn):
    xn = node_coordinates(ops.mesh.X, ops.mesh.tets, ops.p)
    return np.tile(fn(xn), (1, ops.G))


def _run_linear(pg, nu, use_exact_guess, theta=1.0):
    X, T = kuhn_mesh(2)
    ops = SpaceTimeOperators(Mesh(X, T), 2, pg, 0.05)
    u = _nodal_field(ops, lambda x: x @ A.T)
    q = _nodal_scalar(ops, lambda x: -0.5 * np.einsum("...i,ij,...j->...", x, A @ A, x))
    idx = anchor_indices(ops)
    q = q - q.ravel()[idx[0]]                           # anchored at node 0 of element 0
    vhat0 = initial_state(ops, u)
    vhat, vbar, p, _ = picard_step(ops, vhat0, u, u, nu, pg + 1,
                                   p_init=q if use_exact_guess else None, theta=theta,
                                   p_prev=q if theta != 1.0 else None)
    return vhat, vbar, p, vhat0, u, q


@pytest.mark.parametrize("pg", [0, 1])
def test_steady_linear_flow_inviscid_from_zero_pressure(pg):
    vhat, vbar, p, vhat0, u, q = _run_linear(pg, 0.0, False)
    assert np.abs(vhat - vhat0).max() <= 1e-11 * np.abs(vhat0).max()
    assert np.abs(vbar - u).max() <= 1e-11 * np.abs(u).max()
    assert np.abs(p - q).max() <= 1e-10 * np.abs(q).max()


@pytest.mark.parametrize("pg", [0, 1])
def test_steady_linear_flow_viscous_with_previous_pressure(pg):
    vhat, vbar, p, vhat0, u, q = _run_linear(pg, 0.05, True)
    assert np.abs(vhat - vhat0).max() <= 1e-11 * np.abs(vhat0).max()
    assert np.abs(p - q).max() <= 1e-10 * np.abs(q).max()


@pytest.mark.parametrize("periodic,pg", [(False, 0), (True, 1)])
def test_divergence_free_after_step(periodic, pg):
    n = 3 if periodic else 2
    X, T = kuhn_mesh(n)
    ops = SpaceTimeOperators(Mesh(X, T, periodic=periodic), 2, pg, 0.02)
    if periodic:
        from stdg_inputs import fourier_modes, fourier_velocity
        modes = fourier_modes(seed=3, n_modes=4, kmax=1)
        u = _nodal_field(ops, lambda x: fourier_velocity(x, modes))
    else:
        u = _nodal_field(ops, lambda x: beltrami_velocity(x))
    vhat, vbar, p, _ = picard_step(ops, initial_state(ops, u), u, u, 0.01, pg + 1)
    div = divergence(ops, vhat)
    scale = np.abs(divergence(ops, initial_state(ops, u))).max() + 1e-30
    div[0] = 0.0                      # the anchor element absorbs the compatibility defect
    assert np.abs(div).max() <= 1e-10 * max(scale, np.abs(vhat).max() * 0.1)


@pytest.mark.parametrize("theta", [0.5, 0.75])
@pytest.mark.parametrize("nu,exact_guess", [(0.0, False), (0.05, True)])
def test_theta_method_keeps_the_steady_linear_flow(theta, nu, exact_guess):
    vhat, vbar, p, vhat0, u, q = _run_linear(0, nu, exact_guess, theta=theta)
    assert np.abs(vhat - vhat0).max() <= 1e-11 * np.abs(vhat0).max()
    assert np.abs(vbar - u).max() <= 1e-11 * np.abs(u).max()
    assert np.abs(p - q).max() <= 1e-10 * np.abs(q).max()


def _theta_case():
    X, T = kuhn_mesh(2)
    ops = SpaceTimeOperators(Mesh(X, T), 1, 0, 0.02)
    u = _nodal_field(ops, lambda x: beltrami_velocity(x))
    rng = np.random.default_rng(11)
    p_prev = rng.standard_normal((ops.mesh.E, ops.Nst))
    p_prev -= p_prev.ravel()[anchor_indices(ops)[0]]
    return ops, u, p_prev


def test_theta_method_divergence_free():
    ops, u, p_prev = _theta_case()
    vhat, _, _, _ = picard_step(ops, initial_state(ops, u), u, u, 0.01, 2, theta=0.5, p_prev=p_prev)
    div = divergence(ops, vhat)
    div[0] = 0.0
    assert np.abs(div).max() <= 1e-10 * np.abs(vhat).max()


@pytest.mark.parametrize("guess", ["zero", "previous"])
def test_theta_method_is_the_plain_step_in_the_weighted_pressure(guess):
    ops, u, p_prev = _theta_case()
    theta = 0.6
    p0 = None if guess == "zero" else p_prev
    vh_t, vb_t, p_t, _ = picard_step(ops, initial_state(ops, u), u, u, 0.01, 2, p_init=p0,
                                     theta=theta, p_prev=p_prev)
    pi0 = (1.0 - theta) * p_prev + (0.0 if p0 is None else theta * p0)
    vh_1, vb_1, pi, _ = picard_step(ops, initial_state(ops, u), u, u, 0.01, 2, p_init=pi0)
    assert np.abs(vh_t - vh_1).max() <= 1e-12 * np.abs(vh_1).max()
    assert np.abs(vb_t - vb_1).max() <= 1e-12 * np.abs(vb_1).max()
    assert np.abs(theta * p_t + (1.0 - theta) * p_prev - pi).max() <= 1e-11 * np.abs(pi).max()


def test_viscous_system_spd_for_piecewise_constant_time():
    X, T = kuhn_mesh(2, jitter=0.1, seed=4)
    ops = SpaceTimeOperators(Mesh(X, T), 2, 0, 0.05)
    Av = viscous_matrix(ops, 0.3).toarray()
    assert np.abs(Av - Av.T).max() <= 1e-13 * np.abs(Av).max()
    assert np.linalg.eigvalsh(0.5 * (Av + Av.T)).min() > 0


def test_convection_of_continuous_polynomial_is_greens_formula():
    X, T = kuhn_mesh(2)
    dt = 0.1
    ops = SpaceTimeOperators(Mesh(X, T), 2, 1, dt)
    B = np.array([[0.4, -0.3, 0.2], [0.1, 0.5, -0.2], [0.3, 0.1, -0.4]])
    c0 = np.array([0.2, -0.1, 0.3])
    fn = lambda x: x @ B.T + c0
    u = _nodal_field(ops, fn)
    mesh = ops.mesh
    bc = {j: goback(ops, u, j) for j in range(mesh.F) if mesh.right[j] < 0}
    ups = convection(ops, u, bc)
    w = ops.tb.weights.astype(float)
    div_uu = lambda x: fn(x) * np.trace(B) + (x @ B.T + c0) @ B.T     # div(u u^T) = u tr B + B u
    for i in range(0, mesh.E, 5):
        v = mesh.tet_vertices(i)
        xq, wq = simplex_rule(v, 3)
        ph, _ = nodal_phys(ops.phi, TetMap(v), xq)
        f = div_uu(np.asarray(xq, float))
        for c in range(3):
            integ = (wq[:, None] * ph * f[:, c][:, None]).sum(0).astype(float)
            expect = dt * np.concatenate([wa * integ for wa in w])
            assert np.abs(ups[i, c] - expect).max() <= 1e-12 * np.abs(expect).max()


def test_convection_of_piecewise_constant_states_is_the_rusanov_face_sum():
    X, T = kuhn_mesh(3)
    dt = 0.1
    mesh = Mesh(X, T, periodic=True)
    ops = SpaceTimeOperators(mesh, 2, 0, dt)
    rng = np.random.default_rng(5)
    states = rng.standard_normal((mesh.E, 3))
    vbar = np.repeat(states[:, :, None], ops.Nst, axis=2)
    ups = convection(ops, vbar, {})
    for i in range(0, mesh.E, 13):
        v = mesh.tet_vertices(i)
        tm = TetMap(v)
        expect = np.zeros((3, ops.N))
        for f in range(4):
            P = v[[k for k in range(4) if k != f]]
            n = np.cross(P[1] - P[0], P[2] - P[0]); n /= np.linalg.norm(n)
            if n @ (P[0] - v.mean(0)) < 0:
                n = -n
            k, _ = mesh.neighbour(i, f)
            vm, vp = states[i], states[k]
            smax = 2 * max(np.linalg.norm(vm), np.linalg.norm(vp))
            jump = 0.5 * (vp * (vp @ n) - vm * (vm @ n)) - 0.5 * smax * (vp - vm)
            fq, fw = triangle_rule_3d(P, 2)
            ph, _ = nodal_phys(ops.phi, tm, fq)
            integ = (fw[:, None] * ph).sum(0).astype(float)
            expect += np.outer(jump, integ)
        assert np.abs(ups[i] - dt * expect).max() <= 1e-12 * np.abs(dt * expect).max()
