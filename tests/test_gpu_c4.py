"""The high-order configuration on the device: unit cube split into n^3
hexahedra x 6 tetrahedra, p = 4, p_gamma = 4 (175 space-time DoF per
element), Dirichlet velocity from the exact ABC (Beltrami) flow of eq. CT_1
with A = B = C = 1, 5 time steps of the Picard scheme of Sec. 2.6 (p_gamma + 1
Picard iterations).  The pressure solves are the time-decoupled CG with FP32
inner solves on the element-per-lane MFMA operator inside FP64 refinement
(rtol 1e-10); the viscous solves are block-Jacobi preconditioned BiCGStab.
The time step follows the explicit-DG CFL restriction of the convective term
(Courant number 0.3 / (2p + 1) on the flow speed, as in Sec. 3.2): the
dt = 1e-2 of the small C1 configuration is unstable on these meshes (errors
grow ~15x per step on the 8^3 mesh at p = 3).

* nu = 0 (a steady Euler flow): the L2 errors against the exact solution fall
  from n = 8 to n = 16 at no less than p - 1/2 (measured: 5.0 and 5.1).
* nu = 1e-2 on the 24,576-element mesh (the configuration), Dirichlet data
  decaying with the exact flow: errors and time per step are reported, the
  FP32-refined and FP64 pressure solves give the same errors, and the errors
  stay within 4x of the measured 2.7e-5 (pressure) and 7.8e-7 (velocity).
"""

import math
import time

import numpy as np
import pytest

from stdg_inputs import beltrami_velocity, kuhn_mesh, node_coordinates, time_nodes
from test_gpu_convergence import end_weights, l2_errors, l2_projection

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1601_07384_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dirichlet_nodal(X, T, p, G, t0, dt, nu):
    """(3, E, G, N) exact velocity at the element nodes and the slab's time nodes."""
    xn = node_coordinates(X, T, p)
    return np.stack([np.transpose(beltrami_velocity(xn, t0 + dt * ta, nu), (2, 0, 1)) for ta in time_nodes(G)],
                    axis=2)


def run_beltrami(n, p=4, pg=4, nu=1e-2, steps=5, precision=P.STDG_FP32, cfl=0.3):
    X, T = kuhn_mesh(n)
    vmax = (1.0 + math.sin(1.0)) * math.sqrt(3.0)      # largest |v| of the field on the unit cube
    dt = cfl / (n * (2 * p + 1) * vmax)
    t0 = time.perf_counter()
    m = P.Mesh(X, T, p, pg, dt=dt, nu=nu, periodic=False)
    build_s = time.perf_counter() - t0
    E, N, G = m.E, m.N, m.G
    perm = m.permutation()
    v0 = np.transpose(l2_projection(X, T, p, beltrami_velocity), (2, 0, 1))[:, perm, :]      # (3, E, N)
    vbar = torch.tensor(np.ascontiguousarray(np.repeat(v0[:, :, None, :], G, axis=2)).ravel(),
                        dtype=torch.float64, device=DEV)
    vhat = torch.empty(3 * m.n_face * m.Nst, dtype=torch.float64, device=DEV)
    m.dual_from_main(vbar, vhat)
    pr = torch.zeros(E * m.Nst, dtype=torch.float64, device=DEV)
    opts = P.step_opts(pressure_guess=P.STDG_GUESS_ZERO,
                       pressure={"method": P.STDG_CG_TIME, "precision": precision, "rtol": 1e-10,
                                 "inner_rtol": 1e-5, "max_iter": 400000},
                       viscous={"method": P.STDG_BICGSTAB, "restart": 30, "rtol": 1e-12, "check_every": 1})
    step_s, iters = [], []
    for k in range(steps):
        g = dirichlet_nodal(X, T, p, G, k * dt, dt, nu)[:, perm]
        gd = torch.tensor(np.ascontiguousarray(g).ravel(), dtype=torch.float64, device=DEV)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = m.picard_step(vhat, vbar, pr, gd, opts=opts)
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - t0)
        iters.append((rep.pressure_iters, rep.viscous_iters))
        assert rep.status == P.STDG_OK
        assert rep.max_pressure_residual <= 1e-9
    lw = end_weights(G)
    ph = pr.cpu().numpy().reshape(E, G, N).transpose(0, 2, 1)
    vh = np.transpose(vbar.cpu().numpy().reshape(3, E, G, N), (1, 0, 3, 2))
    pres = np.empty((E, N))
    pres[perm] = ph @ lw
    vel = np.empty((E, 3, N))
    vel[perm] = vh @ lw
    ep, ev = l2_errors(X, T, p, pres, vel, steps * dt, nu)
    r = {"n": n, "E": E, "classes": m.n_classes, "layout": m.inner_layout, "dt": dt, "err_p": ep, "err_v": ev,
         "step_s": step_s, "iters": iters, "build_s": build_s}
    print(f"n={n} E={E} nu={nu} dt={dt:.3e} classes={m.n_classes} inner layout={m.inner_layout} "
          f"precision={precision}: err_p {ep:.4e} err_v {ev:.4e}; step time "
          + ", ".join(f"{s * 1e3:.0f}" for s in step_s) + " ms; (pressure, viscous) iterations " + str(iters),
          flush=True)
    return r


def test_beltrami_p4_dirichlet_inviscid_convergence():
    rows = [run_beltrami(n, nu=0.0) for n in (8, 16)]
    assert rows[1]["layout"] == P.STDG_LAYOUT_RUN
    op = math.log(rows[0]["err_p"] / rows[1]["err_p"]) / math.log(2.0)
    ov = math.log(rows[0]["err_v"] / rows[1]["err_v"]) / math.log(2.0)
    print(f"nu = 0, observed order 8^3 -> 16^3: pressure {op:.2f}, velocity {ov:.2f}", flush=True)
    assert op >= 3.5 and ov >= 3.5


def test_beltrami_p4_dirichlet_c4():
    r32 = run_beltrami(16, nu=1e-2)
    r64 = run_beltrami(16, nu=1e-2, precision=P.STDG_FP64)
    assert abs(r32["err_p"] - r64["err_p"]) <= 1e-6 * r64["err_p"]
    assert abs(r32["err_v"] - r64["err_v"]) <= 1e-6 * r64["err_v"]
    assert r32["err_p"] <= 1e-4 and r32["err_v"] <= 3e-6
    print(f"time per step: FP32 refinement {np.mean(r32['step_s']):.2f} s, FP64 {np.mean(r64['step_s']):.2f} s",
          flush=True)
