"""GPU parity of the learned-guess model kernels against the oracle MLP.

The library's feature gather, forward pass (MFMA GEMMs with fused bias/SiLU),
loss gradient (split-K weight gradients) and Adam step are compared with
``oracle/mlp.py`` in FP64 (1e-12 relative for forward values, 1e-11 for
gradients); the FP32 model within 1e-5 / 1e-4.  Sizes are ragged against the
64x64 GEMM tiles.  The last test runs the learned guess inside Picard steps
and checks that the solution is unchanged and the first pressure solve needs
fewer iterations than with the previous-step guess.
"""

import numpy as np
import pytest

from stdg_inputs import kuhn_mesh, node_coordinates, fourier_modes, fourier_velocity
from oracle import mlp
from oracle.mesh import Mesh as OracleMesh

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_1601_07384_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64).ravel(), device=DEV)


def host(t, shape):
    torch.cuda.synchronize()
    return t.cpu().numpy().reshape(shape)


def small_mesh(n=3, p=1, pg=1, periodic=True):
    X, T = kuhn_mesh(n)
    return X, T, P.Mesh(X, T, p, pg, dt=1e-2, periodic=periodic)


def rand_theta(model, seed, scale=0.4):
    rng = np.random.default_rng(seed)
    parts = [scale * rng.standard_normal(s) for s in mlp.shapes(model.n_in, model.hidden, model.n_out)]
    return mlp.flatten(parts)


@pytest.mark.parametrize("precision,hidden,n", [(P.STDG_FP64, 40, 300), (P.STDG_FP64, 128, 77),
                                                (P.STDG_FP32, 40, 300)])
def test_forward_and_gradient_match_oracle(precision, hidden, n):
    print(f"mlp fwd/grad precision={precision} hidden={hidden} n={n}", flush=True)
    _, _, m = small_mesh()
    model = P.Model(m, hidden=hidden, precision=precision, batch=512)
    theta = rand_theta(model, 11)
    model.set_params(theta)
    rng = np.random.default_rng(12)
    F = rng.standard_normal((n, model.n_in))
    T = rng.standard_normal((n, model.n_out))
    Yd = torch.empty(n * model.n_out, dtype=torch.float64, device=DEV)
    model.forward(dev(F), Yd)
    Yo, _ = mlp.forward(theta, F, hidden, model.n_out)
    Yg = host(Yd, Yo.shape)
    tol_f, tol_g = (1e-12, 1e-11) if precision == P.STDG_FP64 else (1e-5, 1e-4)
    assert np.abs(Yg - Yo).max() <= tol_f * np.abs(Yo).max()
    loss = model.loss_grad(dev(F), dev(T))
    lo, go = mlp.loss_and_grad(theta, F, T, hidden, model.n_out)
    assert abs(loss - lo) <= tol_f * lo
    gg = model.grads()
    # every parameter block, each against its own scale
    o = 0
    for s in mlp.shapes(model.n_in, hidden, model.n_out):
        k = int(np.prod(s))
        assert np.abs(gg[o:o + k] - go[o:o + k]).max() <= tol_g * np.abs(go[o:o + k]).max(), s
        o += k


def test_adam_step_matches_oracle():
    _, _, m = small_mesh()
    model = P.Model(m, hidden=24, precision=P.STDG_FP64, batch=256, lr=3e-3)
    theta = rand_theta(model, 5)
    model.set_params(theta)
    rng = np.random.default_rng(6)
    F = rng.standard_normal((100, model.n_in))
    T = rng.standard_normal((100, model.n_out))
    mo = np.zeros_like(theta)
    vo = np.zeros_like(theta)
    th = theta.copy()
    for t in range(1, 4):
        model.loss_grad(dev(F), dev(T))
        model.adam_step()
        _, g = mlp.loss_and_grad(th, F, T, 24, model.n_out)
        th, mo, vo = mlp.adam_step(th, g, mo, vo, t, lr=3e-3)
        assert np.abs(model.params() - th).max() <= 1e-12 * np.abs(th).max()


@pytest.mark.parametrize("periodic", [True, False])
def test_features_and_guess_match_oracle(periodic):
    print(f"mlp features periodic={periodic}", flush=True)
    X, T, m = small_mesh(3, 2, 1, periodic)
    om = OracleMesh(X, T, periodic=periodic)
    nbr = np.array([[om.neighbour(t, f)[0] for f in range(4)] for t in range(om.E)])
    perm = m.permutation()
    rng = np.random.default_rng(7)
    Pn = rng.standard_normal((m.E, m.Nst))
    Pm = Pn - 0.05 * rng.standard_normal((m.E, m.Nst))
    B = rng.standard_normal((m.E, m.Nst))
    Fo = mlp.features(Pn, Pm, B, nbr)
    model = P.Model(m, hidden=33, precision=P.STDG_FP64, batch=100)
    Fd = torch.empty(m.E * model.n_in, dtype=torch.float64, device=DEV)
    model.features(dev(Pn[perm]), dev(Pm[perm]), dev(B[perm]), Fd)
    Fg = host(Fd, (m.E, model.n_in))
    assert np.abs(Fg - Fo[perm]).max() <= 1e-14 * np.abs(Fo).max()
    theta = rand_theta(model, 8, scale=0.3)
    model.set_params(theta)
    xd = torch.empty(m.E * m.Nst, dtype=torch.float64, device=DEV)
    model.predict(dev(Pn[perm]), dev(Pm[perm]), dev(B[perm]), xd)      # E > batch: chunked
    xo = mlp.guess(theta, Pn, Pm, B, nbr, 33)
    assert np.abs(host(xd, (m.E, m.Nst)) - xo[perm]).max() <= 1e-12 * np.abs(xo).max()


def test_training_reduces_loss():
    _, _, m = small_mesh(3, 1, 1)
    model = P.Model(m, hidden=64, precision=P.STDG_FP32, batch=128, lr=3e-3, loss=P.STDG_LOSS_MSE)
    rng = np.random.default_rng(9)
    S, n = 3, m.E * m.Nst
    Pn = rng.standard_normal((S, n))
    Pm = Pn - 0.1 * rng.standard_normal((S, n))
    B = rng.standard_normal((S, n))
    X = 2 * Pn - Pm + 0.5 * (Pn - Pm)        # a correction linear in the features
    rep = model.train(dev(Pn), dev(Pm), dev(B), dev(X), epochs=30)
    assert rep.samples == S * m.E and rep.epochs == 30
    assert rep.last_loss < 0.2 * rep.first_loss


@pytest.mark.parametrize("periodic", [True, False])
def test_residual_objective_matches_oracle(periodic):
    """|S(x0 - x*)|^2 / |S(x_e - x*)|^2 and its gradient (through S^T) in FP64
    against the oracle with the assembled operator, in the library's element
    order."""
    print(f"mlp residual objective periodic={periodic}", flush=True)
    from oracle.pressure import assemble_S
    from oracle.spacetime import SpaceTimeOperators
    X, T, m = small_mesh(3, 1, 1, periodic)
    om = OracleMesh(X, T, periodic=periodic)
    ops = SpaceTimeOperators(om, 1, 1, 1e-2)
    perm = m.permutation()
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(m.E)
    nbr = np.array([[om.neighbour(perm[i], f)[0] for f in range(4)] for i in range(m.E)])
    nbr = np.where(nbr >= 0, iperm[np.maximum(nbr, 0)], -1)
    S = assemble_S(ops).toarray()
    idx = (perm[:, None] * m.Nst + np.arange(m.Nst)).ravel()
    S = S[np.ix_(idx, idx)]
    rng = np.random.default_rng(17)
    Pn = rng.standard_normal((m.E, m.Nst))
    Pm = Pn - 0.1 * rng.standard_normal((m.E, m.Nst))
    B = rng.standard_normal((m.E, m.Nst))
    Xs = 2 * Pn - Pm + 0.05 * rng.standard_normal((m.E, m.Nst))
    model = P.Model(m, hidden=24, precision=P.STDG_FP64, batch=m.E)
    theta = rand_theta(model, 19, scale=0.3)
    model.set_params(theta)
    loss = model.residual_loss_grad(dev(Pn), dev(Pm), dev(B), dev(Xs))
    F = mlp.features(Pn, Pm, B, nbr)
    lo, go = mlp.residual_loss_and_grad(theta, F, Pn, Pm, Xs, S, 24)
    assert abs(loss - lo) <= 1e-11 * lo
    gg = model.grads()
    o = 0
    for shp in mlp.shapes(model.n_in, 24, model.n_out):
        k = int(np.prod(shp))
        assert np.abs(gg[o:o + k] - go[o:o + k]).max() <= 1e-10 * np.abs(go[o:o + k]).max(), shp
        o += k


def fourier_state(m, X, T, p):
    perm = m.permutation()
    modes = fourier_modes(seed=1601)
    xn = node_coordinates(X, T, p)
    v = fourier_velocity(xn, modes)
    v /= np.sqrt((v * v).sum(-1)).max()
    vb = np.tile(np.transpose(v, (2, 0, 1))[:, perm, None, :], (1, 1, m.G, 1))
    vbar = torch.tensor(np.ascontiguousarray(vb).ravel(), dtype=torch.float64, device=DEV)
    vhat = torch.empty(3 * m.n_face * m.Nst, dtype=torch.float64, device=DEV)
    m.dual_from_main(vbar, vhat)
    return vhat, vbar


def test_learned_guess_keeps_solution_and_saves_iterations():
    """8^3 x 6 periodic cube, p=2, p_gamma=1, Fourier flow, dt=1e-3: record 16
    steps, train on them, then start the first pressure solve of 6 further
    steps from the previous step's first Picard pressure, its linear
    extrapolation and the learned guess, each from the same state."""
    n_hex, p, pg, dt, nu = 8, 2, 1, 1e-3, 1e-3
    X, T = kuhn_mesh(n_hex)
    m = P.Mesh(X, T, p, pg, dt=dt, nu=nu, periodic=True)
    vhat, vbar = fourier_state(m, X, T, p)
    n = m.E * m.Nst
    p_cur = torch.zeros(n, dtype=torch.float64, device=DEV)
    hist = torch.zeros(2 * m.G * n, dtype=torch.float64, device=DEV)     # 2 steps x 2 Picard solves
    solve = {"method": P.STDG_CG_TIME, "precision": P.STDG_FP32, "rtol": 1e-10, "inner_rtol": 1e-5,
             "max_iter": 100000}
    visc = {"method": P.STDG_GMRES, "restart": 30, "rtol": 1e-10}
    n_rec, n_eval = 16, 6
    Xr = torch.zeros(n_rec * n, dtype=torch.float64, device=DEV)
    Br = torch.zeros(n_rec * n, dtype=torch.float64, device=DEV)
    for k in range(n_rec):
        opts = P.step_opts(pressure=solve, viscous=visc, krylov_guess=P.STDG_KRYLOV_PREVIOUS, hist=hist,
                           rec_b=Br[k * n:(k + 1) * n], rec_x=Xr[k * n:(k + 1) * n])
        m.picard_step(vhat, vbar, p_cur, None, opts=opts)
    torch.cuda.synchronize()
    assert torch.equal(hist[:n], Xr[(n_rec - 1) * n:]) and torch.equal(hist[n:2 * n], Xr[(n_rec - 2) * n:(n_rec - 1) * n])
    model = P.Model(m, hidden=128, precision=P.STDG_FP32, batch=m.E, lr=1e-3, seed=3)
    S = n_rec - 2
    rep = model.train(Xr[n:(n_rec - 1) * n], Xr[:S * n], Br[2 * n:], Xr[2 * n:], epochs=60)
    assert rep.last_loss < 1.0          # better than plain extrapolation on the training steps
    print(f"train loss {rep.first_loss:.3e} -> {rep.last_loss:.3e} in {rep.seconds:.1f}s", flush=True)
    its = {P.STDG_KRYLOV_ZERO: [], P.STDG_KRYLOV_PREVIOUS: [], P.STDG_KRYLOV_EXTRAPOLATE: [],
           P.STDG_KRYLOV_LEARNED: []}
    steps_its = {k: [] for k in its}
    for step in range(n_eval):
        state = [t.clone() for t in (vhat, vbar, p_cur, hist)]
        ref = None
        for kg in its:
            vh, vb, pc, hs = (t.clone() for t in state) if kg != P.STDG_KRYLOV_PREVIOUS else (vhat, vbar, p_cur, hist)
            r = m.picard_step(vh, vb, pc, None,
                              opts=P.step_opts(pressure=solve, viscous=visc, krylov_guess=kg, hist=hs,
                                               model=model if kg == P.STDG_KRYLOV_LEARNED else None))
            torch.cuda.synchronize()
            its[kg].append(r.first_pressure_iters)
            steps_its[kg].append(r.pressure_iters)
            print(f"eval step {step} guess {kg}: first solve {r.first_pressure_iters} it, r0 "
                  f"{r.first_initial_residual:.2e}; step {r.pressure_iters} it", flush=True)
            if ref is None:
                ref = (pc.clone(), vh.clone())
            else:
                assert float((pc - ref[0]).abs().max()) <= 1e-8 * float(ref[0].abs().max())
                assert float((vh - ref[1]).abs().max()) <= 1e-9 * float(ref[1].abs().max())
    print({k: sum(v) for k, v in its.items()}, {k: sum(v) for k, v in steps_its.items()}, flush=True)
    assert sum(its[P.STDG_KRYLOV_LEARNED]) < sum(its[P.STDG_KRYLOV_PREVIOUS])
    assert sum(its[P.STDG_KRYLOV_LEARNED]) < sum(its[P.STDG_KRYLOV_ZERO])
    # the network's own contribution: the learned start is the extrapolation
    # plus the fitted network term, so it must beat the extrapolation alone
    assert sum(its[P.STDG_KRYLOV_LEARNED]) < sum(its[P.STDG_KRYLOV_EXTRAPOLATE])
