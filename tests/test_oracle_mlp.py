"""Pins of the oracle MLP used for the learned Krylov initial guess.

* SiLU: silu(0) = 0, silu'(0) = 1/2, silu(z) - silu(-z) = z, silu' against
  central differences.
* Gradient of the mean-squared loss against central finite differences of
  the loss itself (every parameter of a small network).
* Closed forms with zero weights: Y = b3, dL/db3 = 2 mean_rows(b3 - T)/n_out,
  dL/dW3[k, j] = silu(b2_k) dL/db3_j (catches a transposed operand).
* Adam with a constant gradient g: the bias-corrected moments are g and g^2
  exactly, so every step moves each parameter by lr g / (|g| + eps).
* Feature gather: the neighbour slots hold the values of the element sharing
  the face opposite each local vertex, found by brute force over all
  elements; flags are 0 exactly on boundary faces; scales are RMS values.
* Residual-norm objective: equals 1 when the network outputs zero (the guess
  is the plain extrapolation), 0 when it outputs the exact correction, and
  its gradient matches central finite differences.
"""

import numpy as np

from stdg_inputs import kuhn_mesh
from oracle import mlp


def _net(seed, n_in=7, hidden=5, n_out=3, scale=0.7):
    rng = np.random.default_rng(seed)
    parts = [scale * rng.standard_normal(s) for s in mlp.shapes(n_in, hidden, n_out)]
    return mlp.flatten(parts)


def test_silu_identities():
    assert mlp.silu(0.0) == 0.0
    assert mlp.silu_prime(0.0) == 0.5
    z = np.linspace(-6, 6, 25)
    assert np.allclose(mlp.silu(z) - mlp.silu(-z), z, rtol=0, atol=1e-14)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.silu_prime(z)).max() < 1e-9


def test_gradient_matches_finite_differences():
    n_in, hidden, n_out, n = 7, 5, 3, 9
    rng = np.random.default_rng(3)
    F = rng.standard_normal((n, n_in))
    T = rng.standard_normal((n, n_out))
    theta = _net(4, n_in, hidden, n_out)
    loss, g = mlp.loss_and_grad(theta, F, T, hidden, n_out)
    h = 1e-6
    fd = np.empty_like(theta)
    for k in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd[k] = (mlp.loss_and_grad(tp, F, T, hidden, n_out)[0]
                 - mlp.loss_and_grad(tm, F, T, hidden, n_out)[0]) / (2 * h)
    assert np.abs(fd - g).max() <= 1e-7 * max(1.0, np.abs(g).max())
    assert loss > 0


def test_zero_weight_closed_forms():
    n_in, hidden, n_out, n = 6, 4, 3, 5
    rng = np.random.default_rng(8)
    b2 = rng.standard_normal(hidden)
    b3 = rng.standard_normal(n_out)
    parts = [np.zeros((n_in, hidden)), rng.standard_normal(hidden), np.zeros((hidden, hidden)),
             b2, np.zeros((hidden, n_out)), b3]
    theta = mlp.flatten(parts)
    F = rng.standard_normal((n, n_in))
    T = rng.standard_normal((n, n_out))
    Y, _ = mlp.forward(theta, F, hidden, n_out)
    assert np.array_equal(Y, np.tile(b3, (n, 1)))
    loss, g = mlp.loss_and_grad(theta, F, T, hidden, n_out)
    gW1, gb1, gW2, gb2, gW3, gb3 = mlp.unflatten(g, n_in, hidden, n_out)
    expect_b3 = 2.0 * (b3[None, :] - T).sum(axis=0) / (n * n_out)
    assert np.allclose(gb3, expect_b3, rtol=1e-14, atol=1e-15)
    s2 = b2 / (1.0 + np.exp(-b2))
    assert np.allclose(gW3, np.outer(s2, expect_b3), rtol=1e-13, atol=1e-15)
    assert np.abs(loss - np.mean((b3[None, :] - T) ** 2)) <= 1e-15 * loss
    # nothing flows back through zero W3
    assert not gW1.any() and not gb1.any() and not gW2.any() and not gb2.any()


def test_adam_constant_gradient_closed_form():
    rng = np.random.default_rng(1)
    theta = rng.standard_normal(11)
    g = rng.standard_normal(11)
    m = np.zeros(11)
    v = np.zeros(11)
    lr, eps = 1e-2, 1e-8
    t0 = theta.copy()
    for t in range(1, 4):
        theta, m, v = mlp.adam_step(theta, g, m, v, t, lr=lr, eps=eps)
        expect = t0 - t * lr * g / (np.abs(g) + eps)
        assert np.abs(theta - expect).max() <= 1e-13


def _brute_neighbours(T):
    E = T.shape[0]
    keys = {}
    for e in range(E):
        for f in range(4):
            keys.setdefault(frozenset(np.delete(T[e], f).tolist()), []).append(e)
    nbr = -np.ones((E, 4), dtype=np.int64)
    for e in range(E):
        for f in range(4):
            other = [k for k in keys[frozenset(np.delete(T[e], f).tolist())] if k != e]
            assert len(other) <= 1
            if other:
                nbr[e, f] = other[0]
    return nbr


def test_feature_gather_against_brute_force_adjacency():
    X, T = kuhn_mesh(2)
    E, nst = T.shape[0], 4
    nbr = _brute_neighbours(T)
    rng = np.random.default_rng(5)
    P = rng.standard_normal((E, nst))
    Pm = P - 0.01 * rng.standard_normal((E, nst))
    B = rng.standard_normal((E, nst))
    F = mlp.features(P, Pm, B, nbr)
    assert F.shape == (E, mlp.n_inputs(nst))
    sP = np.sqrt(np.mean(P ** 2))
    sD = np.sqrt(np.mean((P - Pm) ** 2))
    sB = np.sqrt(np.mean(B ** 2))
    for e in range(E):
        slots = [e] + list(nbr[e])
        for s, k in enumerate(slots):
            pv = F[e, s * nst:(s + 1) * nst]
            dv = F[e, (5 + s) * nst:(6 + s) * nst]
            if k < 0:
                assert not pv.any() and not dv.any()
            else:
                assert np.allclose(pv, P[k] / sP, rtol=1e-15, atol=0)
                assert np.allclose(dv, (P[k] - Pm[k]) / sD, rtol=1e-12, atol=0)
        assert np.allclose(F[e, 10 * nst:11 * nst], B[e] / sB, rtol=1e-15, atol=0)
        assert np.array_equal(F[e, 11 * nst:], (nbr[e] >= 0).astype(float))
    # a Dirichlet cube has boundary faces, a periodic one would have none
    assert (nbr < 0).any()


def test_zero_network_guess_is_linear_extrapolation():
    X, T = kuhn_mesh(2)
    E, nst, hidden = T.shape[0], 4, 6
    nbr = _brute_neighbours(T)
    rng = np.random.default_rng(6)
    P, Pm, B = (rng.standard_normal((E, nst)) for _ in range(3))
    theta = np.zeros(sum(int(np.prod(s)) for s in mlp.shapes(mlp.n_inputs(nst), hidden, nst)))
    assert np.array_equal(mlp.guess(theta, P, Pm, B, nbr, hidden), 2.0 * P - Pm)
    # a sequence linear in the step index (Pm, P, 2P - Pm) needs no correction
    X2 = 2.0 * P - Pm
    assert np.abs(mlp.target(P, Pm, X2)).max() <= 1e-14 * np.abs(X2).max()


def test_adam_reduces_loss_on_a_linear_target():
    """Behaviour, not a pin: a few hundred full-batch Adam steps fit a linear map."""
    n_in, hidden, n_out, n = 8, 16, 2, 64
    rng = np.random.default_rng(2)
    F = rng.standard_normal((n, n_in))
    A = rng.standard_normal((n_in, n_out)) * 0.3
    T = F @ A
    theta = _net(9, n_in, hidden, n_out, scale=0.3)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0, _ = mlp.loss_and_grad(theta, F, T, hidden, n_out)
    for t in range(1, 301):
        _, g = mlp.loss_and_grad(theta, F, T, hidden, n_out)
        theta, m, v = mlp.adam_step(theta, g, m, v, t, lr=1e-2)
    l1, _ = mlp.loss_and_grad(theta, F, T, hidden, n_out)
    assert l1 < 0.05 * l0


def test_residual_loss_closed_forms_and_gradient():
    rng = np.random.default_rng(11)
    E, nst, hidden = 6, 3, 5
    n_in = 8
    S = rng.standard_normal((E * nst, E * nst))
    P = rng.standard_normal((E, nst))
    Pm = P - 0.1 * rng.standard_normal((E, nst))
    X = 2 * P - Pm + 0.05 * rng.standard_normal((E, nst))
    F = rng.standard_normal((E, n_in))
    sD = np.sqrt(np.mean((P - Pm) ** 2))
    zero = np.zeros(sum(int(np.prod(s)) for s in mlp.shapes(n_in, hidden, nst)))
    loss0, _ = mlp.residual_loss_and_grad(zero, F, P, Pm, X, S, hidden)
    assert abs(loss0 - 1.0) <= 1e-14
    # a network whose bias alone is the exact correction (one element-independent
    # correction: choose X so that it is)
    c = 0.03 * rng.standard_normal(nst)
    X2 = 2 * P - Pm + c[None, :]
    parts = mlp.unflatten(zero.copy(), n_in, hidden, nst)
    parts[5] = c / sD
    loss1, _ = mlp.residual_loss_and_grad(mlp.flatten(parts), F, P, Pm, X2, S, hidden)
    assert loss1 <= 1e-26
    theta = _net(12, n_in, hidden, nst, scale=0.3)
    loss, g = mlp.residual_loss_and_grad(theta, F, P, Pm, X, S, hidden)
    h = 1e-6
    fd = np.empty_like(theta)
    for k in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd[k] = (mlp.residual_loss_and_grad(tp, F, P, Pm, X, S, hidden)[0]
                 - mlp.residual_loss_and_grad(tm, F, P, Pm, X, S, hidden)[0]) / (2 * h)
    assert np.abs(fd - g).max() <= 1e-6 * max(1.0, np.abs(g).max())
