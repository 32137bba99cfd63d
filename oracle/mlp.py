"""Oracle multilayer perceptron for the learned Krylov initial guess (test infrastructure only).

The pressure-correction solve at the first Picard iteration of a time step
(Sec. 2.6, step 5 with the zero pressure guess of step 0) yields the first
Picard pressure p^{n+1,1}.  A plain Krylov solver starts it from zero or from
the previous step's value P = p^{n,1}.  With Pm = p^{n-1,1}, the learned guess
corrects the linear extrapolation of that sequence:

    x0 = 2 P - Pm + s_D * MLP(features),

with the network acting element by element on
    * P of the element and of its four face neighbours, divided by s_P,
    * P - Pm of the same five elements, divided by s_D,
    * the element's own right-hand side b, divided by s_B,
    * four neighbour-present flags,
where s_P, s_D, s_B are the root-mean-square values of P, P - Pm and b over
the whole mesh (1 when zero).  Slot order: the element itself,
then the neighbours across local faces 0..3 (local face f is the face
opposite local vertex f); a missing neighbour (Dirichlet boundary) gives
zeros and flag 0.  The training target is (x* - 2P + Pm) / s_D,
x* = p^{n+1,1};
the loss is the mean squared error over samples and outputs.

Network: three affine layers, SiLU after the first two,
    Z1 = F W1 + b1, H1 = silu(Z1), Z2 = H1 W2 + b2, H2 = silu(Z2),
    Y = H2 W3 + b3,
with W stored input-major (W[k, j] multiplies input k into output j) and the
parameters flattened in the order W1, b1, W2, b2, W3, b3.  Training uses Adam
(Kingma & Ba, with bias correction).  Everything is float64.
"""

import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_prime(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def rms(v):
    r = float(np.sqrt(np.mean(np.asarray(v, dtype=np.float64) ** 2)))
    return r if r > 0.0 else 1.0


def n_inputs(nst):
    return 11 * nst + 4


def shapes(n_in, hidden, n_out):
    return [(n_in, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden, n_out), (n_out,)]


def unflatten(theta, n_in, hidden, n_out):
    out, o = [], 0
    for s in shapes(n_in, hidden, n_out):
        k = int(np.prod(s))
        out.append(np.asarray(theta[o:o + k], dtype=np.float64).reshape(s))
        o += k
    assert o == len(theta)
    return out


def flatten(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def features(P, Pm, B, nbr, elements=None):
    """Feature rows (n, 11 Nst + 4) for the given elements.

    P, Pm, B: (E, Nst) the predicted quantity one and two steps back, and the
    right-hand side.
    nbr: (E, 4) neighbour across local face f, -1 if none.
    """
    P = np.asarray(P, dtype=np.float64)
    Pm = np.asarray(Pm, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    E, nst = P.shape
    if elements is None:
        elements = np.arange(E)
    sP, sD, sB = rms(P), rms(P - Pm), rms(B)
    D = P - Pm
    rows = []
    for i in elements:
        slots = [int(i)] + [int(nbr[i, f]) for f in range(4)]
        pv = [P[k] / sP if k >= 0 else np.zeros(nst) for k in slots]
        dv = [D[k] / sD if k >= 0 else np.zeros(nst) for k in slots]
        mask = [1.0 if k >= 0 else 0.0 for k in slots[1:]]
        rows.append(np.concatenate(pv + dv + [B[i] / sB, np.array(mask)]))
    return np.array(rows)


def target(P, Pm, X):
    """(x* - 2P + Pm) / s_D, shape (E, Nst)."""
    P = np.asarray(P, dtype=np.float64)
    return (np.asarray(X, dtype=np.float64) - 2.0 * P + Pm) / rms(P - Pm)


def forward(theta, F, hidden, n_out):
    """Returns (Y, cache) for feature rows F (n, n_in)."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta, F.shape[1], hidden, n_out)
    Z1 = F @ W1 + b1
    H1 = silu(Z1)
    Z2 = H1 @ W2 + b2
    H2 = silu(Z2)
    Y = H2 @ W3 + b3
    return Y, (F, Z1, H1, Z2, H2)


def loss_and_grad(theta, F, T, hidden, n_out):
    """Mean squared error over all entries of Y - T and its gradient (flat)."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta, F.shape[1], hidden, n_out)
    Y, (F, Z1, H1, Z2, H2) = forward(theta, F, hidden, n_out)
    R = Y - T
    loss = float(np.mean(R * R))
    dY = 2.0 * R / R.size
    gW3 = H2.T @ dY
    gb3 = dY.sum(axis=0)
    dZ2 = (dY @ W3.T) * silu_prime(Z2)
    gW2 = H1.T @ dZ2
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2.T) * silu_prime(Z1)
    gW1 = F.T @ dZ1
    gb1 = dZ1.sum(axis=0)
    return loss, flatten([gW1, gb1, gW2, gb2, gW3, gb3])


def adam_step(theta, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1).  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def guess(theta, P, Pm, B, nbr, hidden):
    """x0 = 2P - Pm + s_D * MLP(features), shape (E, Nst)."""
    F = features(P, Pm, B, nbr)
    Y, _ = forward(theta, F, hidden, P.shape[1])
    P = np.asarray(P, dtype=np.float64)
    return (2.0 * P - Pm) + rms(P - Pm) * Y


def residual_loss_and_grad(theta, F, P, Pm, X, S, hidden):
    """Residual-norm training objective of the learned guess.

    With the extrapolation x_e = 2P - Pm, the guess x0 = x_e + s_D MLP(F) and
    the operator S of the solve (a matrix acting on flattened (E, Nst)
    vectors):  L = |S (x0 - x*)|^2 / |S (x_e - x*)|^2, the initial residual of
    the solve relative to that of plain extrapolation.  Returns L and dL/dtheta
    (chain rule: dL/dY = s_D 2 S^T S (x0 - x*) / |S (x_e - x*)|^2, then the
    network's backward pass)."""
    P = np.asarray(P, dtype=np.float64)
    Pm = np.asarray(Pm, dtype=np.float64)
    E, nst = P.shape
    sD = rms(P - Pm)
    W1, b1, W2, b2, W3, b3 = unflatten(theta, F.shape[1], hidden, nst)
    Y, (F, Z1, H1, Z2, H2) = forward(theta, F, hidden, nst)
    ee = (2.0 * P - Pm - X).ravel()
    Re = S @ ee
    den = float(Re @ Re)
    e = ee + sD * Y.ravel()
    R = S @ e
    loss = float(R @ R) / den
    dY = (sD * 2.0 * (S.T @ R) / den).reshape(E, nst)
    gW3 = H2.T @ dY
    gb3 = dY.sum(axis=0)
    dZ2 = (dY @ W3.T) * silu_prime(Z2)
    gW2 = H1.T @ dZ2
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2.T) * silu_prime(Z1)
    gW1 = F.T @ dZ1
    gb1 = dZ1.sum(axis=0)
    return loss, flatten([gW1, gb1, gW2, gb2, gW3, gb3])
