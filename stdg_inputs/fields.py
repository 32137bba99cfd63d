"""Closed-form and seeded velocity fields sampled at given points.

* The Arnold-Beltrami-Childress field of eq. CT_1 (Sec. 3.2) with A=B=C=1,
  an exact Navier-Stokes solution: velocity decays like exp(-nu t), pressure
  like exp(-2 nu t).
* A seeded sum of divergence-free Fourier modes on the unit-periodic cube:
  v(x) = sum_m |k_m|^-2 e_m cos(2 pi k_m . x + phi_m), e_m a unit vector
  orthogonal to k_m, drawn with numpy.random.default_rng(seed) in the order
  k, then e, then phi.
"""

import numpy as np


def beltrami_velocity(x, t=0.0, nu=0.0):
    """(..., 3) ABC velocity of eq. CT_1 at points x (..., 3), time t."""
    x = np.asarray(x, dtype=np.float64)
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    d = np.exp(-nu * t)
    u = (np.sin(Z) + np.cos(Y)) * d
    v = (np.sin(X) + np.cos(Z)) * d
    w = (np.sin(Y) + np.cos(X)) * d
    return np.stack([u, v, w], axis=-1)


def beltrami_pressure(x, t=0.0, nu=0.0, c=0.0):
    """ABC pressure of eq. CT_1 (up to the additive constant c)."""
    x = np.asarray(x, dtype=np.float64)
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    return -(np.cos(X) * np.sin(Y) + np.sin(X) * np.cos(Z)
             + np.sin(Z) * np.cos(Y)) * np.exp(-2.0 * nu * t) + c


def fourier_modes(seed=1601, n_modes=16, kmax=4):
    """Seeded wave vectors k (m,3), unit amplitudes e (m,3) with e.k = 0, phases."""
    rng = np.random.default_rng(seed)
    ks = []
    while len(ks) < n_modes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            ks.append(k)
    k = np.asarray(ks, dtype=np.float64)
    e = np.empty_like(k)
    for m in range(n_modes):
        r = rng.standard_normal(3)
        r -= k[m] * (r @ k[m]) / (k[m] @ k[m])
        e[m] = r / np.linalg.norm(r)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    return k, e, phi


def fourier_velocity(x, modes, scale=1.0):
    """(..., 3) velocity of the Fourier field at points x; multiplied by scale."""
    k, e, phi = modes
    x = np.asarray(x, dtype=np.float64)
    arg = 2.0 * np.pi * np.tensordot(x, k.T, axes=1) + phi    # (..., m)
    amp = 1.0 / np.sum(k * k, axis=1)                          # |k|^-2
    return scale * np.tensordot(np.cos(arg) * amp, e, axes=1)
