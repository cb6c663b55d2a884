"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

This module holds no arithmetic of the method: it only draws link angles.
A "thermalised-like" state is a random gauge transformation of small
Gaussian fluctuations around the trivial field; the fluctuation width sets
the plaquette density (about exp(-2 sigma^2) for independent Gaussians),
so that states with u ~ 0.5-0.7, the range the intervals cover, can be
made without running any update.
"""
import numpy as np


def wrap(x):
    return (x + np.pi) % (2 * np.pi) - np.pi


def random_state(d, L, n_chains, seed, u_target=0.6, dtype=np.float64):
    """(n_chains, d, L^d) link angles in [-pi, pi) with plaquette density near u_target."""
    rng = np.random.default_rng(seed)
    V = L ** d
    sigma = np.sqrt(-np.log(u_target) / 2.0)
    th = rng.normal(0.0, sigma, size=(n_chains, d, V))
    lam = rng.uniform(-np.pi, np.pi, size=(n_chains, V))
    strides = [L ** m for m in range(d)]
    s = np.arange(V)
    for mu in range(d):
        x = (s // strides[mu]) % L
        up = s + np.where(x == L - 1, -(L - 1) * strides[mu], strides[mu])
        th[:, mu, :] += lam[:, s] - lam[:, up]
    th = wrap(th)
    if dtype == np.float32:
        th = th.astype(np.float32)
        th = np.where(th >= np.float32(np.pi), th - np.float32(2 * np.pi), th).astype(np.float32)
    return np.ascontiguousarray(th, dtype=dtype)


def random_gauge(d, L, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-np.pi, np.pi, size=L ** d)


def gauge_transform(theta, d, L, lam):
    """theta_mu(x) -> theta_mu(x) + lam(x) - lam(x + mu) (Sec. 3.1)."""
    V = L ** d
    s = np.arange(V)
    out = theta.copy()
    for mu in range(d):
        x = (s // L ** mu) % L
        up = s + np.where(x == L - 1, -(L - 1) * L ** mu, L ** mu)
        out[..., mu, :] = wrap(theta[..., mu, :] + lam[s] - lam[up])
    return out


def circ_dist(a, b):
    return np.abs(wrap(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)))
