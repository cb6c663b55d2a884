"""Pin of the oracle's non-action observables through restricted double
brackets (Sec. 2.3, eqs. (l9)-(l10)) against the exactly solvable 2D U(1)
model on an 8x8 torus: a full oracle LLR run, restricted measurements at its
converged a_k, and the reconstruction of <cos theta_P>(beta) and of the
adjoint plaquette <cos 2 theta_P>(beta) must reproduce the character
expansion,
    <cos k theta_P> = sum_n I_n^{V-1} (I_{n-k} + I_{n+k}) / 2 / sum_n I_n^V,
within 3e-3 (the Robbins-Monro noise of a_k and the O(dE^2) error of the
double brackets at dE = 6; the observables differ by much more)."""
import numpy as np
from scipy import special

import oracle


def _exact(beta, V, k):
    n = np.arange(-40, 41)
    I = special.ive(n, beta)
    Ik = 0.5 * (special.ive(n - k, beta) + special.ive(n + k, beta))
    return np.sum(I ** (V - 1) * Ik) / np.sum(I ** V)


def test_double_brackets_reproduce_exact_2d_observables():
    d, L = 2, 8
    V = L * L
    dE, nk = 6.0, 8
    E_low = 6.0 + dE * np.arange(nk)
    r = oracle.llr_run(d, L, E_low, dE, 1.0, n_th=20, n_a=200, n_rm=60, seed=77)
    assert np.array_equal(r["conf"], np.arange(nk))
    th, E, a = r["theta"], r["E"].copy(), r["a"]
    Es, Bs = [], []
    for m in range(800):
        E, _ = oracle.sweeps(d, L, th, a, E_low, E_low + dE, np.arange(nk), E, 2, 100000 + 2 * m, seed=77)
        Es.append([oracle.energy(d, L, th[k]) for k in range(nk)])
        Bs.append([oracle.adjoint(d, L, th[k]) for k in range(nk)])
    Es, Bs = np.array(Es), np.array(Bs)
    # the measured samples stay inside their intervals
    assert np.all((Es >= E_low[None, :] - 1e-9) & (Es <= E_low[None, :] + dE + 1e-9))
    cen = E_low + 0.5 * dE
    for beta in (0.9, 1.0, 1.1):
        u = oracle.obs_reconstruct(cen, a, dE, Es, Es, [beta])[0] / V
        b = oracle.obs_reconstruct(cen, a, dE, Es, Bs, [beta])[0] / V
        assert abs(u - _exact(beta, V, 1)) < 3e-3, (beta, u)
        assert abs(b - _exact(beta, V, 2)) < 3e-3, (beta, b)


def test_double_brackets_reduce_to_midpoint_sums_for_the_energy():
    """With B = E and samples at the interval centres only, eqs. (l9)-(l10)
    are the midpoint sums of eqs. (l19)-(l20)."""
    rng = np.random.default_rng(5)
    n, s = 20, 3.0
    c = 100.0 + s * np.arange(n)
    a = 0.8 + 0.02 * np.arange(n) + rng.normal(0, 0.01, n)
    E = np.tile(c, (3, 1))
    for beta in (0.8, 1.0, 1.3):
        got = oracle.obs_reconstruct(c, a, s, E, E, [beta])[0]
        _, u, _ = oracle.reconstruct(c, a, s, 1.0, [beta])
        assert abs(got - u[0]) < 1e-9 * abs(u[0])
