"""Pins of the oracle's multicanonical sampling (Sec. 2.6): class heatbath
proposals at coupling b accepted with min(1, W(E')/W(E) e^{-b dE}) for the
weight W = 1/rho~, and the reweighting of eq. (4.7).  Checked against the
exactly solvable 2D U(1) model:
  * W ~ e^{beta E} (constant a_k = beta) is the canonical ensemble, whatever
    the proposal coupling: the plaquette must be the exact
    sum I_n^{V-1} I_n' / sum I_n^V, and with b = beta every class is accepted
    and the chain is the canonical heatbath itself;
  * with W = 1/rho~ built from the exact density of states of the 2D L=2
    torus (sampled exactly), the visited energies follow rho(E) W(E) bin by
    bin, inside the weight's range (flat up to rho~'s piecewise error) and in
    its continuation outside;
  * reweighting canonical samples to a nearby beta reproduces the exact
    plaquette there."""
import numpy as np
import pytest
from scipy import special

import oracle


def _exact_2d(beta, V):
    n = np.arange(-40, 41)
    I = special.ive(n, beta)
    Ip = 0.5 * (special.ive(n - 1, beta) + special.ive(n + 1, beta))
    return np.sum(I ** (V - 1) * Ip) / np.sum(I ** V)


def _canonical_weight(beta, c0, s, n):
    """a_k = beta on n intervals: ln W = beta (E - c_0) everywhere."""
    return c0 + s * np.arange(n), np.full(n, beta)


def test_equal_coupling_is_the_canonical_heatbath():
    d, L, nch = 4, 4, 3
    beta = 1.0
    c, a = _canonical_weight(beta, 0.0, 50.0, 40)
    oracle.set_muca(c, a, 50.0)
    th = oracle.hot_start(d, L, nch, 3)
    E = np.array([oracle.energy(d, L, th[i]) for i in range(nch)])
    t1, t2 = th.copy(), th.copy()
    big = [1e9] * nch
    E1, b1 = oracle.sweeps(d, L, t1, [beta] * nch, [-1e9] * nch, big, [0, 1, 2], E, 4, 0,
                           mode=oracle.MODE_MUCA, seed=9)
    E2, b2 = oracle.sweeps(d, L, t2, [beta] * nch, [-1e9] * nch, big, [0, 1, 2], E, 4, 0,
                           mode=oracle.MODE_FREE, seed=9)
    assert np.all((b1 & 0xff) == 0xff)
    assert np.array_equal(t1, t2) and np.array_equal(E1, E2)


def _muca_chain_2d(beta, b, nch=8, n_meas=300, gap=4, seed=5):
    d, L = 2, 8
    V = L * L
    c, a = _canonical_weight(beta, -64.0, 4.0, 33)
    oracle.set_muca(c, a, 4.0)
    th = oracle.hot_start(d, L, nch, 7)
    E = np.array([oracle.energy(d, L, th[i]) for i in range(nch)])
    big = [1e9] * nch
    E, bits = oracle.sweeps(d, L, th, [b] * nch, [-1e9] * nch, big, list(range(nch)), E, 100, 0,
                            mode=oracle.MODE_MUCA, seed=seed)
    acc, prop, samples = 0, 0, []
    for k in range(n_meas):
        E, bits = oracle.sweeps(d, L, th, [b] * nch, [-1e9] * nch, big, list(range(nch)), E, gap,
                                1000 + gap * k, mode=oracle.MODE_MUCA, seed=seed)
        acc += sum(bin(int(x) & 0xf).count("1") for x in bits.ravel())
        prop += 4 * bits.size
        samples.append(E.copy())
    return np.array(samples), acc / prop, V


def test_canonical_weight_with_other_proposal_coupling():
    beta = 1.0
    s, acc, V = _muca_chain_2d(beta, b=0.6)
    exact = _exact_2d(beta, V)
    err = (s / V).mean(axis=0).std() / np.sqrt(s.shape[1])
    assert acc < 0.95                                   # the correction is at work
    assert abs((s / V).mean() - exact) < 4 * err + 1e-3


def test_reweighting_to_nearby_couplings():
    beta = 1.0
    s, _, V = _muca_chain_2d(beta, b=beta)
    c, a = _canonical_weight(beta, -64.0, 4.0, 33)
    for bt in (0.9, 1.1):
        u, _ = oracle.muca_reweight(s, c, a, 4.0, V, [bt])
        # per-chain reweighted estimates for the error
        per = [oracle.muca_reweight(s[:, i], c, a, 4.0, V, [bt])[0][0] for i in range(s.shape[1])]
        err = np.std(per) / np.sqrt(len(per))
        assert abs(u[0] - _exact_2d(bt, V)) < 4 * err + 1e-3


def test_visits_follow_rho_times_w_with_the_exact_density():
    """2D L=2 (4 plaquettes): the plaquette angles of Haar-random links are
    uniform subject to sum_P theta_P = 0 (mod 2 pi), which is sampled exactly.
    With W = 1/rho~ built from that rho on [-2, 2.4] (and continued outside as
    in eq. (4.1)), the visited energies follow rho(E) W(E) on all of [-4, 4];
    the canonical weight e^{bE} of the proposal coupling would not."""
    rng = np.random.default_rng(1)
    t = rng.uniform(-np.pi, np.pi, (8000000, 3))
    Ex = np.cos(t).sum(1) + np.cos(-t.sum(1))
    lo, hi, s = -2.0, 2.4, 0.2
    n = int(round((hi - lo) / s))
    c = lo + s * (np.arange(n) + 0.5)
    # ln rho at fine resolution, smoothed by a polynomial, a = -d ln rho / dE
    fine = np.linspace(lo - 0.3, hi + 0.3, 95)
    h, edges = np.histogram(Ex, bins=fine)
    mid = 0.5 * (edges[1:] + edges[:-1])
    coef = np.polyfit(mid, np.log(h), 8)
    a = -np.polyval(np.polyder(coef), c)
    oracle.set_muca(c, a, s)
    d, L = 2, 2
    nch = 4
    th = np.zeros((nch, d, 4))
    E = np.array([oracle.energy(d, L, th[i]) for i in range(nch)])
    big = [1e9] * nch
    bprop = float(np.median(a))
    E, _ = oracle.sweeps(d, L, th, [bprop] * nch, [-1e9] * nch, big, list(range(nch)), E, 200, 0,
                         mode=oracle.MODE_MUCA, seed=3)
    vis = []
    for k in range(6000):
        E, _ = oracle.sweeps(d, L, th, [bprop] * nch, [-1e9] * nch, big, list(range(nch)), E, 3,
                             10 + 3 * k, mode=oracle.MODE_MUCA, seed=3)
        vis.append(E.copy())
    vis = np.ravel(vis)
    bins = np.linspace(-4.0, 4.0, 21)
    hv, _ = np.histogram(vis, bins=bins)
    ex = Ex[:2000000]
    lw = oracle.muca_lnw(ex)
    p, _ = np.histogram(ex, bins=bins, weights=np.exp(lw - lw.max()))
    p /= p.sum()
    m = hv.sum()
    chi2 = np.sum((hv - m * p) ** 2 / (m * p)) / bins.size
    q, _ = np.histogram(ex, bins=bins, weights=np.exp(bprop * ex))
    q /= q.sum()
    chi2q = np.sum((hv - m * q) ** 2 / (m * q)) / bins.size
    # samples 3 sweeps apart are mildly correlated: allow an inflated chi2
    assert chi2 < 4.0
    assert chi2q > 10 * chi2
