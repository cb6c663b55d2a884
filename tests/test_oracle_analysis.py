"""Pins of the oracle's analysis of repeated runs: the probability density
P_beta(E) and its peaks (Sec. 3.4), the bootstrap over N_B runs (Sec. 2.4,
Sec. 3.2) and the finite-size-scaling fits (Sec. 3.4, Tabs. betac and
latentheat), each checked against something other than itself."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_fss_tables.txt")


def _tables():
    out, cur = {}, None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            cur = line.strip("[]")
            out[cur] = []
            continue
        out[cur].append([float(v) for v in line.split()])
    return {k: np.array(v) for k, v in out.items()}


# ------------------------------------------------------------ P_beta(E)
def test_density_closed_form_for_constant_slope():
    """Constant a: rho~ is one exponential and P_beta(E) on [E0, E0 + W] is
    k e^{k (E - E0)} / (e^{k W} - 1), k = beta - a."""
    c = 100.0 + 3.0 * np.arange(12)
    s, a, beta = 3.0, 0.37, 1.1
    E = np.linspace(c[0] - 1.5, c[-1] + 1.5, 777)
    lp = oracle.prob_density(c, np.full(12, a), s, beta, E)
    k, W = beta - a, 36.0
    ref = np.log(k) + k * (E - E[0]) - np.log(np.expm1(k * W))
    assert np.max(np.abs(lp - ref)) < 1e-12
    # outside the covered range the density vanishes
    assert np.all(np.isneginf(oracle.prob_density(c, np.full(12, a), s, beta, [c[0] - 2.0, c[-1] + 1.6])))


def test_density_normalised_and_continuous():
    rng = np.random.default_rng(3)
    n, s = 40, 0.5
    c = -3.0 + s * np.arange(n)
    a = rng.normal(0.0, 3.0, n)
    beta = 0.4
    # per-interval Simpson integration of e^{ln P} (exact to ~1e-10 here)
    tot = 0.0
    for k in range(n):
        x = np.linspace(c[k] - 0.5 * s, c[k] + 0.5 * s, 201)
        x[0] += 1e-12
        x[-1] -= 1e-12
        y = np.exp(oracle.prob_density(c, a, s, beta, x))
        tot += (x[1] - x[0]) / 3 * (y[0] + y[-1] + 4 * y[1:-1:2].sum() + 2 * y[2:-1:2].sum())
    assert abs(tot - 1.0) < 1e-8
    # ln rho~ is continuous at every interior edge
    edges = c[:-1] + 0.5 * s
    left = oracle.prob_density(c, a, s, beta, edges - 1e-9)
    right = oracle.prob_density(c, a, s, beta, edges + 1e-9)
    assert np.max(np.abs(left - right)) < 1e-7


def test_peaks_against_fine_grid():
    """The maxima of the piecewise-linear ln P sit at interval edges: a scan of
    ln P on a fine grid through every edge finds the same interior maxima."""
    n, s, beta = 64, 10.0, 1.0
    c = 1000.0 + s * np.arange(n)
    k = np.arange(n)
    a = beta - 0.02 * np.sin(2 * np.pi * k / n * 2.0 + 0.3)     # two up-crossings of beta
    Ep, lp = oracle.prob_peaks(c, a, s, beta)
    grid = np.concatenate([np.linspace(c[j] - 0.5 * s, c[j] + 0.5 * s, 11)[:-1] for j in range(n)]
                          + [[c[-1] + 0.5 * s]])
    v = oracle.prob_density(c, a, s, beta, grid)
    mx = [i for i in range(1, grid.size - 1) if v[i] > v[i - 1] and v[i] >= v[i + 1]]
    assert np.allclose(grid[mx], Ep)
    assert np.allclose(v[mx], lp)
    assert Ep.size == 2


def test_peaks_of_a_two_phase_density():
    """ln rho built so that P_beta is a mixture of two Gaussians at E1, E2:
    a = -d ln rho / dE sampled at the centres; the peaks land within one
    interval of E1 and E2."""
    beta, E1, E2, sg = 1.0, 300.0, 420.0, 18.0
    s = 4.0
    c = 200.0 + s * np.arange(130)

    def lnrho(E):
        g = np.logaddexp(-0.5 * ((E - E1) / sg) ** 2, -0.5 * ((E - E2) / sg) ** 2 + np.log(0.7))
        return g - beta * E

    a = -(lnrho(c + 1e-4) - lnrho(c - 1e-4)) / 2e-4
    Ep, lp = oracle.prob_peaks(c, a, s, beta)
    assert Ep.size == 2
    assert abs(Ep[0] - E1) <= s and abs(Ep[1] - E2) <= s
    assert lp[0] > lp[1]                                   # the heavier phase


# ------------------------------------------------------------ bootstrap
def test_bootstrap_indices_are_uniform_draws():
    idx = oracle.bootstrap_indices(7, 3000, seed=11)
    assert idx.shape == (3000, 7) and idx.min() == 0 and idx.max() == 6
    counts = np.bincount(idx.ravel(), minlength=7)
    exp = idx.size / 7
    chi2 = np.sum((counts - exp) ** 2 / exp)
    assert chi2 < 22.5                                     # chi2_6, p = 0.001
    # a different seed gives different draws
    assert not np.array_equal(idx, oracle.bootstrap_indices(7, 3000, seed=12))


def test_bootstrap_of_shifted_runs():
    """Runs that differ by a constant shift d_r of every a_k: the shift moves
    the reconstructed weights from beta to beta - d, so beta_c of a sample is
    beta_c(a) + mean of its drawn shifts and the C_V peak is unchanged."""
    n, s = 48, 6.0
    c = 500.0 + s * np.arange(n)
    k = np.arange(n)
    a = 1.0 + 0.004 * np.tanh((k - 24) / 6.0) - 0.003 * np.exp(-((k - 24) / 5.0) ** 2)
    six_v = 1536.0
    d = np.array([0.0, 3e-4, -2e-4, 5e-4, 1e-4])
    runs = a[None, :] + d[:, None]
    bc0, pk0 = oracle.beta_c(c, a, s, six_v, 0.98, 1.02, h=1e-5, tol=1e-10)
    bc, pk = oracle.bootstrap(c, runs, s, six_v, 0.98, 1.02, n_boot=25, seed=5, h=1e-5, tol=1e-10)
    idx = oracle.bootstrap_indices(5, 25, 5)
    assert np.max(np.abs(bc - (bc0 + d[idx].mean(axis=1)))) < 1e-8
    assert np.max(np.abs(pk / pk0 - 1)) < 1e-7
    # identical runs: no spread
    bc1, pk1 = oracle.bootstrap(c, np.tile(a, (4, 1)), s, six_v, 0.98, 1.02, n_boot=6, seed=1, h=1e-5, tol=1e-10)
    assert np.max(np.abs(bc1 - bc0)) < 1e-9 and np.max(np.abs(pk1 - pk0)) < 1e-9 * pk0


# ------------------------------------------------------------ finite-size fits
def _powers(kmax):
    return np.array([0.0] + [-4.0 * k for k in range(1, kmax + 1)])


def test_fss_fit_reproduces_the_paper_beta_c_fits():
    """Tab. betac from Tab. peakloc: every central value within 1.5 of the
    paper's quoted errors (the tabulated beta_c(L) are rounded, which moves
    the fits' chi2 but not their centres)."""
    t = _tables()
    for Lmin, kmax, bc, err, _ in t["betac"]:
        m = t["peakloc"][:, 0] >= Lmin
        p, e, chi2 = oracle.fss_fit(t["peakloc"][m, 0], t["peakloc"][m, 1], t["peakloc"][m, 2], _powers(int(kmax)))
        assert abs(p[0] - bc) < 1.5 * err, (Lmin, kmax, p[0], bc)


def test_fss_fit_reproduces_the_paper_latent_heat_fits():
    """Tab. latentheat from Tab. peak: G = 2 sqrt(p_0) within 0.5 of the
    quoted error and chi2_red within 20 % of the printed value."""
    t = _tables()
    for Lmin, kmax, G, err, chi2p in t["latent"]:
        m = t["peak"][:, 0] >= Lmin
        p, e, chi2 = oracle.fss_fit(t["peak"][m, 0], t["peak"][m, 1], t["peak"][m, 2], _powers(int(kmax)))
        assert abs(2 * np.sqrt(p[0]) - G) < 0.5 * err, (Lmin, kmax, 2 * np.sqrt(p[0]), G)
        assert abs(chi2 / chi2p - 1) < 0.2, (Lmin, kmax, chi2, chi2p)


def test_fss_fit_exact_model_and_errors():
    """Data exactly on the model are recovered with chi2 = 0; for noisy data the
    errors match the spread of refits over independent noise draws."""
    L = np.array([8.0, 10, 12, 14, 16, 18, 20])
    pw = _powers(2)
    p_true = np.array([1.011126, -0.35, 40.0])
    y = (L[:, None] ** pw[None, :]) @ p_true
    sg = np.full(L.size, 2e-6)
    p, e, chi2 = oracle.fss_fit(L, y, sg, pw)
    assert np.max(np.abs(p - p_true) / np.abs(p_true)) < 1e-8 and chi2 < 1e-12
    rng = np.random.default_rng(0)
    fits = np.array([oracle.fss_fit(L, y + rng.normal(0, 2e-6, L.size), sg, pw)[0] for _ in range(2000)])
    assert np.allclose(fits.std(axis=0), e, rtol=0.1)
