"""Pins of the oracle's per-link analytic constraint (Sec. 2.4: the energy
restriction imposed when each new link angle is generated, the alternative
to rejecting a whole colour class):

  * the restricted sampler draws X ~ exp(kappa cos X) on cos X in
    [u_lo, u_hi]: Kolmogorov-Smirnov against the CDF of that density from
    numerical quadrature, for windows in the bulk, in the far tail (where only
    the arc sampler can succeed), narrow bands, kappa = 0, and the full window
    against scipy's von Mises distribution;
  * with an unbounded interval the pass is the free heatbath, angle for angle;
  * on the 2D L=2 torus, where the plaquette angles of Haar-random links are
    uniform subject to sum_P theta_P = 0 (mod 2 pi) and so are sampled
    exactly, the energies visited by restricted sweeps follow
    rho(E) e^{a E} on [lo, hi], for the per-link constraint and for the
    class-wise rejection alike, the latter in both orders of a sweep's
    class passes;
  * the running energy of a 4D chain stays inside its interval after every
    link and agrees with a full recomputation."""
import numpy as np
import pytest
from scipy import integrate, stats

import oracle


def _truncated_cdf(kappa, u_lo, u_hi, n=200001):
    xa, xb = np.arccos(u_hi), np.arccos(u_lo)
    x = np.linspace(xa, xb, n)
    f = np.exp(kappa * (np.cos(x) - 1.0))
    F = integrate.cumulative_trapezoid(f, x, initial=0.0)
    F /= F[-1]
    return lambda v: np.interp(v, x, F)


@pytest.mark.parametrize("kappa,u_lo,u_hi,stage2", [
    (2.0, 0.3, 1.0, False),      # lower cut, bulk
    (6.0, -1.0, -0.5, True),     # far tail: the arc sampler does the work
    (6.0, 0.95, 1.0, False),     # narrow window at the mode
    (0.5, 0.2, 0.3, True),       # narrow band, weak coupling
    (12.0, -0.2, 0.4, True),     # band away from a sharp mode
    (3.0, -1.0, 0.99, False),    # upper cut excluding the mode
    (0.0, -0.3, 0.9, False),     # uniform on the arc
])
def test_restricted_sampler_is_the_truncated_von_mises(kappa, u_lo, u_hi, stage2):
    n = 100000
    X, how = oracle.link_draw(n, kappa, u_lo, u_hi, seed=1509 + int(10 * kappa))
    assert np.all(how > 0)
    c = np.cos(X)
    assert np.all((c >= u_lo - 1e-15) & (c <= u_hi + 1e-15))
    p = stats.kstest(np.abs(X), _truncated_cdf(kappa, u_lo, u_hi)).pvalue
    assert p > 1e-3, p
    assert abs(np.mean(np.sign(X))) < 5.0 / np.sqrt(n)
    if stage2:
        assert np.mean(how == 2) > 0.05
    else:
        assert np.mean(how == 1) > 0.3


def test_full_window_is_von_mises():
    n = 100000
    for kappa in (0.7, 4.0):
        X, how = oracle.link_draw(n, kappa, -1.0, 1.0, seed=77)
        assert np.all(how == 1)
        assert stats.kstest(X, stats.vonmises(kappa).cdf).pvalue > 1e-3


def test_unbounded_interval_is_the_free_heatbath():
    d, L = 4, 4
    th = oracle.hot_start(d, L, 1, 3)[0]
    E = oracle.energy(d, L, th)
    t1, t2 = th.copy(), th.copy()
    E1, E2 = E, E
    for colour in range(2 * d):
        E1, _, how = oracle.link_pass(d, L, t1, colour, 0.9, -1e9, 1e9, E1, seed=5, sweep=2, interval=1)
        assert np.all(how == 1)
        _, E2, _, _ = oracle.class_pass(d, L, t2, 1, colour, oracle.MODE_FREE, 0.9, -1e9, 1e9, E2, seed=5,
                                        sweep=2, interval=1)
    assert np.array_equal(t1, t2)
    assert abs(E1 - E2) < 1e-12 * abs(E2)


def _exact_2d_l2(n=8000000, seed=1):
    rng = np.random.default_rng(seed)
    t = rng.uniform(-np.pi, np.pi, (n, 3))
    return np.cos(t).sum(1) + np.cos(-t.sum(1))


def _start_inside(d, L, lo, hi, n, seed):
    rng = np.random.default_rng(seed)
    V = L ** d
    out = []
    while len(out) < n:
        th = rng.uniform(-np.pi, np.pi, (d, V))
        if lo <= oracle.energy(d, L, th) <= hi:
            out.append(th)
    return np.array(out)


@pytest.mark.parametrize("lo,hi,a", [(0.5, 1.5, 1.3), (2.6, 3.4, 0.8)])
def test_restricted_sweeps_sample_rho_e_aE_2d(lo, hi, a):
    d, L, nch = 2, 2, 4
    Ex = _exact_2d_l2()
    m = (Ex >= lo) & (Ex <= hi)
    bins = np.linspace(lo, hi, 9)
    p, _ = np.histogram(Ex[m], bins=bins, weights=np.exp(a * (Ex[m] - hi)))
    p /= p.sum()
    for mode, order in ((oracle.MODE_LINK, oracle.SWEEP_GROUPED), (oracle.MODE_RESTRICTED, oracle.SWEEP_GROUPED),
                        (oracle.MODE_RESTRICTED, oracle.SWEEP_INTERLEAVED)):
        th = _start_inside(d, L, lo, hi, nch, 11)
        E = np.array([oracle.energy(d, L, th[i]) for i in range(nch)])
        args = ([a] * nch, [lo] * nch, [hi] * nch, list(range(nch)))
        E, _ = oracle.sweeps(d, L, th, *args, E, 200, 0, mode=mode, seed=4, order=order)
        vis = []
        for k in range(6000):
            E, _ = oracle.sweeps(d, L, th, *args, E, 2, 1000 + 2 * k, mode=mode, seed=4, order=order)
            vis.append(E.copy())
        vis = np.ravel(vis)
        assert np.all((vis >= lo) & (vis <= hi))
        h, _ = np.histogram(vis, bins=bins)
        chi2 = np.sum((h - h.sum() * p) ** 2 / (h.sum() * p)) / (bins.size - 1)
        # consecutive samples are mildly correlated: an inflated chi2 bar
        assert chi2 < 4.0, (mode, order, chi2)


def test_running_energy_stays_inside_4d():
    d, L = 4, 4
    V6 = 6 * L ** d
    th = oracle.hot_start(d, L, 1, 8)[0]
    # bring the chain to u ~ 0.55 with free sweeps at a coupling that gets there
    E = oracle.energy(d, L, th)
    E, _ = oracle.sweeps(d, L, th[None], [1.0], [-1e9], [1e9], [0], [E], 30, 0, mode=oracle.MODE_FREE, seed=2)
    E = float(E[0])
    lo, hi = E - 6.0, E + 6.0           # narrow: the constraint binds often
    n2 = 0
    for sweep in range(3):
        for colour in range(2 * d):
            E, mg, how = oracle.link_pass(d, L, th, colour, 1.0, lo, hi, E, seed=9, sweep=sweep)
            assert np.all(how > 0)
            n2 += int(np.sum(how == 2))
            assert lo <= E <= hi
            assert abs(E - oracle.energy(d, L, th)) < 1e-10 * V6
    assert n2 > 0
