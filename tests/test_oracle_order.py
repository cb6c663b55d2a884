"""The oracle's orders of a sweep's class passes (Algorithm 1 asks for one
sweep of the whole system) are the compositions of single class passes they
are defined as: grouped = heatbath of colours 0..2d-1, then overrelaxation
of colours 0..2d-1; interleaved = heatbath then overrelaxation of colour 0,
then of colour 1, ...; staggered = grouped on the first ceil(n/2) chains of
a lattice and overrelaxation of colours 0..2d-1, then heatbath of colours
0..2d-1, on the others.  Angles and energies are compared bit for bit, for
the restricted and the free mode, in 4D and 2D; the orders give different
states, so a swapped dispatch fails too."""
import numpy as np
import pytest

import oracle
from tests.inputs import random_state

SEED = 99


def _compose(d, L, th, a, lo, hi, E, sweep, mode, order):
    if order == "or_first":
        for col in range(2 * d):
            _, E, _, _ = oracle.class_pass(d, L, th, 0, col, mode, a, lo, hi, E, SEED, sweep=sweep, interval=0)
        for col in range(2 * d):
            _, E, _, _ = oracle.class_pass(d, L, th, 1, col, mode, a, lo, hi, E, SEED, sweep=sweep, interval=0)
        return E
    for col in range(2 * d):
        _, E, _, _ = oracle.class_pass(d, L, th, 1, col, mode, a, lo, hi, E, SEED, sweep=sweep, interval=0)
        if order == oracle.SWEEP_INTERLEAVED:
            _, E, _, _ = oracle.class_pass(d, L, th, 0, col, mode, a, lo, hi, E, SEED, sweep=sweep, interval=0)
    if order == oracle.SWEEP_GROUPED:
        for col in range(2 * d):
            _, E, _, _ = oracle.class_pass(d, L, th, 0, col, mode, a, lo, hi, E, SEED, sweep=sweep, interval=0)
    return E


@pytest.mark.parametrize("d,L", [(4, 4), (2, 6)])
@pytest.mark.parametrize("mode", [oracle.MODE_RESTRICTED, oracle.MODE_FREE])
def test_sweep_orders_are_their_pass_compositions(d, L, mode):
    th0 = random_state(d, L, 1, seed=5 + L, u_target=0.6)[0]
    E0 = oracle.energy(d, L, th0)
    lo, hi = E0 - 6.0, E0 + 6.0          # narrow: restricted heatbath passes get rejected
    out = {}
    for order in (oracle.SWEEP_GROUPED, oracle.SWEEP_INTERLEAVED):
        t_sw = np.ascontiguousarray(th0[None].copy())
        E_sw, _ = oracle.sweeps(d, L, t_sw, [1.1], [lo], [hi], [0], [E0], 1, 3, mode=mode, seed=SEED, order=order)
        t_cp = th0.copy()
        E_cp = _compose(d, L, t_cp, 1.1, lo, hi, E0, 3, mode, order)
        assert np.array_equal(t_sw[0], t_cp), order
        assert E_sw[0] == E_cp, order
        out[order] = t_sw[0]
    assert not np.array_equal(out[oracle.SWEEP_GROUPED], out[oracle.SWEEP_INTERLEAVED])


@pytest.mark.parametrize("mode", [oracle.MODE_RESTRICTED, oracle.MODE_FREE])
def test_staggered_order_splits_each_lattice_in_two(mode):
    """Five chains of one 4D L=4 lattice: chains 0-2 (the first ceil(5/2))
    sweep in the grouped order, chains 3-4 overrelaxation first; the same
    with a subset of the chains given by their indices in the lattice."""
    d, L = 4, 4
    th0 = random_state(d, L, 5, seed=17, u_target=0.6)
    E0 = np.array([oracle.energy(d, L, th0[k]) for k in range(5)])
    lo, hi = E0 - 6.0, E0 + 6.0
    t_sw = th0.copy()
    E_sw, bits = oracle.sweeps(d, L, t_sw, [1.1] * 5, lo, hi, [0] * 5, E0, 1, 3, mode=mode, seed=SEED,
                               order=oracle.SWEEP_STAGGERED)
    for k in range(5):
        t_cp = th0[k].copy()
        E_cp = _compose(d, L, t_cp, 1.1, lo[k], hi[k], E0[k], 3, mode, oracle.SWEEP_GROUPED if k < 3 else "or_first")
        assert np.array_equal(t_sw[k], t_cp), k
        assert E_sw[k] == E_cp, k
        t_g = th0[k].copy()
        _compose(d, L, t_g, 1.1, lo[k], hi[k], E0[k], 3, mode, oracle.SWEEP_GROUPED)
        assert np.array_equal(t_sw[k], t_g) == (k < 3), k
    # chains 1 and 4 alone, as chains of the five-chain lattice
    t_sub = np.ascontiguousarray(th0[[1, 4]])
    E_sub, _ = oracle.sweeps(d, L, t_sub, [1.1] * 2, lo[[1, 4]], hi[[1, 4]], [0, 0], E0[[1, 4]], 1, 3, mode=mode,
                             seed=SEED, order=oracle.SWEEP_STAGGERED, chain=[1, 4], n_lattice_chains=5)
    assert np.array_equal(t_sub, t_sw[[1, 4]])
    assert np.array_equal(E_sub, E_sw[[1, 4]])


def test_overrelaxation_right_after_the_heatbath_of_its_class_is_a_relabelled_draw():
    """In the interleaved order the overrelaxation of colour c follows the
    heatbath of colour c on the same staples (links of one colour share no
    plaquette).  The heatbath writes theta' = X - phi with X ~ vM(a R); the
    reflection then gives -2 phi - theta' = -X - phi.  Since the von Mises
    law is symmetric, that is one more heatbath draw, not a second update:
    an accepted heatbath class followed by its overrelaxation counts as one
    update, a rejected one as the overrelaxation of the old angles.  Checked
    link by link (the staples unchanged by the pass, the identity to
    rounding) and in law (probability integral transforms of -X through each
    link's von Mises CDF are uniform)."""
    from scipy import stats

    d, L, a = 4, 4, 1.1
    V = L ** d
    pit = []
    for rep in range(6):
        th = random_state(d, L, 1, seed=40 + rep, u_target=0.62)[0]
        for col in range(2 * d):
            mu, p = col >> 1, col & 1
            sites = [s for s in range(V) if sum((s // L ** m) % L for m in range(d)) % 2 == p]
            CS = np.array([oracle.local_field(d, L, th, mu, s) for s in sites])
            phi = np.arctan2(CS[:, 1], CS[:, 0])
            kap = a * np.hypot(CS[:, 0], CS[:, 1])
            E = oracle.energy(d, L, th)
            acc, E, _, _ = oracle.class_pass(d, L, th, 1, col, oracle.MODE_FREE, a, -1e9, 1e9, E, SEED,
                                             sweep=100 + rep, interval=col)
            assert acc
            CS2 = np.array([oracle.local_field(d, L, th, mu, s) for s in sites])
            assert np.array_equal(CS, CS2)          # the class's own staples are untouched
            X = np.angle(np.exp(1j * (th[mu, sites] + phi)))
            oracle.class_pass(d, L, th, 0, col, oracle.MODE_FREE, a, -1e9, 1e9, E, SEED, sweep=100 + rep,
                              interval=col)
            Xo = np.angle(np.exp(1j * (th[mu, sites] + phi)))
            dist = np.abs(np.angle(np.exp(1j * (Xo + X))))
            assert dist.max() < 1e-12, dist.max()   # -2 phi - (X - phi) = -X - phi
            pit.append(stats.vonmises.cdf(Xo, kap))
    pit = np.concatenate(pit)
    assert stats.kstest(pit, "uniform").pvalue > 1e-3
