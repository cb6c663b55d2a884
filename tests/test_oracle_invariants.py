"""Oracle pins from invariants of the model (Sec. 3.1): the local-field identity,
gauge invariance of the energy and of the heatbath/overrelaxation updates, the
overrelaxation energy invariant, and the hot start."""
import numpy as np
import pytest

import oracle
from tests.inputs import circ_dist, gauge_transform, random_gauge, random_state


@pytest.mark.parametrize("d,L", [(2, 4), (4, 4)])
def test_local_field_sums_to_four_times_energy(d, L):
    # each plaquette contains 4 links, so sum over links of the local action is 4 E
    th = random_state(d, L, 1, seed=3)[0]
    V = L ** d
    tot = 0.0
    for mu in range(d):
        for s in range(V):
            C, S = oracle.local_field(d, L, th, mu, s)
            tot += C * np.cos(th[mu, s]) - S * np.sin(th[mu, s])
    E = oracle.energy(d, L, th)
    assert abs(tot - 4 * E) < 1e-12 * 4 * d * V


def test_energy_of_trivial_and_random_fields():
    d, L = 4, 4
    V = L ** d
    assert abs(oracle.energy(d, L, np.zeros((d, V))) - 6 * V) < 1e-9
    # a pure gauge is trivial too
    lam = random_gauge(d, L, 1)
    assert abs(oracle.energy(d, L, gauge_transform(np.zeros((d, V)), d, L, lam)) - 6 * V) < 1e-9
    # a constant field theta_mu = c_mu has every plaquette angle 0
    assert abs(oracle.energy(d, L, np.tile(np.array([0.3, -1.2, 2.0, 0.7])[:, None], (1, V))) - 6 * V) < 1e-9


@pytest.mark.parametrize("hb", [1, 0])
def test_gauge_covariance_of_class_pass(hb):
    d, L = 4, 4
    th = random_state(d, L, 1, seed=5)[0]
    lam = random_gauge(d, L, 6)
    thg = gauge_transform(th, d, L, lam)
    E0 = oracle.energy(d, L, th)
    assert abs(oracle.energy(d, L, thg) - E0) < 1e-9
    for colour in range(8):
        a1 = th.copy()
        a2 = thg.copy()
        r1 = oracle.class_pass(d, L, a1, hb, colour, oracle.MODE_FREE, 1.05, 0, 0, E0, seed=77,
                               sweep=3, interval=2)
        r2 = oracle.class_pass(d, L, a2, hb, colour, oracle.MODE_FREE, 1.05, 0, 0, E0, seed=77,
                               sweep=3, interval=2)
        assert abs(r1[2] - r2[2]) < 1e-9
        assert np.max(circ_dist(gauge_transform(a1, d, L, lam), a2)) < 1e-11
        th, thg = a1, a2


def test_overrelaxation_preserves_energy_and_is_involution():
    d, L = 4, 4
    th = random_state(d, L, 1, seed=9)[0]
    E0 = oracle.energy(d, L, th)
    for colour in range(8):
        t0 = th.copy()
        oracle.class_pass(d, L, th, 0, colour, oracle.MODE_RESTRICTED, 1.0, E0 - 1, E0 + 1, E0, seed=1)
        E1 = oracle.energy(d, L, th)
        assert abs(E1 - E0) < 1e-12 * (L ** d // 2) * 8
        changed = circ_dist(th, t0).max()
        assert changed > 1e-3
        t1 = th.copy()
        oracle.class_pass(d, L, t1, 0, colour, oracle.MODE_RESTRICTED, 1.0, E0 - 1, E0 + 1, E0, seed=1)
        assert circ_dist(t1, t0).max() < 1e-12


def test_restricted_pass_respects_interval_and_energy_bookkeeping():
    d, L = 4, 4
    th = random_state(d, L, 1, seed=11)[0]
    E = oracle.energy(d, L, th)
    lo, hi = E - 10.0, E + 10.0
    n_acc = 0
    for sweep in range(20):
        for colour in range(8):
            acc, E, dE, _ = oracle.class_pass(d, L, th, 1, colour, oracle.MODE_RESTRICTED, 1.0, lo, hi,
                                              E, seed=4, sweep=sweep)
            n_acc += acc
            assert lo <= E <= hi
        assert abs(E - oracle.energy(d, L, th)) < 1e-9
    assert 0 < n_acc < 160


def test_hot_start_uniform_and_single_precision_rounding():
    d, L = 4, 4
    th = oracle.hot_start(d, L, 3, seed=42)
    assert th.shape == (3, d, L ** d)
    assert np.all(th >= -np.pi) and np.all(th < np.pi)
    assert abs(th.mean()) < 0.05 and abs(th.var() - np.pi ** 2 / 3) < 0.1
    th32 = oracle.hot_start(d, L, 3, seed=42, f32=True)
    assert np.all(th32.astype(np.float32).astype(np.float64) == th32)
    assert np.max(np.abs(th32 - th)) < 2e-6
    assert not np.array_equal(oracle.hot_start(d, L, 1, seed=43), th[:1])
