"""The oracle's two orders of a sweep's class passes (Algorithm 1 asks for
one sweep of the whole system; every link gets one heatbath and one
overrelaxation update in either) are the compositions of single class passes
they are defined as: grouped = heatbath of colours 0..2d-1, then
overrelaxation of colours 0..2d-1; interleaved = heatbath then
overrelaxation of colour 0, then of colour 1, ...  Angles and energies are
compared bit for bit, for the restricted and the free mode, in 4D and 2D;
the two orders give different states, so a swapped dispatch fails too."""
import numpy as np
import pytest

import oracle
from tests.inputs import random_state

SEED = 99


def _compose(d, L, th, a, lo, hi, E, sweep, mode, order):
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
