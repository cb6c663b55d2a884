"""What the interleaved order's relabelling costs in decorrelation, on the
oracle (CPU): integrated autocorrelation times (Sokal's window) of the
energy in both sweep orders of the class passes.

Canonically (4D, L=4, beta = 1, no restriction) the overrelaxation right
after an accepted heatbath of its class is a relabelled heatbath draw, so
the interleaved sweep decorrelates E about as slowly as heatbath-only
sweeps, clearly slower than the grouped sweep, whose overrelaxations all act
on staples the heatbath has since changed (seeded; measured tau_int(E) 7.7
grouped, 13.0 interleaved over 12000 sweeps of 8 chains).  In a narrow
restriction (the LLR regime, L=6, w = 0.001 6V) E changes only through
accepted heatbath classes, and the overrelaxations between them (energy
preserving) are what keep the proposals acceptable: both orders decorrelate
E within about a sweep (measured 1.13 and 1.10; E changes in 60 % of the
sweeps), while heatbath-only chains from the same synthetic states never
had a class accepted in 1500 sweeps."""
import numpy as np

import oracle
from tests.inputs import random_state

D = 4


def _tau_int(x, c=6.0):
    """Integrated autocorrelation time of each column (rows: sweeps), with
    Sokal's automatic window W >= c tau."""
    x = x - x.mean(axis=0)
    n = x.shape[0]
    f = np.fft.rfft(x, n=2 * n, axis=0)
    acf = np.fft.irfft(f * np.conj(f), axis=0)[:n]
    acf = acf / acf[0]
    out = np.empty(x.shape[1])
    for k in range(x.shape[1]):
        t = 0.5
        for w in range(1, n):
            t += acf[w, k]
            if w >= c * t:
                break
        out[k] = t
    return out


def _series(L, th, a, lo, hi, E, n, order, do_or, mode):
    """E of every chain after each of n sweeps."""
    nch = th.shape[0]
    out = np.zeros((n, nch))
    for t in range(n):
        E, _ = oracle.sweeps(D, L, th, a, lo, hi, list(range(nch)), E, 1, 1000 + t, mode=mode, seed=5, order=order,
                             do_or=do_or)
        out[t] = E
    return out


def test_canonical_interleaved_order_decorrelates_like_heatbath_only():
    L, nch, n = 4, 8, 12000
    tau = {}
    for name, order, do_or in [("grouped", oracle.SWEEP_GROUPED, True),
                               ("interleaved", oracle.SWEEP_INTERLEAVED, True)]:
        th = oracle.hot_start(D, L, nch, seed=77)
        E = np.array([oracle.energy(D, L, th[k]) for k in range(nch)])
        lo, hi = [-1e9] * nch, [1e9] * nch
        E, _ = oracle.sweeps(D, L, th, [1.0] * nch, lo, hi, list(range(nch)), E, 300, 0, mode=oracle.MODE_FREE,
                             seed=5, order=order, do_or=do_or)
        tau[name] = _tau_int(_series(L, th, [1.0] * nch, lo, hi, E, n, order, do_or, oracle.MODE_FREE)).mean()
    print(f"\ncanonical L=4: tau_int(E) {tau}")
    assert tau["grouped"] < 10.0
    assert tau["interleaved"] > 1.4 * tau["grouped"], tau


def test_restricted_sampling_decorrelates_within_a_sweep_in_both_orders():
    L, nch, n = 6, 4, 1500
    V6 = 6 * L ** 4
    w = 0.001 * V6
    th0 = np.concatenate([random_state(D, L, 1, seed=300 + k, u_target=0.60 + 0.005 * k) for k in range(nch)])
    E0 = np.array([oracle.energy(D, L, th0[k]) for k in range(nch)])
    lo, hi = E0 - 0.5 * w, E0 + 0.5 * w
    a = [1.01] * nch
    tau = {}
    moved = {}
    for name, order, do_or in [("grouped", oracle.SWEEP_GROUPED, True),
                               ("interleaved", oracle.SWEEP_INTERLEAVED, True),
                               ("heatbath only", oracle.SWEEP_GROUPED, False)]:
        th = th0.copy()
        E, _ = oracle.sweeps(D, L, th, a, lo, hi, list(range(nch)), E0, 100, 0, seed=5, order=order, do_or=do_or)
        s = _series(L, th, a, lo, hi, E, n, order, do_or, oracle.MODE_RESTRICTED)
        moved[name] = float(np.mean(np.abs(np.diff(s, axis=0)) > 0))
        if moved[name] > 0.5:
            tau[name] = _tau_int(s).mean()
    print(f"\nrestricted L=6: tau_int(E) {tau}, fraction of sweeps that change E {moved}")
    assert tau["grouped"] < 1.5 and tau["interleaved"] < 1.5, tau
    # heatbath-only chains almost never change their energy
    assert moved["heatbath only"] < 0.05, moved
