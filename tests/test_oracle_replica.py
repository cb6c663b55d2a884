"""Pin of the oracle's replica exchange (Sec. 2.5, the swap probability).

With overlapping intervals I_k = [c_k - w/2, c_k + w/2], w = 2 dE, the chains
of one lattice jointly sample prod_k rho(E_k) e^{a_k E_k} 1[E_k in I_k].  A
swap of the configurations of intervals k and k+1 is a Metropolis move on that
product, so with replica exchange after every sweep the energies visited by
each interval must still follow its own restricted density
rho(E) e^{a_k E} on I_k.  On the 2D L=2 torus the plaquette angles of
Haar-random links are uniform subject to sum_P theta_P = 0 (mod 2 pi), so
that density is sampled exactly and compared bin by bin (chi^2).

The same run with the swap exponent's sign flipped (the exponent as printed,
which belongs to e^{-aS} weights, taken over into the e^{+aE} convention) is
built from the oracle's own source with OR_PLANT_RE_SIGN and must fail.
"""
import numpy as np
import pytest

import oracle

D, L = 2, 2
NP = 4


_EXACT = []


def _exact_2d_l2(n=20_000_000, seed=1):
    """Exact draws of E on the torus (cached: the reference histogram's own
    sampling error must stay below the chains')."""
    if not _EXACT:
        rng = np.random.default_rng(seed)
        t = rng.uniform(-np.pi, np.pi, (n, NP - 1))
        _EXACT.append(np.cos(t).sum(1) + np.cos(-t.sum(1)))
    return _EXACT[0]


def _start_inside(lo, hi, seed):
    rng = np.random.default_rng(seed)
    while True:
        th = rng.uniform(-np.pi, np.pi, (1, D, L ** D))
        if lo <= oracle.energy(D, L, th[0]) <= hi:
            return th


# four intervals, centres 0.8 apart, restriction width 1.6, couplings far
# enough apart that a wrong swap rule visibly distorts the overlaps
CEN = np.array([0.2, 1.0, 1.8, 2.6])
A = np.array([0.0, 1.2, 2.4, 3.6])
W = 1.6
LO, HI = CEN - 0.5 * W, CEN + 0.5 * W


def _run(use, n_sweeps, n_sys=4, seed0=70, order=oracle.SWEEP_GROUPED):
    """n_sys independent systems of 4 chains: a restricted sweep of every
    chain at the coupling of the interval it serves, then replica exchange
    (pairs alternate with the sweep index).  Returns the energies visited by
    each interval, [proposed, accepted] swaps."""
    n = CEN.size
    vis = [[] for _ in range(n)]
    re = np.zeros(2, dtype=np.int64)
    for sys_ in range(n_sys):
        seed = seed0 + sys_
        th = np.ascontiguousarray(np.concatenate([_start_inside(LO[k], HI[k], 1000 * seed + k) for k in range(n)]))
        E = np.array([oracle.energy(D, L, th[c]) for c in range(n)])
        conf = np.arange(n, dtype=np.int32)   # interval -> chain
        itv = np.arange(n, dtype=np.int32)    # chain -> interval
        v = oracle.replica_run(D, L, th, A, LO, HI, E, conf, itv, n_sweeps, 0, seed, lattice_id=sys_,
                               order=order, re_acc=re, use=use)
        for k in range(n):
            vis[k].append(v[200:, k])
        assert sorted(conf.tolist()) == list(range(n))
        assert np.all(itv[conf] == np.arange(n))
        assert np.allclose(E, [oracle.energy(D, L, th[c]) for c in range(n)], atol=1e-9)
    return [np.concatenate(x) for x in vis], re


def _chi2(vis):
    Ex = _exact_2d_l2()
    out = []
    for k, v in enumerate(vis):
        assert np.all((v >= LO[k]) & (v <= HI[k]))
        bins = np.linspace(LO[k], HI[k], 9)
        m = (Ex >= LO[k]) & (Ex <= HI[k])
        p, _ = np.histogram(Ex[m], bins=bins, weights=np.exp(A[k] * (Ex[m] - HI[k])))
        p /= p.sum()
        h, _ = np.histogram(v, bins=bins)
        out.append(np.sum((h - h.sum() * p) ** 2 / (h.sum() * p)) / (bins.size - 1))
    return np.array(out)


@pytest.fixture(scope="module")
def planted(tmp_path_factory):
    return oracle.build_variant(str(tmp_path_factory.mktemp("plant") / "liboracle_re_sign.so"),
                                ["OR_PLANT_RE_SIGN"])


@pytest.mark.parametrize("order", [oracle.SWEEP_GROUPED, oracle.SWEEP_INTERLEAVED])
def test_replica_exchange_keeps_each_restricted_density(order):
    vis, re = _run(None, 40000, order=order)
    chi2 = _chi2(vis)
    acc = re[1] / re[0]
    # swaps are frequent and not always accepted: the rule is exercised
    assert re[0] > 5000 and 0.2 < acc < 0.95, (re, acc)
    # consecutive sweeps are mildly correlated: an inflated chi^2 bar
    # (measured 0.9-1.5 per degree of freedom)
    assert np.all(chi2 < 4.0), chi2


def test_planted_swap_sign_fails(planted):
    vis, re = _run(planted, 40000)
    chi2 = _chi2(vis)
    # measured 56-167 per degree of freedom
    assert np.max(chi2) > 20.0, chi2


def test_swap_rule_on_constructed_pairs():
    """The exchange of one pair against its closed form: eligibility, the
    acceptance exp[(a_k - a_{k+1})(E_{k+1} - E_k)] against the Philox
    uniform, and the label bookkeeping."""
    n = 2
    a = np.array([0.5, 1.7])
    lo, hi = np.array([0.0, 1.0]), np.array([2.0, 3.0])
    seed, t = 99, 4   # t even: pair (0, 1)
    w = oracle.philox(np.array([[0, oracle.ctr1(kind=oracle.KIND_REPLICA), t, 0]], dtype=np.uint32), seed)
    u = (float(w[0, 0]) + 0.5) * 2.0 ** -32
    for EA, EB in [(1.2, 1.9), (1.9, 1.2), (1.5, 1.5), (0.5, 1.9), (1.2, 2.5)]:
        conf = np.arange(n, dtype=np.int32)
        itv = np.arange(n, dtype=np.int32)
        E = np.array([EA, EB])
        re = np.zeros(2, dtype=np.int64)
        oracle.replica_step(conf, itv, E, a, lo, hi, seed, t, re_acc=re)
        eligible = lo[1] <= EA <= hi[1] and lo[0] <= EB <= hi[0]
        x = (a[0] - a[1]) * (EB - EA)
        swap = eligible and (x >= 0 or u < np.exp(x))
        assert re[0] == int(eligible) and re[1] == int(swap)
        assert conf.tolist() == ([1, 0] if swap else [0, 1])
        assert itv.tolist() == conf.tolist()
    # odd sweep index: pair (1, 2) only, which does not exist for n = 2
    conf = np.arange(n, dtype=np.int32)
    itv = np.arange(n, dtype=np.int32)
    re = np.zeros(2, dtype=np.int64)
    oracle.replica_step(conf, itv, np.array([1.5, 1.5]), a, lo, hi, seed, 5, re_acc=re)
    assert re[0] == 0 and conf.tolist() == [0, 1]
