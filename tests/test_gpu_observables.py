"""GPU parity of the non-action observable measurement and of the
double-bracket reconstruction (Sec. 2.3, eqs. (l9)-(l10)) through the C ABI:
the measurement's restricted sweeps and FP64 (E, sum_P cos 2 theta_P) within
1e-9 relative of the oracle's over two measurements (inside the divergence
horizon of the two implementations), samples reported in interval order
(also with replica exchange), the reconstruction within 1e-10."""
import numpy as np
import pytest

import oracle
from tests.inputs import random_state

pytestmark = pytest.mark.gpu

SEED = 1509083910


@pytest.fixture(scope="module")
def llr():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1509_08391_amd import llr as m
    m.lib()
    return m


def _setup(llr, L, n, replica):
    import torch
    d = 4
    th = np.concatenate([random_state(d, L, 1, seed=300 + k, u_target=0.5 + 0.2 * k / n) for k in range(n)])
    E = np.array([oracle.energy(d, L, th[k]) for k in range(n)])
    order = np.argsort(E)
    th, E = np.ascontiguousarray(th[order]), E[order]
    # each state at the centre of its own interval; wide enough that
    # neighbouring intervals overlap (replica exchange then has partners)
    dE = 400.0
    E_low = E - 0.5 * dE
    ctx = llr.Context(precision=llr.FP64)
    ctx.set_params(seed=SEED, replica_exchange=replica)
    ctx.add_lattice(L, E_low, dE)
    ctx.bind_state()
    a = np.linspace(0.9, 1.1, n)
    ctx.set_a(0, a)
    ctx.import_state(0, torch.from_numpy(th))
    return ctx, th, E, E_low, dE, a


@pytest.mark.parametrize("order", ["grouped", "interleaved"])
@pytest.mark.parametrize("L", [4, 6])
def test_observables_match_oracle_fp64(llr, L, order):
    d, n = 4, 5
    ctx, th, E, E_low, dE, a = _setup(llr, L, n, replica=False)
    ctx.set_sweep_order(llr.SWEEP_INTERLEAVED if order == "interleaved" else llr.SWEEP_GROUPED)
    Eg, Bg = ctx.observables(2, 1, 7)
    ctx.close()
    tr, Er = th.copy(), E.copy()
    o_order = oracle.SWEEP_INTERLEAVED if order == "interleaved" else oracle.SWEEP_GROUPED
    for m in range(2):
        Er, _ = oracle.sweeps(d, L, tr, a, E_low, E_low + dE, np.arange(n), Er, 1, 7 + m, seed=SEED,
                              order=o_order)
        Eo = np.array([oracle.energy(d, L, tr[k]) for k in range(n)])
        Bo = np.array([oracle.adjoint(d, L, tr[k]) for k in range(n)])
        assert np.max(np.abs(Eg[m] - Eo) / np.abs(Eo)) < 1e-9
        assert np.max(np.abs(Bg[m] - Bo)) < 1e-9 * 6 * L ** 4


def test_observables_follow_the_interval_labels(llr):
    """With replica exchange the configurations move between chains; column k
    must hold the energy of whichever chain serves interval k."""
    L, n = 4, 6
    ctx, th, E, E_low, dE, a = _setup(llr, L, n, replica=True)
    Eg, _ = ctx.observables(20, 1, 7)
    ctx_stats = ctx.stats()
    ctx.close()
    # with replica exchange the restriction is [c_k - dE, c_k + dE]
    cen = E_low + 0.5 * dE
    inside = (Eg >= cen[None, :] - dE - 1e-6) & (Eg <= cen[None, :] + dE + 1e-6)
    assert np.all(inside)
    # and the configurations did move between chains
    hp, ha, rp, ra = ctx_stats
    assert ra > 0


def test_obs_reconstruct_matches_oracle(llr):
    rng = np.random.default_rng(8)
    n, s, m = 32, 122.88, 200
    c = 13516.8 + s * (np.arange(n) + 0.5)
    a = 0.98 + 0.003 * np.arange(n) + rng.normal(0, 0.002, n)
    E = c[None, :] + rng.uniform(-0.5 * s, 0.5 * s, (m, n))
    B = 0.1 * E + rng.normal(0, 5.0, (m, n))
    beta = np.linspace(0.98, 1.04, 7)
    ctx = llr.Context(precision=llr.FP64)
    g = ctx.obs_reconstruct(c, a, s, E, B, beta)
    ctx.close()
    o = oracle.obs_reconstruct(c, a, s, E, B, beta)
    assert np.max(np.abs(g / o - 1)) < 1e-10
