"""GPU parity of the heatbath under the per-link analytic constraint (Sec.
2.4; mode LLR_MODE_LINK) through the C ABI, against the oracle:

  * FP64 sweeps on L=4 and L=6 with intervals narrow enough that the
    constraint binds (links re-drawn, some by the arc sampler), four sweeps
    in a row, each compared with one oracle sweep from the GPU's state and
    carried energy before it: energies within 1e-9 relative, angles with a
    median within 1e-11 and a maximum within 1e-8.  The walk carries the
    running energy in fixed point, the oracle in FP64, so the window bounds
    of the two differ by the rounding of either; the arc
    sampler starts at x_a = acos(u_hi), whose slope 1/sqrt(1 - u_hi^2)
    magnifies that near the top of the arc (measured with the class sums'
    2^-38 at L=4: 7e-10 at most, the other links ~1e-13; at L=6, 2^-36,
    1.5e-8; the walk now carries E 12 bits finer).  Run on without re-synchronising, the two
    trajectories separate by ~30x per sweep for that reason (measured: a
    median of 8e-9 and a maximum of 1e-3 after four sweeps, energies still
    within 1e-4, so no draw differed), which is why each sweep is checked
    from a common state;
  * with an unbounded interval the pass is the free heatbath: angles bit for
    bit in both precisions, FP32 energies bit for bit (the same 2^-25
    per-link values), FP64 energies within five standard deviations of the
    class sums' rounding walk (the walk rounds each link 12 bits finer);
  * FP32 single passes against the FP32 oracle, chain by chain, with chains
    whose oracle walk took a decision within 1e-4 of its threshold set aside;
  * the walk keeps every chain inside its interval, and its carried FP32
    energy drifts from a full recomputation no more than the class-wise
    passes' does (measured: ~1e-3 after 5 sweeps at L=6, ~2e-8 per link
    update, the reason the FP64 recompute runs every K sweeps);
  * Algorithm 1 with the restriction imposed per link (llr_set_restriction):
    two Robbins-Monro iterations of one sweep each, replayed from captured
    graphs, against the oracle's run from the same states (a_k, energies,
    angles), and the full L=4 run over 8 seeds as distributions of the final
    a_k, FP64 and FP32."""
import numpy as np
import pytest

import oracle
from tests.inputs import circ_dist, random_state
from tests.test_gpu_parity import _states_in_intervals

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


def _states(L, n, seed, dtype=np.float64):
    d = 4
    th = np.concatenate([random_state(d, L, 1, seed=seed + k, u_target=0.5 + 0.15 * k / n, dtype=dtype)
                         for k in range(n)]).astype(np.float64)
    E = np.array([oracle.energy(d, L, th[k]) for k in range(n)])
    o = np.argsort(E)
    return np.ascontiguousarray(th[o]), E[o]


def _ctx(llr, prec, L, th, E_low, dE, a):
    import torch
    ctx = llr.Context(precision=prec)
    ctx.set_params(seed=SEED)
    ctx.add_lattice(L, E_low, dE)
    ctx.bind_state()
    ctx.set_a(0, a)
    dt = np.float32 if prec == llr.FP32 else np.float64
    ctx.import_state(0, torch.from_numpy(th.astype(dt)))
    return ctx


@pytest.mark.parametrize("L", [4, 6])
def test_link_sweeps_match_oracle_fp64(llr, L):
    d, n = 4, 8
    th, E = _states(L, n, 500 + L)
    dE = 16.0                            # per-link |Delta E| reaches 12: the window binds
    E_low = E - 0.5 * dE
    a = 0.9 + 0.02 * np.arange(n)
    ctx = _ctx(llr, llr.FP64, L, th, E_low, dE, a)
    for t in range(4):
        tr = ctx.export_state(0).cpu().numpy().copy()
        E0, _ = ctx.get_energy(0)
        bits = ctx.sweeps(1, sweep0=3 + t, mode=llr.MODE_LINK)
        assert np.all((bits & 0xff) == 0xff)            # every heatbath pass accepted
        Eg, _ = ctx.get_energy(0)
        Er, _ = oracle.sweeps(d, L, tr, a, E_low, E_low + dE, np.arange(n), E0, 1, 3 + t,
                              mode=oracle.MODE_LINK, seed=SEED)
        assert np.max(np.abs(Eg - Er) / np.abs(Er)) < 1e-9, (t, Eg - Er)
        dist = circ_dist(ctx.export_state(0).cpu().numpy(), tr)
        assert np.max(dist) < 1e-8 and np.median(dist) < 1e-11, (t, np.max(dist), np.median(dist))
        assert np.all((Eg >= E_low - 1e-9) & (Eg <= E_low + dE + 1e-9))
    fixes, arcs = ctx.link_stats()
    ctx.close()
    assert fixes.sum() > 0 and arcs.sum() > 0, (fixes, arcs)


@pytest.mark.parametrize("prec", ["FP64", "FP32"])
def test_link_unbounded_is_free_heatbath(llr, prec):
    L, n = 6, 4
    p = getattr(llr, prec)
    th, E = _states(L, n, 40, np.float32 if prec == "FP32" else np.float64)
    out = []
    for mode in (llr.MODE_LINK, llr.MODE_FREE):
        V6 = 6.0 * L ** 4                # intervals spanning [-6V, 6V]: nothing binds
        ctx = _ctx(llr, p, L, th, -V6 + 1e-3 * np.arange(n), 2 * V6 - 0.01, np.full(n, 0.95))
        ctx.sweeps(2, sweep0=9, mode=mode)
        out.append((ctx.export_state(0).cpu().numpy(), ctx.get_energy(0)[0]))
        if mode == llr.MODE_LINK:
            fixes, _ = ctx.link_stats()
            assert fixes.sum() == 0
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0])
    if prec == "FP32":
        assert np.array_equal(out[0][1], out[1][1])
    else:
        # the class sums round each link to 2^-fxb (fxb = floor(49 - log2 6V)):
        # over n_upd link updates their energy carries a rounding walk of
        # standard deviation 2^-fxb sqrt(n_upd / 12); 5 of those
        fxb = np.floor(49 - np.log2(6.0 * L ** 4))
        n_upd = 2 * 8 * L ** 4 // 2
        assert np.max(np.abs(out[0][1] - out[1][1])) < 5 * 2.0 ** -fxb * np.sqrt(n_upd / 12)


def test_link_class_pass_fp32_matches_oracle(llr):
    d, L, n = 4, 6, 8
    th, E = _states(L, n, 900, np.float32)
    dE = 16.0
    E_low = E - 0.5 * dE
    a = np.full(n, 1.0)
    ctx = _ctx(llr, llr.FP32, L, th, E_low, dE, a)
    E0, _ = ctx.get_energy(0)
    checked = 0
    for colour in (0, 5):
        ctx.class_pass(1, colour, mode=llr.MODE_LINK, sweep_index=11)
        got = ctx.export_state(0).cpu().numpy().astype(np.float64)
        Eg, _ = ctx.get_energy(0)
        for k in range(n):
            t = th[k].copy()
            Eo, mg, how = oracle.link_pass(d, L, t, colour, 1.0, E_low[k], E_low[k] + dE, E0[k], SEED,
                                           sweep=11, interval=k, f32=True)
            assert np.all(how > 0)
            if np.min(mg) < 1e-4:
                continue
            dist = circ_dist(got[k], t)
            assert np.median(dist) < 1e-6 and np.max(dist) < 1e-3, (colour, k, np.max(dist))
            assert abs(Eg[k] - Eo) < 1e-3, (colour, k, Eg[k] - Eo)
            checked += 1
        th = got
        E0 = Eg
    ctx.close()
    assert checked >= n


def test_link_walk_stays_inside_fp32(llr):
    """Every chain stays inside its interval; the carried FP32 energy drifts
    from a full FP64 recomputation no more than that of the class-wise
    passes (free sweeps on the same states) does over as many sweeps."""
    L, n = 6, 16
    th, E = _states(L, n, 77, np.float32)
    dE = 12.0
    E_low = E - 0.5 * dE
    drift = {}
    for mode in (llr.MODE_LINK, llr.MODE_FREE):
        ctx = _ctx(llr, llr.FP32, L, th, E_low, dE, np.full(n, 1.0))
        d = []
        for r in range(4):
            ctx.sweeps(5, sweep0=20 + 5 * r, mode=mode)
            Eg, _ = ctx.get_energy(0)
            if mode == llr.MODE_LINK:
                assert np.all((Eg >= E_low - 1e-6) & (Eg <= E_low + dE + 1e-6))
            ctx.recompute_energy()
            Er, _ = ctx.get_energy(0)
            d.append(np.max(np.abs(Er - Eg)))
        if mode == llr.MODE_LINK:
            fixes, arcs = ctx.link_stats()
            hp, ha, _, _ = ctx.stats()
            assert np.array_equal(hp, ha) and fixes.sum() > 0
        ctx.close()
        drift[mode] = max(d)
    assert drift[llr.MODE_LINK] < 2.0 * drift[llr.MODE_FREE] + 1e-4, drift


def test_link_mode_arguments(llr):
    """Modes outside the public set and the multicanonical mode through the
    plain sweep hooks are rejected; the per-link counters need bound state
    and start at zero."""
    ctx = llr.Context(precision=llr.FP64)
    with pytest.raises(llr.LLRError):
        ctx.link_stats()
    ctx.set_params(seed=SEED)
    ctx.add_lattice(4, [100.0, 200.0], 50.0)
    ctx.bind_state()
    with pytest.raises(llr.LLRError):
        ctx.sweeps(1, mode=5)
    with pytest.raises(llr.LLRError):
        ctx.class_pass(1, 0, mode=llr.MODE_MUCA)
    fixes, arcs = ctx.link_stats()
    ctx.close()
    assert fixes.sum() == 0 and arcs.sum() == 0


def test_run_per_link_matches_oracle_fp64(llr):
    """Two Robbins-Monro iterations (N_TH = 0, N_A = 1, E recomputed after
    every sweep) with the per-link restriction from the same states: the
    trajectories separate only through the window bounds' rounding (see the
    module notes), ~1e-8 after two sweeps."""
    import torch
    d, L, n = 4, 4, 6
    V6 = 6 * L ** 4
    dE = 0.02 * V6
    E_low = 0.58 * V6 + dE * np.arange(n)
    th = _states_in_intervals(L, E_low, dE, seed=31)
    ctx = llr.Context(precision=llr.FP64)
    ctx.set_params(seed=SEED, n_th=0, n_a=1, n_rm=2, recompute_every=1)
    ctx.add_lattice(L, E_low, dE)
    ctx.bind_state()
    ctx.set_a(0, 1.0)
    ctx.import_state(0, torch.from_numpy(th))
    ctx.set_restriction(True)
    ctx.run()
    a, _, _ = ctx.get_a(0)
    hist = ctx.get_history(0)
    E, _ = ctx.get_energy(0)
    got = ctx.export_state(0).cpu().numpy()
    fixes, _ = ctx.link_stats()
    ctx.close()
    r = oracle.llr_run(d, L, E_low, dE, 1.0, n_th=0, n_a=1, n_rm=2, seed=SEED, recompute_every=1,
                       theta=th, approach_cap=0, per_link=True)
    assert fixes.sum() > 0
    assert np.max(np.abs(hist - r["a_hist"])) < 1e-7
    assert np.max(np.abs(a - r["a"])) < 1e-7
    assert np.max(np.abs(E - r["E"]) / np.abs(r["E"])) < 1e-9
    dist = circ_dist(got, r["theta"])
    assert np.max(dist) < 1e-5 and np.median(dist) < 1e-10, (np.max(dist), np.median(dist))


def test_set_restriction_arguments(llr):
    """Only 0 and 1 are accepted; switching back to the class-wise restriction
    leaves the per-link counters untouched."""
    ctx = llr.Context(precision=llr.FP32)
    ctx.set_params(seed=SEED, n_th=0, n_a=2, n_rm=1)
    L = 4
    V6 = 6 * L ** 4
    dE = 0.02 * V6
    E_low = 0.58 * V6 + dE * np.arange(3)
    ctx.add_lattice(L, E_low, dE)
    ctx.bind_state()
    with pytest.raises(llr.LLRError):
        ctx.set_restriction(2)
    import torch
    ctx.import_state(0, torch.from_numpy(_states_in_intervals(L, E_low, dE, seed=32).astype(np.float32)))
    ctx.set_a(0, 1.0)
    ctx.set_restriction(False)
    ctx.run()
    fixes0, _ = ctx.link_stats()
    ctx.close()
    assert fixes0.sum() == 0


@pytest.mark.slow
def test_full_run_per_link_statistical(llr):
    """The L=4 case of Algorithm 1 in full (8 intervals over u in [0.5, 0.7],
    dE = 0.025 6V, N_TH = N_A = 100, N_RM = 20, a^(0) = 1, hot start) with the
    per-link restriction: final a_k over 8 seeds, GPU FP64 and FP32 against
    the oracle's per-link runs, means within 4 combined standard errors."""
    L, d = 4, 4
    V6 = 6 * L ** 4
    dE = 0.025 * V6
    E_low = 0.5 * V6 + dE * np.arange(8)
    # 8 seeds: with 4, a sample standard deviation can fall several times below
    # the true one (measured: 0.0009 against 0.0036 over 12 seeds) and the
    # 4-standard-error bar with it
    seeds = [SEED + 17 * i for i in range(8)]
    O = np.array([oracle.llr_run(d, L, E_low, dE, 1.0, n_th=100, n_a=100, n_rm=20, seed=sd,
                                 approach_cap=20000, per_link=True)["a"] for sd in seeds])
    for prec in ("FP64", "FP32"):
        G = []
        for sd in seeds:
            ctx = llr.Context(precision=getattr(llr, prec))
            ctx.set_params(seed=sd, n_th=100, n_a=100, n_rm=20, approach_cap=20000)
            ctx.add_lattice(L, E_low, dE)
            ctx.bind_state()
            ctx.set_a(0, 1.0)
            ctx.set_restriction(True)
            ctx.hot_start()
            ctx.approach()
            ctx.run()
            G.append(ctx.get_a(0)[0])
            fixes, _ = ctx.link_stats()
            assert fixes.sum() > 0
            ctx.close()
        G = np.array(G)
        se = np.maximum(np.sqrt(G.var(0, ddof=1) / len(seeds) + O.var(0, ddof=1) / len(seeds)), 2e-4)
        z = np.abs(G.mean(0) - O.mean(0)) / se
        assert np.all(z < 4.0), (prec, z, G.mean(0) - O.mean(0))
