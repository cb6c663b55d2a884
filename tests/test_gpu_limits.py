"""GPU parity at the largest sizes the boundary accepts (llr_add_lattice:
L <= 32, at most 4096 intervals per lattice).

- L = 32, the largest lattice: 4 * 32^4 links per chain, 2^19 class links
  per colour, the fixed-point energy scale at its smallest (2^26); one
  restricted sweep of two chains in both tile shapes, with both outcomes of
  the interval test among the class passes, accept bits identical,
  energies within 1e-9 relative, the FP64 energy recompute equal to the
  oracle's energy of the swept state, and angles to the bar of the full-size
  FP64 parity test: 99.999 % within 1e-12 of the oracle, all within 1e-10
  (a link with a small staple modulus R amplifies the two sides' ulp-level
  differences of sin, cos and atan2 by ~1/R in the staple phase, and the
  largest such amplification grows with the number of links; measured:
  8 of the 8.4 M links above 1e-12, maximum 4.4e-12).  The same in FP32 with the
  benchmark's tiles, against the oracle's sweep of the same FP32 state, to
  the bar of the full-size FP32 parity test (per link 1e-6 x max(10, the
  link's amplification through the sweep), at least 99.9 % of links;
  measured 99.997 %, median 2.4e-7, energy within 0.06).
- 4096 intervals, the most per lattice, on L = 2 (the degenerate lattice
  whose forward and backward neighbours coincide): a short Robbins-Monro run
  (two iterations, four sweeps) with replica exchange, where the single-block kernels (end of sweep,
  replica exchange, Robbins-Monro update) loop over four times their 1024
  threads; accept bits, chain <-> interval labels and replica counts
  identical to the oracle, every a_k^(n) within 1e-7, energies within 1e-12
  relative at the median and 1e-8 at the worst chain."""
import numpy as np
import pytest

import oracle
from tests.inputs import circ_dist, random_state

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


@pytest.mark.parametrize("tiles", [(1, 1), (4, 2)])
def test_largest_lattice_one_sweep_fp64(llr, tiles):
    import torch
    d, L, n = 4, 32, 2
    th = random_state(d, L, n, seed=3201, u_target=0.6)
    E0 = np.array([oracle.energy(d, L, th[k]) for k in range(n)])
    order = np.argsort(E0)
    th, E0 = np.ascontiguousarray(th[order]), E0[order]
    # each chain inside its own interval, placed so that both outcomes of the
    # interval test occur: this state gains ~0.05-0.24 per class link and
    # pass (1e4-1e5 at L = 32), so the first class passes are accepted and
    # the later ones, which would leave the interval, refused
    width = 0.05 * 6 * L ** 4
    lo = E0 - 0.1 * width
    assert lo[1] > lo[0]
    a = np.array([0.97, 1.03])
    ctx = llr.Context(precision=llr.FP64, device=0)
    ctx.set_params(seed=SEED)
    # uneven edges: each interval is placed on its own chain
    ctx.add_lattice(L, lo, width)
    ctx.bind_state()
    ctx.set_a(0, a)
    ctx.set_tiles(*tiles)
    ctx.import_state(0, torch.from_numpy(th.copy()))
    bits = ctx.sweeps(1, sweep0=5)
    got = ctx.export_state(0).cpu().numpy()
    Eg, _ = ctx.get_energy(0)
    tr = th.copy()                                     # swept in place by the oracle
    Er, br = oracle.sweeps(d, L, tr, a, lo, lo + width, [0, 1], E0.copy(), 1, 5, seed=SEED)
    assert np.array_equal(bits.astype(np.int64), br.astype(np.int64)), (bits, br)
    n_acc = sum(bin(int(b) & 0xff).count("1") for b in br[0])
    assert 0 < n_acc < 8 * n                           # both outcomes of the interval test
    assert np.median(circ_dist(got, th)) > 0.1         # the sweep moved the links
    dist = circ_dist(got, tr)
    print(f"\nL=32 FP64 sweep, tiles {tiles}: max angle difference {dist.max():.2e}, "
          f"links above 1e-12: {int(np.sum(dist > 1e-12))} of {dist.size}")
    assert np.mean(dist <= 1e-12) >= 0.99999
    assert dist.max() < 1e-10
    assert np.max(np.abs(Eg - Er) / np.abs(Er)) < 1e-9
    ctx.recompute_energy()
    Eg2, _ = ctx.get_energy(0)
    for k in range(n):
        assert abs(Eg2[k] - oracle.energy(d, L, tr[k])) < 1e-9 * abs(Er[k])
    flags, _ = ctx.health()
    assert flags.max() == 0
    ctx.close()


def test_largest_lattice_one_sweep_fp32(llr):
    import torch
    from tests.test_gpu_parity import _amplification, _oracle_sweep_f32_with_flags
    d, L = 4, 32
    th = random_state(d, L, 1, seed=3202, u_target=0.6, dtype=np.float32).astype(np.float64)
    E0 = oracle.energy(d, L, th[0])
    # as in the FP64 case: accepted first class passes, refused later ones,
    # every decision 1e4 or more from an edge, so that FP32 and the oracle
    # take the same decisions
    width = 0.05 * 6 * L ** 4
    lo = E0 - 0.1 * width
    ctx = llr.Context(precision=llr.FP32, device=0)
    ctx.set_params(seed=SEED)
    ctx.add_lattice(L, [lo], width)
    ctx.bind_state()
    ctx.set_a(0, np.array([1.0]))
    ctx.set_tiles(4, 2)
    ctx.import_state(0, torch.from_numpy(th.astype(np.float32)))
    bits = ctx.sweeps(1, sweep0=9)
    got = ctx.export_state(0).cpu().numpy().astype(np.float64)
    Eg, _ = ctx.get_energy(0)
    ctx.close()
    tr = th[0].copy()
    Er, flagged = _oracle_sweep_f32_with_flags(d, L, tr, 1.0, lo, lo + width, E0, 9)
    tb = np.ascontiguousarray(th.copy())
    _, br = oracle.sweeps(d, L, tb, [1.0], [lo], [lo + width], [0], [E0], 1, 9, seed=SEED, f32=True)
    assert int(bits[0, 0]) & 0xff == int(br[0, 0]) & 0xff
    assert 0 < bin(int(br[0, 0]) & 0xff).count("1") < 8
    amp = _amplification(d, L, th[0], lo, lo + width, E0, 9, n_dir=2)
    dist = circ_dist(got[0], tr)
    bar = 1e-6 * np.maximum(amp, 10.0)
    frac = np.mean(dist <= bar)
    n_div = int(np.sum(flagged & (dist > 1e-3)))
    print(f"\nL=32 FP32 sweep: {int(flagged.sum())} flagged links, median {np.median(dist):.2e}, "
          f"within bar {frac:.6f}, max {dist.max():.2e}, |dE| {abs(Eg[0] - Er):.3e}")
    assert np.median(dist) < 1e-6
    assert frac >= 0.999
    # energy: the full-size test's 0.1 at L = 20, scaled by the plaquette count
    assert abs(Eg[0] - Er) < 0.1 * (32 / 20) ** 4 + 12.0 * n_div


def test_most_intervals_driver_run_fp64(llr):
    import torch
    d, L, n = 4, 2, 4096
    th = random_state(d, L, n, seed=4096, u_target=0.6)
    E0 = np.array([oracle.energy(d, L, th[k]) for k in range(n)])
    order = np.argsort(E0)
    th, E0 = np.ascontiguousarray(th[order]), E0[order]
    assert np.all(np.diff(E0) > 0)
    # interval k centred on chain k's energy, the Robbins-Monro gain
    # 12 / ((n + 1) w^2) near that of the L = 4 driver test.  Two iterations
    # (four sweeps) stay inside the divergence horizon: over these 4096 L = 2
    # chains the largest |a_GPU - a_oracle| measured 0, 1e-14, 1e-10 at
    # n = 0, 1, 2 and 7e-7 at n = 3, with bits, labels and swaps identical
    # throughout (last-bit differences amplified ~100x per sweep by links of
    # small staple modulus, of which the many chains hold the extreme ones)
    dE = 30.0
    E_low = E0 - 0.5 * dE
    assert E_low[0] > -96.0 and E_low[-1] + dE < 96.0
    a0 = np.linspace(0.9, 1.1, n)
    ctx = llr.Context(precision=llr.FP64, device=0)
    ctx.set_params(seed=SEED, n_th=1, n_a=1, n_rm=2, recompute_every=2, replica_exchange=True)
    ctx.add_lattice(L, E_low, dE)
    ctx.bind_state()
    ctx.set_a(0, a0)
    ctx.enable_bits_log(100)
    ctx.import_state(0, torch.from_numpy(th.copy()))
    ctx.run()
    hist = ctx.get_history(0)
    a, it, _ = ctx.get_a(0)
    E, conf = ctx.get_energy(0)
    bits = ctx.get_bits_log()
    _, _, re_prop, re_acc = ctx.stats()
    r = oracle.llr_run(d, L, E_low, dE, a0, n_th=1, n_a=1, n_rm=2, seed=SEED, recompute_every=2,
                       replica_exchange=True, theta=th, record_bits=True, approach_cap=0)
    assert r["approach_sweeps"] == 0
    assert np.array_equal(bits.astype(np.int64), r["bits"].astype(np.int64))
    assert np.array_equal(conf, r["conf"])
    assert (re_prop, re_acc) == (int(r["re"][0]), int(r["re"][1]))
    assert re_acc > 1024                               # swaps beyond the first 1024 pairs' threads
    assert not np.array_equal(conf, np.arange(n))
    print(f"\n4096 intervals: max |a_GPU - a_oracle| per iteration "
          f"{np.abs(hist - r['a_hist']).max(axis=1)}, replica swaps {re_acc} of {re_prop}")
    assert np.max(np.abs(hist - r["a_hist"])) < 1e-7
    # energies after the fourth sweep: the worst of the 4096 chains measured
    # 1.1e-9 relative (its angles carry the amplified differences), the
    # median chain stays at the rounding level
    rel = np.abs(E - r["E"]) / np.abs(r["E"])
    assert np.median(rel) < 1e-12 and rel.max() < 1e-8
    assert np.array_equal(it, r["conv_iter"])
    ctx.close()
