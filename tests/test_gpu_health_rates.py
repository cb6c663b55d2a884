"""Work accounting (llr_get_rates) and runtime health tests (llr_health)
through the C ABI.

Rates: the link updates the library reports are the heatbath class passes
(every chain, V/2 links each, approach included) plus the overrelaxation
class passes, less, in the interleaved order, the overrelaxations fused after
an accepted heatbath of their class (relabelled draws); checked against the
acceptance counters of llr_stats in both orders.

Health: a clean run raises no flag and its recompute drift stays far below
the bound; a non-finite angle, an incremental E that no longer matches the
angles, and a chain whose E left its restriction each raise their flag at the
next recompute, the call returns LLR_ENUMERIC, and clearing resets the flags.
Faults are planted in the caller-owned state from the host side (values
only; every kernel runs to completion on finite or non-finite data)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SEED = 1509083912


@pytest.fixture(scope="module")
def llr():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1509_08391_amd import llr as m
    m.lib()
    return m


def _ctx(llr, prec, order, L=4, n=6, replica=False, K=5):
    ctx = llr.Context(precision=prec, device=0)
    ctx.set_params(n_th=2, n_a=3, n_rm=4, seed=SEED, replica_exchange=replica, overlap=1.0, recompute_every=K,
                   approach_cap=4000)
    V6 = 6 * L ** 4
    dE = 0.01 * V6
    ctx.add_lattice(L, 0.57 * V6 + dE * np.arange(n), dE)
    ctx.bind_state()
    ctx.set_a(0, 1.0)
    ctx.set_sweep_order(order)
    ctx.hot_start()
    ctx.approach()
    return ctx


@pytest.mark.parametrize("order", [0, 1, 2])
@pytest.mark.parametrize("prec", ["FP64", "FP32"])
def test_link_updates_follow_the_acceptance_counters(llr, prec, order):
    L, n = 4, 6
    half = L ** 4 // 2
    ctx = _ctx(llr, getattr(llr, prec), order, L, n)
    r0 = ctx.rates()
    hp0, ha0, _, _ = ctx.stats()
    assert r0["sweeps"] == 0 and r0["or_class_passes"] == 0 and r0["or_class_relabelled"] == 0
    # approach: heatbath passes only
    assert r0["link_updates"] == half * hp0.sum()
    nsw = 7
    ctx.sweeps(nsw, sweep0=100, mode=llr.MODE_RESTRICTED, want_bits=False)
    r = ctx.rates()
    hp, ha, _, _ = ctx.stats()
    assert r["sweeps"] == nsw
    assert r["or_class_passes"] == 8 * nsw * n
    assert r["hb_class_passes"] == hp.sum() and r["hb_class_accepts"] == ha.sum()
    assert (hp - hp0).sum() == 8 * nsw * n
    relabelled = (ha - ha0).sum() if order == 1 else 0
    assert r["or_class_relabelled"] == relabelled
    assert r["link_updates"] == half * (hp.sum() + 8 * nsw * n - relabelled)
    assert r["or_acceptance"] == 1.0
    assert r["seconds"] > 0 and r["link_updates_per_s"] == pytest.approx(r["link_updates"] / r["seconds"])
    ctx.close()


@pytest.mark.parametrize("prec,bound", [("FP64", 1e-9), ("FP32", 1e-5)])
def test_clean_run_raises_no_flag(llr, prec, bound):
    L = 6
    ctx = _ctx(llr, getattr(llr, prec), 0, L=L, n=4, replica=True, K=3)
    ctx.rm_begin()
    ctx.rm_step(2)
    f, d = ctx.health()
    ctx.close()
    print(f"\n{prec}: largest recompute drift {d.max():.3e} (bound {bound * 6 * L ** 4:.3e})")
    assert not f.any()
    assert d.max() < 0.05 * bound * 6 * L ** 4


def test_non_finite_angle_is_flagged(llr):
    ctx = _ctx(llr, llr.FP64, 0)
    th = ctx.export_state(0)
    th[2, 1, 17] = float("nan")
    ctx.import_state(0, th)   # the import's own recompute applies no test
    with pytest.raises(llr.LLRNumericError):
        ctx.recompute_energy()
    f, _ = ctx.health()
    assert f[2] & 1 and not np.delete(f, 2).any()
    f, _ = ctx.health(clear=True)
    f, _ = ctx.health()
    assert not f.any()
    ctx.close()


def test_drift_and_restriction_flags(llr):
    L, n = 4, 6
    ctx = _ctx(llr, llr.FP64, 0, L, n, K=1)
    # change chain 3's angles behind the library's back: its incremental E
    # no longer matches them (each chain holds 2 x 4V angles)
    st = ctx.state
    per = 8 * L ** 4
    st[3 * per:4 * per] *= 0.5
    with pytest.raises(llr.LLRNumericError):
        ctx.recompute_energy()
    f, d = ctx.health()
    assert f[3] == 2 and not np.delete(f, 3).any() and d[3] > 1.0
    # the recompute has taken the new E; it lies far outside chain 3's
    # restriction, which the restricted sweeps' recompute reports
    ctx.health(clear=True)
    ctx.rm_begin()
    with pytest.raises(llr.LLRNumericError):
        ctx.rm_step(1)
    f, _ = ctx.health(clear=True)
    assert f[3] & 4 and not np.delete(f, 3).any()
    ctx.close()
