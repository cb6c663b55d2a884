"""Checkpoint and restore of Algorithm 1's state through the C ABI: a run
interrupted after N sweeps, saved, restored into a fresh context and
continued for N more sweeps is the uninterrupted 2N-sweep run bit for bit
(angles, accept bits, chain <-> interval labels, a^(n), energies, counters,
the work counts of llr_get_rates)."""
import numpy as np
import pytest

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


def _setup(llr, prec, order):
    ctx = llr.Context(precision=prec, device=0)
    ctx.set_params(n_th=3, n_a=4, n_rm=4, seed=SEED, replica_exchange=True, overlap=1.0, recompute_every=3,
                   approach_cap=4000)
    for L, n, u0 in [(4, 6, 0.56), (6, 4, 0.60)]:
        V6 = 6 * L ** 4
        dE = 0.01 * V6
        ctx.add_lattice(L, u0 * V6 + dE * np.arange(n), dE)
    ctx.bind_state()
    ctx.set_a(0, np.linspace(0.95, 1.05, 6))
    ctx.set_a(1, np.linspace(0.98, 1.02, 4))
    ctx.set_sweep_order(order)
    ctx.hot_start()
    return ctx


def _snapshot(ctx):
    out = {}
    for i in range(len(ctx.lattices)):
        out[f"theta{i}"] = ctx.export_state(i).cpu().numpy()
        out[f"E{i}"], out[f"conf{i}"] = ctx.get_energy(i)
        out[f"a{i}"], out[f"it{i}"], out[f"sw{i}"] = ctx.get_a(i)
        out[f"hist{i}"] = ctx.get_history(i)
    hp, ha, rp, ra = ctx.stats()
    out["hp"], out["ha"], out["re"] = hp, ha, np.array([rp, ra])
    r = ctx.rates()
    out["rates"] = np.array([r[k] for k in ("sweeps", "hb_class_passes", "hb_class_accepts", "or_class_passes",
                                            "or_class_relabelled", "re_proposals", "re_accepts", "link_updates")])
    return out


@pytest.mark.parametrize("prec,order", [("FP64", 0), ("FP32", 0), ("FP32", 1), ("FP64", 2), ("FP32", 2)])
def test_restore_continues_bit_for_bit(llr, prec, order, tmp_path):
    p = getattr(llr, prec)
    path = str(tmp_path / "run.ckpt")
    # reference: approach, then 4 Robbins-Monro iterations uninterrupted
    ref = _setup(llr, p, order)
    ref.approach()
    ref.rm_begin()
    ref.rm_step(2)
    ref.checkpoint(path)
    ref.enable_bits_log(64)
    ref.rm_step(2)
    want = _snapshot(ref)
    want_bits = ref.get_bits_log()
    ref.close()
    # a fresh context built from the file alone continues the run
    ctx = llr.Context.from_checkpoint(path)
    assert ctx.precision == p
    ctx.enable_bits_log(64)
    ctx.rm_step(2)
    got = _snapshot(ctx)
    got_bits = ctx.get_bits_log()
    ctx.close()
    assert got_bits.shape == want_bits.shape and want_bits.shape[0] == 2 * 7
    assert np.array_equal(got_bits, want_bits)
    for k in want:
        assert np.array_equal(got[k], want[k]), k


def test_restore_rejects_other_lattice_sets(llr, tmp_path):
    path = str(tmp_path / "a.ckpt")
    ctx = _setup(llr, llr.FP32, 0)
    ctx.checkpoint(path)
    ctx.close()
    other = llr.Context(precision=llr.FP32, device=0)
    other.set_params(seed=SEED)
    other.add_lattice(4, 0.56 * 6 * 256 + 15.36 * np.arange(6), 15.36)
    other.bind_state()
    with pytest.raises(llr.LLRError):
        other.restore(path)
    other.close()
    wrong_prec = llr.Context(precision=llr.FP64, device=0)
    info = llr.checkpoint_info(path)
    for L, E_low, dE in info["lattices"]:
        wrong_prec.add_lattice(L, E_low, dE)
    wrong_prec.bind_state()
    with pytest.raises(llr.LLRError):
        wrong_prec.restore(path)
    wrong_prec.close()


def test_checkpoint_during_the_approach(llr, tmp_path):
    """A checkpoint taken between two llr_approach_continue calls: the restored
    context finishes the approach and the Robbins-Monro iterations exactly as
    the uninterrupted one (approach counters, per-colour couplings and steps
    of the approach rule, and the open approach are part of the state)."""
    path = str(tmp_path / "ap.ckpt")
    ref = _setup(llr, llr.FP32, 0)
    ref.approach_begin()
    ref.approach_continue(3)
    ref.checkpoint(path)
    s_ref, done_ref = ref.approach_continue(4000)
    ref.rm_begin()
    ref.rm_step(1)
    want = _snapshot(ref)
    ref.close()
    ctx = llr.Context.from_checkpoint(path)
    s_got, done_got = ctx.approach_continue(4000)
    ctx.rm_begin()
    ctx.rm_step(1)
    got = _snapshot(ctx)
    ctx.close()
    assert done_ref and done_got and np.array_equal(s_ref, s_got)
    for k in want:
        assert np.array_equal(got[k], want[k]), k
