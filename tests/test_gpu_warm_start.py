"""What the learned warm start gains (Sec. 2.4: the Robbins-Monro recursion of
eq. (kk21) from an initial a_i close to the result, here from the network
a(u, 1/L) trained on converged a_k that the method itself produced).

The method produces converged a_k at L = 6, 8 and 10 (one batched context,
a^(0) = 1).  The network is trained on them with the library's kernels and
predicts a_k at L = 12, a size it never saw.  Robbins-Monro at L = 12 then
runs from the prediction and from a^(0) = 1 with the same seed.

Why it pays: eq. (kk19)'s variance dE^2/12 holds only while dE |a - a*| is
small.  Far from the root the restricted distribution piles up at one edge,
<E> - c saturates at +-w/2, and each step moves a by at most 6/((n+1) w): a
harmonic series.  At L = 12 (w = 933) a cold start from 1 therefore takes
several iterations per interval (measured: 6.5 on average, one interval not
within 16), while a start inside the linear range needs the Newton step and
then the recursion's noise (measured: 3.4).  The network extrapolates in 1/L
here, and is least accurate at the ordered-phase end of the interval set
(u ~ 0.67, errors up to 5e-3), so the bar is set on the typical interval and
on the total.  At L = 20 with 128 intervals the same comparison gives 4.3x
fewer sweeps."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SEED = 1509083910
U0, NK, DU = 0.56, 16, 0.0075     # intervals: u in [0.56, 0.68], dE = 0.0075 6V


@pytest.fixture(scope="module")
def llr():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1509_08391_amd import llr as m
    m.lib()
    return m


def _intervals(L):
    V6 = 6 * L ** 4
    dE = DU * V6
    return V6, U0 * V6 + dE * np.arange(NK), dE


def _run(llr, Ls, a0, n_rm, seed, eps):
    ctx = llr.Context(precision=llr.FP32, device=0)
    ctx.set_params(n_th=100, n_a=400, n_rm=n_rm, seed=seed, replica_exchange=False, recompute_every=10,
                   eps=eps, approach_cap=20000)
    for L in Ls:
        _, E_low, dE = _intervals(L)
        ctx.add_lattice(L, E_low, dE)
    ctx.bind_state()
    for i in range(len(Ls)):
        ctx.set_a(i, a0[i])
    ctx.hot_start()
    ctx.approach()
    ctx.run()
    out = [ctx.get_a(i) for i in range(len(Ls))]
    hist = [ctx.get_history(i) for i in range(len(Ls))]
    ctx.close()
    return out, hist


def test_mlp_warm_start_converges_in_fewer_sweeps(llr):
    eps = 2.5e-4
    # converged a_k at L = 6, 8, 10 from a^(0) = 1
    sizes = [6, 8, 10]
    train, _ = _run(llr, sizes, [1.0] * len(sizes), 24, SEED + 1, eps)
    u, il, a = [], [], []
    for L, (ak, _, _) in zip(sizes, train):
        V6, E_low, dE = _intervals(L)
        u.append((E_low + 0.5 * dE) / V6)
        il.append(np.full(NK, 1.0 / L))
        a.append(ak)
    u, il, a = np.concatenate(u), np.concatenate(il), np.concatenate(a)
    assert np.all(np.abs(a - 1.0) < 0.2)

    ctx = llr.Context(precision=llr.FP32, device=0)
    w, hist = ctx.mlp_train(ctx.mlp_init(SEED), u, il, a, epochs=3000, lr=3e-3, bf16=True)
    assert hist[-1] < 0.05 * hist[0]
    V6, E_low, dE = _intervals(12)
    u12 = (E_low + 0.5 * dE) / V6
    a_pred = ctx.mlp_predict(w, u12, np.full(NK, 1.0 / 12), bf16=True)
    ctx.close()

    n_rm = 16
    (cold, ), _ = _run(llr, [12], [1.0], n_rm, SEED, eps)
    (warm, ), _ = _run(llr, [12], [a_pred], n_rm, SEED, eps)
    ic = np.where(cold[1] < 0, n_rm, cold[1])
    iw = np.where(warm[1] < 0, n_rm, warm[1])
    sweeps = 500
    print(f"\nL=12, {NK} intervals, eps {eps}: RM sweeps to |da| < eps summed over intervals: "
          f"cold {int(np.sum(ic + 1) * sweeps)}, warm {int(np.sum(iw + 1) * sweeps)}; "
          f"cold not converged in {int(np.sum(cold[1] < 0))}; prediction - warm result rms "
          f"{np.sqrt(np.mean((a_pred - warm[0]) ** 2)):.2e}")
    # the warm start converges everywhere ...
    assert np.all(warm[1] >= 0)
    # ... the typical interval's prediction lies inside the Newton step's linear range ...
    assert np.median(np.abs(a_pred - warm[0])) * dE < 1.0
    # ... and the whole set needs far fewer sweeps than the cold start
    assert np.sum(iw + 1) < 0.75 * np.sum(ic + 1)
    # where the cold start converged, the typical interval agrees within the
    # recursion's noise (at the top of the set the cold start's stopping rule
    # fires while a_k is still 1.5e-3 - 4.5e-3 short of the root: its steps
    # have shrunk as 1/(n+1) before it got there)
    both = cold[1] >= 0
    assert both.sum() >= NK // 2
    assert np.median(np.abs(cold[0][both] - warm[0][both])) < 1.5e-3


@pytest.mark.parametrize("bf16", [True, False])
def test_warm_start_sets_predictions_and_falls_back(llr, bf16):
    """llr_mlp_warm_start (Sec. 2.4's initial a_i, with plain Robbins-Monro
    kept as the fallback): with a range that holds every prediction, a_k^(0)
    is the network's prediction at the interval centres u = c_k/(6V), 1/L,
    bit for bit as llr_mlp_predict gives it; predictions outside
    [a_min, a_max] and non-finite ones are replaced by the cold start
    a^(0) = 1 and counted; an empty range is an argument error."""
    L, n = 8, 24
    V6 = 6 * L ** 4
    dE = 0.005 * V6
    E_low = 0.55 * V6 + dE * np.arange(n)
    ctx = llr.Context(precision=llr.FP32, device=0)
    ctx.set_params(seed=SEED)
    ctx.add_lattice(L, E_low, dE)
    ctx.bind_state()
    w = ctx.mlp_init(7)
    u = ((E_low + 0.5 * dE) / V6).astype(np.float32)
    pred = ctx.mlp_predict(w, u, np.full(n, 1.0 / L, dtype=np.float32), bf16=bf16)
    assert np.all(np.isfinite(pred)) and np.ptp(pred) > 0
    a0, nf = ctx.mlp_warm_start(0, w, pred.min() - 1.0, pred.max() + 1.0, bf16=bf16)
    assert nf == 0 and np.array_equal(a0, pred)
    assert np.array_equal(ctx.get_a(0)[0], pred)
    lo, hi = np.quantile(pred, [0.25, 0.75])
    a0, nf = ctx.mlp_warm_start(0, w, lo, hi, bf16=bf16)
    out = (pred < lo) | (pred > hi)
    assert nf == int(out.sum()) > 0
    assert np.all(a0[out] == 1.0) and np.array_equal(a0[~out], pred[~out])
    assert np.array_equal(ctx.get_a(0)[0], a0)
    w_bad = w.copy()
    w_bad[:] = np.nan
    a0, nf = ctx.mlp_warm_start(0, w_bad, pred.min() - 1.0, pred.max() + 1.0, bf16=bf16)
    assert nf == n and np.all(a0 == 1.0)
    with pytest.raises(llr.LLRError):
        ctx.mlp_warm_start(0, w, 1.1, 0.9, bf16=bf16)
    ctx.close()
