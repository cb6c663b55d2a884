"""Writes the warm start's training set and the L=20 reference slopes (GPU).

The network a(u, 1/L) is trained on converged a_k that the method itself
produces (Sec. 2.4: initial values close to the result), so its training set
is this library's own output:

  train_ak.json  (u, 1/L, a_k) of
    * L=8: 32 intervals from u = 0.55, dE = 0.005 6V, mean of 4 independent
      runs (lattices of one context), N_TH 200, N_A 500, N_RM 50;
    * L=12 and 16: 64 intervals each over u in [0.58, 0.68], replica
      exchange, N_TH 200, N_A 1000, N_RM 100;
  aref_L20.json  long-run a_k of the full-pipeline interval set (L=20, 128
    intervals from u = 0.60, dE = 0.0005 6V, replica exchange, N_TH 500,
    N_A 2000), two independent runs of N_RM 60 from the network's warm start;
    their mean is the reference against which the benchmark times both
    starts, their difference its uncertainty.

All runs FP32 angles with FP64 energies, grouped sweep order.  The training
runs use seed 1509083910; the reference runs seeds 1509083910 + 101 and
+ 102, so that they share no random numbers with the benchmark's runs (seed
1509083910).  Usage (on a GPU), --reference-only to keep train_ak.json:
    python -m paper_1509_08391_amd.warmstart.make_data [--reference-only]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1509_08391_amd import experiments as ex  # noqa: E402
from paper_1509_08391_amd import llr  # noqa: E402

SEED = 1509083910
EPOCHS, LR = 4000, 3e-3
REF_SEEDS = (SEED + 101, SEED + 102)


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def training_points():
    pts = []
    L = 8
    V6 = 6 * L ** 4
    dE = 0.005 * V6
    E_low = 0.55 * V6 + dE * np.arange(32)
    res, meta = ex._run([(L, E_low, dE)] * 4, llr.FP32, 200, 500, 50, False, log=log)
    a8 = np.mean([r["a"] for r in res], axis=0)
    pts += [((e + 0.5 * dE) / V6, 1.0 / L, float(a)) for e, a in zip(E_low, a8)]
    lats = []
    for L in (12, 16):
        V6 = 6 * L ** 4
        dE = 0.1 / 64 * V6
        lats.append((L, 0.58 * V6 + dE * np.arange(64), dE))
    res, meta2 = ex._run(lats, llr.FP32, 200, 1000, 100, True, log=log)
    for (L, E_low, dE), r in zip(lats, res):
        V6 = 6 * L ** 4
        pts += [((e + 0.5 * dE) / V6, 1.0 / L, float(a)) for e, a in zip(E_low, r["a"])]
    return pts, [meta, meta2]


def train(pts):
    ctx = llr.Context(precision=llr.FP32, device=0)
    u = np.array([p[0] for p in pts])
    il = np.array([p[1] for p in pts])
    a = np.array([p[2] for p in pts])
    w0 = ctx.mlp_init(SEED)
    w, hist = ctx.mlp_train(w0, u, il, a, epochs=EPOCHS, lr=LR, bf16=True)
    rms = float(np.sqrt(np.mean((ctx.mlp_predict(w, u, il, bf16=True) - a) ** 2)))
    ctx.close()
    return w, rms


def reference(w, a_lo, a_hi, n_rm=60):
    L, E_low, dE = ex.l20_intervals()
    runs = []
    for k, seed in enumerate(REF_SEEDS):
        ctx = llr.Context(precision=llr.FP32, device=0)
        ctx.set_params(n_th=500, n_a=2000, n_rm=n_rm, seed=seed, replica_exchange=True, overlap=1.0,
                       recompute_every=10, eps=1e-4, approach_cap=20000)
        ctx.add_lattice(L, E_low, dE)
        ctx.bind_state()
        a0, nf = ctx.mlp_warm_start(0, w, a_lo, a_hi)
        ctx.hot_start()
        ctx.approach()
        ctx.rm_begin()
        t0 = time.perf_counter()
        for it in range(n_rm):
            ctx.rm_step(1)
            if it % 10 == 9:
                log(f"reference run {k}: RM iteration {it + 1}/{n_rm}, {time.perf_counter() - t0:.0f} s")
        a, conv, _ = ctx.get_a(0)
        runs.append(dict(seed=seed, a=a.tolist(), a0=a0.tolist(), fallbacks=nf,
                         a_hist_last11=ctx.get_history(0)[-11:].tolist()))
        ctx.close()
    A = np.array([r["a"] for r in runs])
    return dict(L=L, E_low=E_low.tolist(), dE=dE, n_th=500, n_a=2000, n_rm=n_rm, replica_exchange=True,
                a_ref=A.mean(0).tolist(), half_difference=(0.5 * np.abs(A[0] - A[1])).tolist(), runs=runs)


def main():
    path = os.path.join(HERE, "train_ak.json")
    if "--reference-only" in sys.argv[1:]:
        with open(path) as f:
            pts = [tuple(p) for p in json.load(f)["points"]]
        w, rms = train(pts)
    else:
        pts, metas = training_points()
        w, rms = train(pts)
        with open(path, "w") as f:
            json.dump(dict(points=pts, seed=SEED, epochs=EPOCHS, lr=LR, fit_rms=rms,
                           runs=[{k: m[k] for k in ("precision", "n_th", "n_a", "n_rm", "replica", "sweep_order")}
                                 for m in metas],
                           made_by="python -m paper_1509_08391_amd.warmstart.make_data"), f, indent=1)
    a = np.array([p[2] for p in pts])
    log(f"{len(pts)} training points, a in [{a.min():.5f}, {a.max():.5f}], fit rms {rms:.2e}")
    margin = 0.1 * (a.max() - a.min())
    ref = reference(w, a.min() - margin, a.max() + margin)
    hd = np.array(ref["half_difference"])
    log(f"reference a_k: two runs differ by at most {2 * hd.max():.2e} (median {2 * np.median(hd):.2e})")
    ref["made_by"] = "python -m paper_1509_08391_amd.warmstart.make_data"
    with open(os.path.join(HERE, "aref_L20.json"), "w") as f:
        json.dump(ref, f)


if __name__ == "__main__":
    main()
