"""Runs of Algorithm 1 on the configurations the method is measured on.

  l8        L=8, 32 intervals from u = 0.55, dE = 0.005 6V, N_TH = 200,
           N_A = 500, N_RM = 50, a^(0) = 1; once in FP64 and once with FP32
           angles; <u>(beta), C_V(beta) on beta in [0.98, 1.04].
  batched   L = 12, 16, 20 batched in one launch, 64 intervals each over
           u in [0.58, 0.68], replica exchange after every sweep, FP32,
           N_TH = 200, N_A = 1000, N_RM = 100.
  warmstart warm start: the network a(u, 1/L) trained on the converged a_k of
           l8 (L=8) and batched (L=12, 16), predicting the L=20 interval
           set of l20; Robbins-Monro from the prediction and from
           a^(0) = 1, compared by the sweeps until |a^(n+1) - a^(n)| < 1e-4.
  l20       L = 20, 128 intervals from u = 0.60, dE = 0.0005 6V, warm start,
           replica exchange, FP32, N_TH = 500, N_A = 2000, N_RM = 100;
           ln rho, C_V(beta) on beta in [1.008, 1.012], beta_c and peak.

  l20reps   N_B = 8 independent repetitions of l20 (eight lattices of one
           context; the lattice index enters every random counter), warm
           start, N_RM = 25: bootstrap errors of beta_c and the C_V peak
           (Sec. 2.4, Sec. 3.2), and the two peaks of P_beta(E) at beta_c.

  muca12   multicanonical sampling at L = 12 with W = 1/rho~ from the
           converged L=12 a_k of batched (Sec. 2.6): 64 chains, flatness of
           the energy histogram, tunnellings between the ends of the range,
           and <u>(beta) by reweighting (eq. (4.7)) next to the LLR
           reconstruction from the same a_k.

  dE8      the delta E study of Sec. 3.5 at L = 8: the l8 range
           u in [0.55, 0.71] cut into 16, 32, 64 and 128 intervals, eight
           replicas each, FP32; the C_V peak against delta E and the fit
           C_V(dE) = C_V(0) + 6V b_dis dE^2.
  dE12     the same at L = 12 with 8, 16, 32, 64 and 128 intervals.

  obs8     a non-action observable through restricted double brackets
           (Sec. 2.3): after an L=8 run with l8's dE over u in
           [0.50, 0.71] (42 intervals, FP32), 400 restricted
           measurements per interval of E and sum_P cos 2 theta_P;
           <u>(beta) and <cos 2 theta_P>(beta) on [0.98, 1.04] by eqs.
           (l9)-(l10), next to direct canonical runs at beta = 0.98, 1.04.

  l20parts  l20 repeated: part p runs two independent replicas as two
           lattices of one context (seed SEED + 1000 p) with the warm start
           and N_RM = 100;
           "l20parts --combine" bootstraps beta_c and the C_V peak over all
           parts' runs and locates the peaks of P_beta(E) at beta_c.

  linkcmp  the restriction imposed per link when each angle is drawn
           (Sec. 2.4) against class-wise rejection, FP32, no replica
           exchange, from one thermalised state per lattice: ms per sweep,
           the integrated autocorrelation time of E per interval, class
           acceptance, links re-drawn per class pass.  L = 8 (l8's
           intervals, a_k from a 20-iteration run) and L = 20 (l20's
           intervals, a_k of a converged run from an l20parts_part0.json
           under --inputs, else a_k = 1.011 ~ beta_c(20) throughout).
  linkprof 60 sweeps per mode of the L = 20 set only, for a kernel trace.

  ordercmp the grouped and the interleaved order of a sweep's class
           passes (the latter with fused launches) on the lattices and a_k of
           linkcmp, 8000 sweeps each: mean E per interval against a second
           grouped run with other random numbers.

  --order  grouped (default), interleaved or staggered: the sweep order
           of the Algorithm 1 runs of every configuration.
  --jsonl  a file to which every Robbins-Monro iteration of those runs
           appends one JSON line: a_k and max |a^(n+1) - a^(n)| per lattice,
           acceptance rates, link updates and updates/s so far, the largest
           recompute drift and the chains the health tests flagged.

  batchprof the batched lattice set (L = 12, 16, 20, 64 intervals each, one
           launch per class pass for all three), FP32, replica exchange,
           a_k = 1: hot start, approach, autotune, then 200 restricted sweeps
           timed; for a kernel trace of the batched launch.

  fss      beta_c(L) and the C_V peak for the finite-size analysis of Sec. 3.4
           on this implementation's own runs: L = 8, 10, 12, 14 (part 0) and
           16, 18 (part 1), 96 intervals over u in [0.56, 0.70], four replicas
           each (lattices of one context), replica exchange, FP32,
           N_TH = 200, N_A = 800, N_RM = 80, warm start from the network of
           warmstart evaluated at (u, 1/L); per L a bootstrap over the replicas.
           "fss --combine" adds L = 20 from the l20parts parts and fits
           beta_c(L) = beta_c + sum_k B_k L^-4k and C_V/(6V) = G^2/4 + ...

Each writes a JSON record.  Usage:
    python -m paper_1509_08391_amd.experiments l8 [--out DIR]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import llr

SEED = 1509083910
_ORDER_NAMES = {llr.SWEEP_GROUPED: "grouped", llr.SWEEP_INTERLEAVED: "interleaved",
                llr.SWEEP_STAGGERED: "staggered"}
# order of the class passes in the sweeps of _run (command-line --order)
SWEEP_ORDER = llr.SWEEP_GROUPED
# JSON-lines record of every Robbins-Monro iteration of _run (command-line
# --jsonl), None for none
JSONL = None


def _iteration_record(ctx, lattices, it, a_prev, t):
    """One line of the per-iteration record: per lattice a_k and the largest
    |a^(n+1) - a^(n)|; acceptance rates, link updates and their rate so far
    (llr_get_rates); the largest drift of the incremental energy at a
    recompute and the chains the health tests flagged (llr_health)."""
    r = ctx.rates()
    flags, drift = ctx.health()
    lats = []
    for i in range(len(lattices)):
        a = ctx.get_a(i)[0]
        lats.append(dict(L=lattices[i][0], a=a.tolist(), max_da=float(np.max(np.abs(a - a_prev[i])))))
        a_prev[i] = a
    return dict(iteration=it + 1, seconds=t, lattices=lats, hb_acceptance=r["hb_acceptance"],
                re_acceptance=r["re_acceptance"], or_acceptance=r["or_acceptance"], sweeps=r["sweeps"],
                link_updates=r["link_updates"], link_updates_per_s=r["link_updates_per_s"],
                max_recompute_drift=float(drift.max()), chains_flagged=int(np.count_nonzero(flags)))


def _updates_per_class_link(ctx, before):
    """Link updates per class link and class pass since the stats() snapshot
    `before`: 2 in the grouped and staggered orders (one heatbath, one
    overrelaxation); in
    the interleaved order the overrelaxation right after an accepted heatbath
    of its class is a relabelled draw, so 1 for an accepted class and 2 (the
    rejected proposal and one overrelaxation) for a rejected one."""
    if SWEEP_ORDER != llr.SWEEP_INTERLEAVED:
        return 2.0
    hp, ha, _, _ = ctx.stats()
    passes = float((hp - before[0]).sum())
    return 2.0 - (float((ha - before[1]).sum()) / passes if passes > 0 else 0.0)


def _run(lattices, prec, n_th, n_a, n_rm, replica, seed=SEED, a0=None, log=None, eps=1e-4):
    """lattices: list of (L, E_low, dE).  a0: list of per-lattice arrays or None."""
    ctx = llr.Context(precision=prec, device=0)
    ctx.set_params(n_th=n_th, n_a=n_a, n_rm=n_rm, seed=seed, replica_exchange=replica, overlap=1.0,
                   recompute_every=10, eps=eps, approach_cap=20000)
    ctx.set_sweep_order(SWEEP_ORDER)
    for (L, E_low, dE) in lattices:
        ctx.add_lattice(L, E_low, dE)
    ctx.bind_state()
    for i, (L, E_low, dE) in enumerate(lattices):
        ctx.set_a(i, 1.0 if a0 is None else a0[i])
    t0 = time.perf_counter()
    ctx.hot_start()
    ctx.approach_begin()
    done = False
    while not done:
        ap, done = ctx.approach_continue(100)
        if ap.max() >= 20000:
            raise RuntimeError("approach did not finish")
    t_ap = time.perf_counter() - t0
    tiles = ctx.autotune()
    ctx.rm_begin()
    st0 = ctx.stats()
    jl = open(JSONL, "a") if JSONL else None
    a_prev = [ctx.get_a(i)[0] for i in range(len(lattices))]
    t1 = time.perf_counter()
    t_log = t1
    for it in range(n_rm):
        ctx.rm_step(1)
        now = time.perf_counter()
        if jl:
            jl.write(json.dumps(_iteration_record(ctx, lattices, it, a_prev, now - t1)) + "\n")
            jl.flush()
        if log and (now - t_log > 20.0 or it == n_rm - 1):
            log(f"RM iteration {it + 1}/{n_rm}, {now - t1:.1f} s")
            t_log = now
    t_rm = time.perf_counter() - t1
    if jl:
        jl.close()
    per_link = _updates_per_class_link(ctx, st0)
    out = []
    for i, (L, E_low, dE) in enumerate(lattices):
        a, conv, sw = ctx.get_a(i)
        hist = ctx.get_history(i)
        E, conf = ctx.get_energy(i)
        out.append(dict(L=L, E_low=np.asarray(E_low).tolist(), dE=dE, a=a.tolist(), conv_iter=conv.tolist(),
                        conv_sweeps=sw.tolist(), a_hist=hist.tolist(), approach_sweeps=int(ap[i]),
                        E=E.tolist()))
    hp, ha, rp, ra = ctx.stats()
    nsw = n_th + n_a
    upd = sum(per_link * 4 * L ** 4 * len(E_low) for (L, E_low, dE) in lattices) * nsw * n_rm
    meta = dict(precision="fp32" if prec == llr.FP32 else "fp64", n_th=n_th, n_a=n_a, n_rm=n_rm, replica=replica,
                sweep_order=_ORDER_NAMES[SWEEP_ORDER],
                seed=seed, seconds_approach=t_ap, seconds_rm=t_rm, updates_per_s=upd / t_rm, tiles=list(tiles),
                hb_acceptance=float(ha.sum() / max(hp.sum(), 1)),
                re_acceptance=float(ra / max(rp, 1)) if replica else None)
    ctx.close()
    return out, meta


def _reconstruct(L, E_low, dE, a, blo, bhi, nb=61):
    ctx = llr.Context(precision=llr.FP64, device=0)
    V6 = 6 * L ** 4
    cen = np.asarray(E_low) + 0.5 * dE
    beta = np.linspace(blo, bhi, nb)
    lr, u, cv = ctx.reconstruct(cen, a, dE, V6, beta)
    bc, pk = ctx.beta_c(cen, a, dE, V6, blo, bhi, h=1e-5, tol=1e-9)
    ctx.close()
    return dict(beta=beta.tolist(), u_mean=u.tolist(), cv=cv.tolist(), ln_rho=lr.tolist(), beta_c=bc,
                cv_peak=pk, cv_peak_over_6v=pk / V6)


def run_l8(log, replicas=8):
    """The L=8 interval set as `replicas` independent lattices of one context
    (the lattice index enters every random counter), in FP64 and in FP32."""
    L = 8
    V6 = 6 * L ** 4
    dE = 0.005 * V6
    E_low = 0.55 * V6 + dE * np.arange(32)
    rec = {}
    for prec in (llr.FP64, llr.FP32):
        res, meta = _run([(L, E_low, dE)] * replicas, prec, 200, 500, 50, False, log=log)
        for r in res:
            r.update(_reconstruct(L, E_low, dE, np.array(r["a"]), 0.98, 1.04))
        rec[meta["precision"]] = dict(results=res, meta=meta)
        a = np.array([r["a"] for r in res])
        bc = np.array([r["beta_c"] for r in res])
        pk = np.array([r["cv_peak_over_6v"] for r in res])
        log(f"{meta['precision']}: a_k spread (std over replicas) max {a.std(0, ddof=1).max():.2e}; "
            f"beta_c {bc.mean():.6f} +- {bc.std(ddof=1) / np.sqrt(len(bc)):.6f}; "
            f"C_V/(6V) peak {pk.mean():.3e} +- {pk.std(ddof=1) / np.sqrt(len(pk)):.1e}; "
            f"{meta['updates_per_s']:.3e} updates/s")
    return rec


def run_batched(log):
    lats = []
    for L in (12, 16, 20):
        V6 = 6 * L ** 4
        dE = 0.1 / 64 * V6
        lats.append((L, 0.58 * V6 + dE * np.arange(64), dE))
    res, meta = _run(lats, llr.FP32, 200, 1000, 100, True, log=log)
    for r in res:
        r.update(_reconstruct(r["L"], r["E_low"], r["dE"], np.array(r["a"]), 0.98, 1.04))
    return dict(results=res, meta=meta)


def l20_intervals():
    L = 20
    V6 = 6 * L ** 4
    dE = 0.0005 * V6
    return L, 0.60 * V6 + dE * np.arange(128), dE


def train_network(points, epochs=4000, lr=3e-3, seed=SEED):
    """points: list of (u, 1/L, a).  Trained on the GPU with the library's
    kernels (BF16 MFMA forward, FP32 backward, Adam)."""
    ctx = llr.Context(precision=llr.FP32, device=0)
    u = np.array([p[0] for p in points])
    il = np.array([p[1] for p in points])
    a = np.array([p[2] for p in points])
    w0 = ctx.mlp_init(seed)
    w, hist = ctx.mlp_train(w0, u, il, a, epochs=epochs, lr=lr, bf16=True)
    pred = ctx.mlp_predict(w, u, il, bf16=True)
    ctx.close()
    return w, hist, float(np.sqrt(np.mean((pred - a) ** 2)))


def run_warmstart(log, c1, c2, n_rm=20):
    pts = []
    r1 = c1["fp64"]["results"]
    a8 = np.mean([r["a"] for r in r1], axis=0)
    V6 = 6 * 8 ** 4
    for e, a in zip(r1[0]["E_low"], a8):
        pts.append(((e + 0.5 * r1[0]["dE"]) / V6, 1.0 / 8, a))
    for r in c2["results"]:
        if r["L"] in (12, 16):
            V6 = 6 * r["L"] ** 4
            for e, a in zip(r["E_low"], r["a"]):
                pts.append(((e + 0.5 * r["dE"]) / V6, 1.0 / r["L"], a))
    w, hist, rms = train_network(pts)
    L, E_low, dE = l20_intervals()
    V6 = 6 * L ** 4
    u20 = (E_low + 0.5 * dE) / V6
    ctx = llr.Context(precision=llr.FP32, device=0)
    a_mlp = ctx.mlp_predict(w, u20, np.full(u20.size, 1.0 / L), bf16=True)
    ctx.close()
    log(f"network trained on {len(pts)} points, fit rms {rms:.2e}; prediction range "
        f"{a_mlp.min():.4f}..{a_mlp.max():.4f}")
    runs = {}
    for name, a0 in (("cold", np.full(128, 1.0)), ("mlp", a_mlp)):
        res, meta = _run([(L, E_low, dE)], llr.FP32, 500, 2000, n_rm, True, a0=[a0], log=log)
        runs[name] = dict(result=res[0], meta=meta)
    return dict(training_points=len(pts), fit_rms=rms, loss_hist=hist[::100].tolist(), weights=w.tolist(),
                a_mlp=a_mlp.tolist(), runs=runs, n_rm=n_rm)


def run_l20(log, c3, n_rm=100):
    L, E_low, dE = l20_intervals()
    a0 = np.array(c3["a_mlp"])
    res, meta = _run([(L, E_low, dE)], llr.FP32, 500, 2000, n_rm, True, a0=[a0], log=log)
    r = res[0]
    r.update(_reconstruct(L, E_low, dE, np.array(r["a"]), 1.008, 1.012, nb=41))
    return dict(result=r, meta=meta)


def l20_replicas(log, c3, n_rep=8, n_rm=25, n_boot=1000):
    L, E_low, dE = l20_intervals()
    V6 = 6 * L ** 4
    a0 = np.array(c3["a_mlp"])
    res, meta = _run([(L, E_low, dE)] * n_rep, llr.FP32, 500, 2000, n_rm, True, a0=[a0] * n_rep, log=log)
    A = np.array([r["a"] for r in res])
    cen = E_low + 0.5 * dE
    ctx = llr.Context(precision=llr.FP64, device=0)
    per = [ctx.beta_c(cen, A[i], dE, V6, 1.008, 1.012, h=1e-5, tol=1e-9) for i in range(n_rep)]
    bc_b, pk_b = ctx.bootstrap(cen, A, dE, V6, 1.008, 1.012, n_boot=n_boot, seed=SEED)
    abar = A.mean(axis=0)
    bc, pk = ctx.beta_c(cen, abar, dE, V6, 1.008, 1.012, h=1e-5, tol=1e-9)
    Ep, lp = ctx.prob_peaks(cen, abar, dE, bc)
    # peaks of every bootstrap-free replica for their spread
    Ep_rep = []
    for i in range(n_rep):
        bci = per[i][0]
        e, l = ctx.prob_peaks(cen, A[i], dE, bci)
        Ep_rep.append(sorted(e[np.argsort(l)[-2:]].tolist()) if e.size >= 2 else [])
    Egrid = np.linspace(E_low[0], E_low[-1] + dE, 801)
    logp = ctx.prob_density(cen, abar, dE, bc, Egrid)
    ctx.close()
    two = sorted(Ep[np.argsort(lp)[-2:]].tolist()) if Ep.size >= 2 else Ep.tolist()
    log(f"beta_c {bc:.7f} +- {bc_b.std(ddof=1):.7f} (bootstrap, {n_boot} samples of {n_rep} runs); "
        f"C_V/(6V) {pk / V6:.4e} +- {pk_b.std(ddof=1) / V6:.1e}; peaks of P at beta_c: "
        f"{[round(e / V6, 5) for e in two]}")
    return dict(a_runs=A.tolist(), per_run=[list(p) for p in per], beta_c=bc, cv_peak=pk, cv_peak_over_6v=pk / V6,
                boot_beta_c=bc_b.tolist(), boot_cv_peak=pk_b.tolist(), beta_c_err=float(bc_b.std(ddof=1)),
                cv_peak_over_6v_err=float(pk_b.std(ddof=1) / V6), peaks_E=Ep.tolist(), peaks_logp=lp.tolist(),
                two_peaks_u=[e / V6 for e in two], peaks_u_per_run=[[e / V6 for e in r] for r in Ep_rep],
                E_grid=Egrid.tolist(), logp=logp.tolist(), meta=meta,
                conv_iter=[r["conv_iter"] for r in res], n_rm=n_rm)


def muca12(log, c2, n_sweeps=100000, chunk=2000, n_therm=2000):
    r = [x for x in c2["results"] if x["L"] == 12][0]
    L, E_low, dE, a = 12, np.array(r["E_low"]), r["dE"], np.array(r["a"])
    V6 = 6 * L ** 4
    n = E_low.size
    cen = E_low + 0.5 * dE
    b = float(np.median(a))
    ctx = llr.Context(precision=llr.FP32, device=0)
    ctx.set_params(n_th=100, n_a=100, n_rm=1, seed=SEED + 12, replica_exchange=False, recompute_every=10,
                   approach_cap=20000)
    ctx.add_lattice(L, E_low, dE)
    ctx.bind_state()
    ctx.set_a(0, a)
    ctx.hot_start()
    ap = ctx.approach()
    ctx.autotune()
    ctx.muca_begin([b])
    t0 = time.perf_counter()
    hist = []
    for k in range(0, n_sweeps, chunk):
        hist.append(ctx.muca_sweeps(chunk, sweep0=k))
        log(f"{k + chunk}/{n_sweeps} multicanonical sweeps, {time.perf_counter() - t0:.1f} s")
    t_run = time.perf_counter() - t0
    hp, ha, _, _ = ctx.stats()
    H = np.concatenate(hist)                         # (n_sweeps, n chains)
    lo, hi = E_low[0], E_low[-1] + dE
    meas = H[n_therm:]
    hv, _ = np.histogram(meas.ravel(), bins=np.linspace(lo, hi, 33))
    inside = float(np.mean((meas >= lo) & (meas <= hi)))
    # round trips: from the bottom tenth of the range to the top tenth and back
    band = 0.1 * (hi - lo)
    trips = []
    for ch in range(H.shape[1]):
        state, t = 0, 0
        for e in H[:, ch]:
            if state == 0 and e <= lo + band:
                state = 1
            elif state == 1 and e >= hi - band:
                state = 2
            elif state == 2 and e <= lo + band:
                state, t = 1, t + 1
        trips.append(t)
    betas = np.array([1.006, 1.008, 1.010, 1.01023, 1.012, 1.014])
    u_rw, cv_rw = ctx.muca_reweight(meas, cen, a, dE, V6, betas)
    # error from 8 blocks of the measured sweeps
    blocks = np.array_split(meas, 8, axis=0)
    ub = np.array([ctx.muca_reweight(bk, cen, a, dE, V6, betas)[0] for bk in blocks])
    u_err = ub.std(axis=0, ddof=1) / np.sqrt(len(blocks))
    _, u_llr, cv_llr = ctx.reconstruct(cen, a, dE, V6, betas)
    ctx.close()
    log(f"{n_sweeps} sweeps x {n} chains in {t_run:.1f} s; histogram max/min {hv.max() / max(hv.min(), 1):.2f}, "
        f"{inside:.2f} of samples inside; round trips {sum(trips)} ({np.mean(trips):.1f} per chain)")
    for i, bt in enumerate(betas):
        log(f"beta {bt}: <u> reweighted {u_rw[i]:.5f} +- {u_err[i]:.5f}, LLR {u_llr[i]:.5f}")
    return dict(b=b, n_sweeps=n_sweeps, n_therm=n_therm, seconds=t_run, approach_sweeps=int(ap[0]),
                hb_acceptance=float(ha.sum() / max(hp.sum(), 1)), hist=hv.tolist(), inside=inside,
                round_trips=trips, beta=betas.tolist(), u_reweighted=u_rw.tolist(), u_reweighted_err=u_err.tolist(),
                cv_reweighted=cv_rw.tolist(), u_llr=u_llr.tolist(), cv_llr=cv_llr.tolist(),
                E_series_chain0=H[::10, 0].tolist())


def dE_study(log, L=8, counts=(16, 32, 64, 128), replicas=8):
    """Sec. 3.5: the C_V peak against the interval width over u in
    [0.55, 0.71], cut into `counts` intervals, `replicas` runs each; the fit
    C_V(dE) = C_V(0) + 6V b_dis dE^2."""
    V6 = 6 * L ** 4
    rows = []
    for nk in counts:
        dE = 0.16 / nk * V6
        E_low = 0.55 * V6 + dE * np.arange(nk)
        seed = SEED + nk if L == 8 else SEED + 1000 * L + nk
        res, meta = _run([(L, E_low, dE)] * replicas, llr.FP32, 200, 500, 50, False, seed=seed, log=log)
        cen = E_low + 0.5 * dE
        ctx = llr.Context(precision=llr.FP64, device=0)
        pk = np.array([ctx.beta_c(cen, np.array(r["a"]), dE, V6, 0.98, 1.04, h=1e-5, tol=1e-9) for r in res])
        ctx.close()
        rows.append(dict(n_intervals=nk, dE=dE, beta_c=pk[:, 0].tolist(), cv_peak=pk[:, 1].tolist(),
                         cv_mean=float(pk[:, 1].mean()), cv_err=float(pk[:, 1].std(ddof=1) / np.sqrt(replicas)),
                         bc_mean=float(pk[:, 0].mean()), bc_err=float(pk[:, 0].std(ddof=1) / np.sqrt(replicas)),
                         seconds=meta["seconds_rm"]))
        log(f"{nk} intervals (dE = {dE:.2f}): C_V/(6V) peak {rows[-1]['cv_mean'] / V6:.4e} "
            f"+- {rows[-1]['cv_err'] / V6:.1e}, beta_c {rows[-1]['bc_mean']:.6f} +- {rows[-1]['bc_err']:.6f}")
    def fit(rs, what):
        x = np.array([r["dE"] for r in rs])
        y = np.array([r["cv_mean"] for r in rs])
        sg = np.array([r["cv_err"] for r in rs])
        p, e, chi2 = llr.fss_fit(x, y, sg, [0.0, 2.0])
        inflate = np.sqrt(max(chi2, 1.0))
        b_dis, b_err = p[1] / V6, e[1] / V6 * inflate
        log(f"fit C_V = C_V(0) + 6V b_dis dE^2 ({what}): C_V(0)/(6V) = {p[0] / V6:.4e} +- "
            f"{e[0] / V6 * inflate:.1e}, b_dis = {b_dis:.2e} +- {b_err:.1e}, chi2_red {chi2:.2f}")
        return dict(cv0=p[0], cv0_over_6v=p[0] / V6, cv0_over_6v_err=e[0] / V6 * inflate, b_dis=b_dis,
                    b_dis_err=b_err, chi2_red=chi2)

    # the quadratic law holds for fine spacings (Sec. 3.5); the coarsest one
    # is also fitted without, to show where it stops holding
    out = dict(rows=rows, **fit(rows, "all spacings"))
    out["without_coarsest"] = fit(rows[1:], f"without dE = {rows[0]['dE']:.1f}")
    return out


def obs8(log, n_meas=400, gap=2):
    L = 8
    V6 = 6 * L ** 4
    NP = V6
    dE = 0.005 * V6
    # l8's dE, with the range extended down to u = 0.50 so that the
    # canonical distribution at beta = 0.98 (<u> ~ 0.55) lies inside it
    E_low = 0.50 * V6 + dE * np.arange(42)
    cen = E_low + 0.5 * dE
    ctx = llr.Context(precision=llr.FP32, device=0)
    ctx.set_params(n_th=200, n_a=500, n_rm=50, seed=SEED + 8, replica_exchange=False, recompute_every=10,
                   approach_cap=20000)
    ctx.add_lattice(L, E_low, dE)
    ctx.bind_state()
    ctx.set_a(0, 1.0)
    ctx.hot_start()
    ctx.approach()
    ctx.autotune()
    ctx.run()
    a, _, _ = ctx.get_a(0)
    log("LLR run done; measuring")
    E, B = ctx.observables(n_meas, gap, 1 << 24)
    ctx.close()
    beta = np.linspace(0.98, 1.04, 31)
    ctx = llr.Context(precision=llr.FP64, device=0)
    u = ctx.obs_reconstruct(cen, a, dE, E, E, beta) / V6
    b2 = ctx.obs_reconstruct(cen, a, dE, E, B, beta) / NP
    blocks = [(ctx.obs_reconstruct(cen, a, dE, E[i::4], E[i::4], beta) / V6,
               ctx.obs_reconstruct(cen, a, dE, E[i::4], B[i::4], beta) / NP) for i in range(4)]
    _, u_mid, _ = ctx.reconstruct(cen, a, dE, V6, beta)
    ctx.close()
    u_err = np.std([x[0] for x in blocks], axis=0, ddof=1) / 2
    b_err = np.std([x[1] for x in blocks], axis=0, ddof=1) / 2
    # direct canonical runs: 16 chains whose intervals cover every energy
    canon = {}
    for bt in (0.98, 1.04):
        n = 16
        ctx = llr.Context(precision=llr.FP32, device=0)
        ctx.set_params(seed=SEED + 9, replica_exchange=False, recompute_every=10)
        ctx.add_lattice(L, -V6 + 1e-3 * np.arange(n), 2 * V6 - 1.0)
        ctx.bind_state()
        ctx.set_a(0, bt)
        ctx.hot_start()
        ctx.observables(1, 500, 0)                        # thermalisation
        Ec, Bc = ctx.observables(400, 5, 1000)
        ctx.close()
        per = np.array([Ec.mean(axis=0) / V6, Bc.mean(axis=0) / NP])
        canon[bt] = dict(u=float(per[0].mean()), u_err=float(per[0].std(ddof=1) / np.sqrt(n)),
                         cos2=float(per[1].mean()), cos2_err=float(per[1].std(ddof=1) / np.sqrt(n)))
        i = int(np.argmin(np.abs(beta - bt)))
        log(f"beta {bt}: <u> brackets {u[i]:.5f} +- {u_err[i]:.5f}, canonical {canon[bt]['u']:.5f} +- "
            f"{canon[bt]['u_err']:.5f}; <cos 2 theta_P> brackets {b2[i]:.5f} +- {b_err[i]:.5f}, canonical "
            f"{canon[bt]['cos2']:.5f} +- {canon[bt]['cos2_err']:.5f}")
    return dict(a=a.tolist(), beta=beta.tolist(), u=u.tolist(), u_err=u_err.tolist(), u_midpoint=u_mid.tolist(),
                cos2=b2.tolist(), cos2_err=b_err.tolist(), canonical={str(k): v for k, v in canon.items()},
                n_meas=n_meas, gap=gap)


def l20_part(log, c3, part, n_rep=2, n_rm=100):
    L, E_low, dE = l20_intervals()
    a0 = np.array(c3["a_mlp"])
    res, meta = _run([(L, E_low, dE)] * n_rep, llr.FP32, 500, 2000, n_rm, True, seed=SEED + 1000 * part,
                     a0=[a0] * n_rep, log=log)
    return dict(part=part, runs=[dict(a=r["a"], a_hist=r["a_hist"], conv_iter=r["conv_iter"]) for r in res],
                meta=meta)


def l20_parts_combine(log, parts, n_boot=2000):
    L, E_low, dE = l20_intervals()
    V6 = 6 * L ** 4
    cen = E_low + 0.5 * dE
    A = np.array([r["a"] for p in parts for r in p["runs"]])
    ctx = llr.Context(precision=llr.FP64, device=0)
    per = np.array([ctx.beta_c(cen, a, dE, V6, 1.008, 1.012, h=1e-5, tol=1e-9) for a in A])
    bc_b, pk_b = ctx.bootstrap(cen, A, dE, V6, 1.008, 1.012, n_boot=n_boot, seed=SEED)
    abar = A.mean(axis=0)
    bc, pk = ctx.beta_c(cen, abar, dE, V6, 1.008, 1.012, h=1e-5, tol=1e-9)
    Ep, lp = ctx.prob_peaks(cen, abar, dE, bc)
    ctx.close()
    two = sorted(Ep[np.argsort(lp)[-2:]].tolist()) if Ep.size >= 2 else Ep.tolist()
    log(f"{A.shape[0]} runs: beta_c {bc:.7f} +- {bc_b.std(ddof=1):.7f}, C_V/(6V) {pk / V6:.4e} +- "
        f"{pk_b.std(ddof=1) / V6:.1e}; per-run beta_c spread {per[:, 0].std(ddof=1):.2e}; peaks of P at beta_c "
        f"{[round(e / V6, 5) for e in two]}")
    return dict(n_runs=int(A.shape[0]), beta_c=bc, beta_c_err=float(bc_b.std(ddof=1)), cv_peak_over_6v=pk / V6,
                cv_peak_over_6v_err=float(pk_b.std(ddof=1) / V6), per_run=per.tolist(), two_peaks_u=[e / V6 for e in two],
                peaks_u=(Ep / V6).tolist())


def _tau_int(x, c=6.0):
    """Integrated autocorrelation time of each column of x (rows: sweeps),
    with Sokal's automatic window W >= c tau."""
    x = x - x.mean(axis=0)
    n = x.shape[0]
    f = np.fft.rfft(x, n=2 * n, axis=0)
    acf = np.fft.irfft(f * np.conj(f), axis=0)[:n]
    acf = acf / acf[0]
    tau = np.empty(x.shape[1])
    for k in range(x.shape[1]):
        t = 0.5
        for w in range(1, n):
            t += acf[w, k]
            if w >= c * t:
                break
        tau[k] = t
    return tau


def _link_lattice(log, L, E_low, dE, a, n_meas, n_time, seed, runs=None, pairs=None):
    """runs: (name, mode, first sweep index, sweep order) of each sampler;
    pairs: the runs whose mean energies are compared."""
    if runs is None:
        runs = (("class", llr.MODE_RESTRICTED, 1 << 22, llr.SWEEP_GROUPED),
                ("class2", llr.MODE_RESTRICTED, 1 << 23, llr.SWEEP_GROUPED),
                ("link", llr.MODE_LINK, 1 << 22, llr.SWEEP_GROUPED))
    if pairs is None:
        pairs = (("class", "class2"), ("class", "link"), ("class2", "link"))
    ctx = llr.Context(precision=llr.FP32, device=0)
    ctx.set_params(seed=seed, replica_exchange=False, recompute_every=10, approach_cap=20000)
    ctx.add_lattice(L, E_low, dE)
    ctx.bind_state()
    ctx.set_a(0, np.asarray(a))
    ctx.hot_start()
    ctx.approach()
    ctx.autotune()
    ctx.sweeps(200, sweep0=1 << 20, mode=llr.MODE_RESTRICTED, want_bits=False)
    start = ctx.export_state(0).clone()
    n = len(E_low)
    out = {}
    # class2: the class-wise mode again with other random numbers (other sweep
    # indices), the reference for how far two runs of one ensemble differ
    for name, mode, s0, order in runs:
        ctx.set_sweep_order(order)
        ctx.import_state(0, start)
        ctx.sweeps(5, sweep0=1 << 21, mode=mode, want_bits=False)          # warm-up (first use allocates)
        t0 = time.perf_counter()
        ctx.sweeps(n_time, sweep0=(1 << 21) + 8, mode=mode, want_bits=False)
        ms = (time.perf_counter() - t0) / n_time * 1e3
        ctx.import_state(0, start)
        hp0, ha0, _, _ = ctx.stats()
        f0, r0 = ctx.link_stats()
        E = np.empty((n_meas, n))
        for t in range(n_meas):
            ctx.sweeps(1, sweep0=s0 + t, mode=mode, want_bits=False)
            if (t + 1) % 10 == 0:
                ctx.recompute_energy()
            E[t] = ctx.get_energy(0)[0]
        hp1, ha1, _, _ = ctx.stats()
        f1, r1 = ctx.link_stats()
        tau = _tau_int(E)
        # error of the mean per interval from 20 batch means (blind to the
        # window choice of tau_int)
        nb = 20
        bm = E[: (n_meas // nb) * nb].reshape(nb, -1, n).mean(axis=1)
        err_b = bm.std(axis=0, ddof=1) / np.sqrt(nb)
        acc = float((ha1 - ha0).sum() / max((hp1 - hp0).sum(), 1))
        red = float((f1 - f0).sum() / (n_meas * 8 * n))
        arc = float((r1 - r0).sum() / (n_meas * 8 * n))
        eff = 1.0 / (2.0 * np.median(tau) * ms * 1e-3)
        out[name] = dict(ms_per_sweep=ms, tau_int=tau.tolist(), tau_median=float(np.median(tau)),
                         tau_max=float(tau.max()), class_acceptance=acc, redrawn_per_pass=red, arc_per_pass=arc,
                         independent_per_s=eff, E_mean=E.mean(axis=0).tolist(), E_std=E.std(axis=0).tolist(),
                         E_err_batch=err_b.tolist())
        log(f"L={L} {name}: {ms:.3f} ms/sweep, tau_int median {np.median(tau):.2f} (max {tau.max():.2f}) sweeps, "
            f"class acceptance {acc:.3f}, re-drawn links per class pass {red:.1f} (arc {arc:.2f}), "
            f"{eff:.1f} independent samples/s per chain")
    ctx.close()
    # both modes sample the same restricted ensemble: compare the means, and
    # two class-wise runs with each other for the spread one ensemble shows
    for a_, b_ in pairs:
        z = (np.array(out[a_]["E_mean"]) - np.array(out[b_]["E_mean"])) / np.hypot(
            out[a_]["E_err_batch"], out[b_]["E_err_batch"])
        out[f"mean_difference_{a_}_{b_}"] = dict(chi2_per_interval=float(np.mean(z ** 2)),
                                                 max_abs_z=float(np.abs(z).max()), argmax=int(np.abs(z).argmax()),
                                                 mean_z=float(z.mean()), n=int(z.size), z=z.tolist())
        log(f"L={L} {a_} vs {b_}, mean E per interval (batch errors): chi2/n {np.mean(z ** 2):.2f}, "
            f"max |z| {np.abs(z).max():.2f} (interval {int(np.abs(z).argmax())}), mean z {z.mean():+.2f} over {z.size}")
    return out


def link_compare(log, a20, n_meas8=8000, n_meas20=4000):
    L = 8
    V6 = 6 * L ** 4
    dE = 0.005 * V6
    E_low = 0.55 * V6 + dE * np.arange(32)
    res, _ = _run([(L, E_low, dE)], llr.FP32, 200, 500, 20, False, log=log)
    rec = dict(L8=_link_lattice(log, L, E_low, dE, res[0]["a"], n_meas8, 500, SEED + 17))
    L, E_low, dE = l20_intervals()
    rec["L20"] = _link_lattice(log, L, E_low, dE, a20, n_meas20, 200, SEED + 19)
    return rec


def order_compare(log, a20, n_meas8=8000, n_meas20=8000):
    """The grouped and the interleaved order of a sweep's class passes (the
    latter with fused launches) at fixed a_k: mean E per interval against a second grouped run
    with other random numbers, which gives the spread of one ensemble."""
    runs = (("grouped", llr.MODE_RESTRICTED, 1 << 22, llr.SWEEP_GROUPED),
            ("grouped2", llr.MODE_RESTRICTED, 1 << 23, llr.SWEEP_GROUPED),
            ("interleaved", llr.MODE_RESTRICTED, 1 << 22, llr.SWEEP_INTERLEAVED))
    pairs = (("grouped", "grouped2"), ("grouped", "interleaved"), ("grouped2", "interleaved"))
    L = 8
    V6 = 6 * L ** 4
    dE = 0.005 * V6
    E_low = 0.55 * V6 + dE * np.arange(32)
    res, _ = _run([(L, E_low, dE)], llr.FP32, 200, 500, 20, False, log=log)
    rec = dict(L8=_link_lattice(log, L, E_low, dE, res[0]["a"], n_meas8, 500, SEED + 23, runs, pairs))
    L, E_low, dE = l20_intervals()
    rec["L20"] = _link_lattice(log, L, E_low, dE, a20, n_meas20, 200, SEED + 29, runs, pairs)
    return rec


def link_profile(log, a20, n=60):
    L, E_low, dE = l20_intervals()
    ctx = llr.Context(precision=llr.FP32, device=0)
    ctx.set_params(seed=SEED + 19, replica_exchange=False, recompute_every=10, approach_cap=20000)
    ctx.add_lattice(L, E_low, dE)
    ctx.bind_state()
    ctx.set_a(0, np.asarray(a20))
    ctx.hot_start()
    ctx.approach()
    ctx.autotune()
    ctx.sweeps(100, sweep0=1 << 20, mode=llr.MODE_RESTRICTED, want_bits=False)
    for name, mode in (("class", llr.MODE_RESTRICTED), ("link", llr.MODE_LINK)):
        t0 = time.perf_counter()
        ctx.sweeps(n, sweep0=1 << 21, mode=mode, want_bits=False)
        log(f"{name}: {(time.perf_counter() - t0) / n * 1e3:.3f} ms/sweep")
    f, r = ctx.link_stats()
    ctx.close()
    return dict(redrawn_per_pass=float(f.sum() / (n * 8 * len(E_low))), arc_per_pass=float(r.sum() / (n * 8 * len(E_low))))


def batch_profile(log, n=200):
    lats = []
    for L in (12, 16, 20):
        V6 = 6 * L ** 4
        dE = 0.1 / 64 * V6
        lats.append((L, 0.58 * V6 + dE * np.arange(64), dE))
    ctx = llr.Context(precision=llr.FP32, device=0)
    ctx.set_params(seed=SEED, replica_exchange=True, recompute_every=10, approach_cap=20000)
    ctx.set_sweep_order(SWEEP_ORDER)
    for (L, E_low, dE) in lats:
        ctx.add_lattice(L, E_low, dE)
    ctx.bind_state()
    for i in range(3):
        ctx.set_a(i, 1.0)
    ctx.hot_start()
    ap = ctx.approach()
    tiles = ctx.autotune()
    ctx.sweeps(10, sweep0=1 << 20, mode=llr.MODE_RESTRICTED, want_bits=False)
    st0 = ctx.stats()
    t0 = time.perf_counter()
    ctx.sweeps(n, sweep0=(1 << 20) + 16, mode=llr.MODE_RESTRICTED, want_bits=False)
    dt = (time.perf_counter() - t0) / n
    upd = sum(_updates_per_class_link(ctx, st0) * 4 * L ** 4 * len(E_low) for (L, E_low, dE) in lats)
    ctx.close()
    log(f"{dt * 1e3:.3f} ms per sweep of 192 chains (L = 12, 16, 20), {upd / dt:.4g} link updates/s, "
        f"tiles {tiles}, approach sweeps {[int(x) for x in ap]}")
    return dict(ms_per_sweep=dt * 1e3, updates_per_s=upd / dt, tiles=list(tiles), approach_sweeps=list(map(int, ap)),
                sweep_order=_ORDER_NAMES[SWEEP_ORDER])


FSS_PARTS = {0: (8, 10, 12, 14), 1: (16, 18)}


def fss_part(log, c3, part, n_rep=4, n_int=96, n_rm=80, n_boot=1000):
    w = np.array(c3["weights"], dtype=np.float32)
    out = {}
    for L in FSS_PARTS[part]:
        V6 = 6 * L ** 4
        dE = 0.14 / n_int * V6
        E_low = 0.56 * V6 + dE * np.arange(n_int)
        cen = E_low + 0.5 * dE
        ctx = llr.Context(precision=llr.FP32, device=0)
        a0 = ctx.mlp_predict(w, cen / V6, np.full(n_int, 1.0 / L))
        ctx.close()
        res, meta = _run([(L, E_low, dE)] * n_rep, llr.FP32, 200, 800, n_rm, True, seed=SEED + 100 * L,
                         a0=[a0] * n_rep, log=log)
        A = np.array([r["a"] for r in res])
        ctx = llr.Context(precision=llr.FP64, device=0)
        per = np.array([ctx.beta_c(cen, A[i], dE, V6, 0.995, 1.02, h=1e-5, tol=1e-9) for i in range(n_rep)])
        bc_b, pk_b = ctx.bootstrap(cen, A, dE, V6, 0.995, 1.02, n_boot=n_boot, seed=SEED + L)
        bc, pk = ctx.beta_c(cen, A.mean(axis=0), dE, V6, 0.995, 1.02, h=1e-5, tol=1e-9)
        ctx.close()
        out[str(L)] = dict(L=L, dE=dE, a_runs=A.tolist(), a0=a0.tolist(), per_run=per.tolist(), beta_c=bc,
                           beta_c_err=float(bc_b.std(ddof=1)), cv_peak_over_6v=pk / V6,
                           cv_peak_over_6v_err=float(pk_b.std(ddof=1) / V6), meta=meta,
                           conv_iter=[r["conv_iter"] for r in res])
        log(f"L={L}: beta_c {bc:.6f} +- {bc_b.std(ddof=1):.6f}, C_V/(6V) {pk / V6:.4e} +- "
            f"{pk_b.std(ddof=1) / V6:.1e} ({meta['seconds_rm']:.0f} s)")
    return out


def fss_combine(log, parts, c4b_parts, n_boot=2000):
    rows = {}
    for p in parts:
        for k, v in p.items():
            if k.isdigit():
                rows[int(k)] = (v["beta_c"], v["beta_c_err"], v["cv_peak_over_6v"], v["cv_peak_over_6v_err"])
    if c4b_parts:
        L, E_low, dE = l20_intervals()
        V6 = 6 * L ** 4
        cen = E_low + 0.5 * dE
        A = np.array([r["a"] for p in c4b_parts for r in p["runs"]])
        ctx = llr.Context(precision=llr.FP64, device=0)
        bc_b, pk_b = ctx.bootstrap(cen, A, dE, V6, 1.008, 1.012, n_boot=n_boot, seed=SEED)
        bc, pk = ctx.beta_c(cen, A.mean(axis=0), dE, V6, 1.008, 1.012, h=1e-5, tol=1e-9)
        ctx.close()
        rows[20] = (bc, float(bc_b.std(ddof=1)), pk / V6, float(pk_b.std(ddof=1) / V6))
        log(f"L=20 ({A.shape[0]} runs): beta_c {bc:.7f} +- {bc_b.std(ddof=1):.7f}, C_V/(6V) {pk / V6:.4e} +- "
            f"{pk_b.std(ddof=1) / V6:.1e}")
    Ls = np.array(sorted(rows))
    tab = np.array([rows[L] for L in Ls])
    fits = []
    for Lmin in (8, 10, 12, 14):
        m = Ls >= Lmin
        for kmax in (1, 2):
            if m.sum() <= kmax + 1:
                continue
            pw = np.array([0.0] + [-4.0 * k for k in range(1, kmax + 1)])
            pb, eb, cb = llr.fss_fit(Ls[m], tab[m, 0], tab[m, 1], pw)
            pc, ec, cc = llr.fss_fit(Ls[m], tab[m, 2], tab[m, 3], pw)
            G = 2.0 * np.sqrt(max(pc[0], 0.0))
            fits.append(dict(L_min=int(Lmin), k_max=kmax, beta_c=pb[0], beta_c_err=eb[0], chi2_beta=cb,
                             G=G, G_err=ec[0] / max(G, 1e-300) * 2.0, chi2_cv=cc))
            log(f"L >= {Lmin}, k_max {kmax}: beta_c(inf) {pb[0]:.7f} +- {eb[0]:.7f} (chi2/dof {cb:.2f}); "
                f"G {G:.5f} +- {fits[-1]['G_err']:.5f} (chi2/dof {cc:.2f})")
    return dict(L=Ls.tolist(), table=tab.tolist(), fits=fits)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["l8", "batched", "warmstart", "l20", "l20reps", "muca12",
                                            "dE8", "dE12", "obs8",
                                            "l20parts", "linkcmp", "linkprof", "fss", "batchprof", "ordercmp"])
    ap.add_argument("--out", default="experiment_out")
    ap.add_argument("--inputs", default=None, help="directory holding the records a run starts from "
                    "(warmstart reads l8 and batched, l20 reads warmstart); default --out")
    ap.add_argument("--n-rm", type=int, default=None)
    ap.add_argument("--part", type=int, default=0)
    ap.add_argument("--combine", action="store_true")
    ap.add_argument("--order", choices=["grouped", "interleaved", "staggered"], default="grouped",
                    help="order of the class passes in the sweeps of the Algorithm 1 runs")
    ap.add_argument("--jsonl", default=None,
                    help="append one JSON line per Robbins-Monro iteration of the Algorithm 1 runs to this file "
                         "(a_k, max |da_k|, acceptance rates, link updates/s, recompute drift, health)")
    args = ap.parse_args()
    global SWEEP_ORDER, JSONL
    JSONL = args.jsonl
    SWEEP_ORDER = {v: k for k, v in _ORDER_NAMES.items()}[args.order]
    os.makedirs(args.out, exist_ok=True)

    def log(msg):
        print(f"# {args.which}: {msg}", flush=True)

    def load(name):
        with open(os.path.join(args.inputs or args.out, f"{name}.json")) as f:
            return json.load(f)

    t0 = time.perf_counter()
    if args.which == "l8":
        rec = run_l8(log)
    elif args.which == "batched":
        rec = run_batched(log)
    elif args.which == "warmstart":
        rec = run_warmstart(log, load("l8"), load("batched"), n_rm=args.n_rm or 20)
    elif args.which == "l20":
        rec = run_l20(log, load("warmstart"), n_rm=args.n_rm or 100)
    elif args.which == "muca12":
        rec = muca12(log, load("batched"))
    elif args.which == "dE8":
        rec = dE_study(log, 8)
    elif args.which == "dE12":
        rec = dE_study(log, 12, counts=(8, 16, 32, 64, 128))
    elif args.which == "obs8":
        rec = obs8(log)
    elif args.which == "batchprof":
        rec = batch_profile(log)
    elif args.which == "fss" and args.combine:
        import glob
        src = args.inputs or args.out

        def recs(pattern):
            out = []
            for f in sorted(glob.glob(os.path.join(src, pattern))):
                with open(f) as fh:
                    out.append(json.load(fh))
            return out
        rec = fss_combine(log, recs("fss_part*.json"), recs("l20_part*.json"))
    elif args.which == "fss":
        rec = fss_part(log, load("warmstart"), args.part)
    elif args.which in ("linkcmp", "linkprof", "ordercmp"):
        # converged L=20 a_k when a l20parts record is given, else beta_c(20) throughout
        src = os.path.join(args.inputs or args.out, "l20parts_part0.json")
        a20 = load("l20parts_part0")["runs"][0]["a"] if os.path.exists(src) else [1.011] * 128
        if args.which == "linkcmp":
            rec = link_compare(log, a20)
        elif args.which == "ordercmp":
            rec = order_compare(log, a20)
        else:
            rec = link_profile(log, a20)
    elif args.which == "l20parts" and args.combine:
        import glob
        parts = []
        for f in sorted(glob.glob(os.path.join(args.inputs or args.out, "l20_part*.json"))):
            with open(f) as fh:
                parts.append(json.load(fh))
        rec = l20_parts_combine(log, parts)
    elif args.which == "l20parts":
        rec = l20_part(log, load("warmstart"), args.part, n_rm=args.n_rm or 100)
    else:
        rec = l20_replicas(log, load("warmstart"), n_rm=args.n_rm or 25)
    rec["wall_seconds"] = time.perf_counter() - t0
    name = args.which
    if args.which in ("l20parts", "fss"):
        name = f"{args.which}_combined" if args.combine else f"{args.which}_part{args.part}"
    with open(os.path.join(args.out, f"{name}.json"), "w") as f:
        json.dump(rec, f)
    log(f"done in {rec['wall_seconds']:.1f} s")


if __name__ == "__main__":
    sys.exit(main())
