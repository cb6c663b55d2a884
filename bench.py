"""Throughput benchmark of the LLR restricted sweep on one MI355X.

Workload (the metric's configuration): 4D compact U(1), L = 20 (640 000
links per chain), 128 intervals over u = E/(6V) in [0.60, 0.664] with
dE = 0.0005 6V = 480, replica exchange between neighbouring intervals after
every sweep (restriction width 2 dE), FP32 link angles with FP64 energies,
interval tests and Robbins-Monro updates, N_TH = 500, N_A = 2000, FP64
recompute every 10 sweeps.  Synthetic data: uniform hot start from the seed,
then the approach phase (untimed).

One step = one Robbins-Monro iteration of all 128 intervals: 2500 sweeps (8
heatbath + 8 overrelaxation class passes of all chains, recompute, replica
exchange, measurement), the a_k update, and the FP64 reconstruction of
beta_c and the C_V peak on beta in [1.008, 1.012].  One link update = one
heatbath or one overrelaxation of one link.

--order: grouped (default; heatbath of every colour, then overrelaxation of
every colour, 16 launches per sweep: 2 x 4V updates per sweep), staggered
(the grouped passes on the first 64 chains and, overrelaxation first, on the
other 64, the two halves on two streams so that heatbath and overrelaxation
passes overlap; 2 x 4V updates per sweep) or interleaved
(heatbath then overrelaxation per colour, one fused launch per colour).  In
the interleaved order the overrelaxation reflects the heatbath draw just made
on the same staples, which is again a von Mises draw: an accepted heatbath
class gives its links one update, a rejected one gives the rejected proposal
and one overrelaxation.  Its count is (2 - acceptance) x V/2 per class pass,
with the heatbath class acceptance measured over the timed steps.

The metric's second half (rm_sweeps_plain_vs_mlp in the JSON line): Robbins-
Monro sweeps to the stopping rule |a^(n+1) - a^(n)| < 1e-4 on the same
interval set, from a^(0) = 1 and from the warm start of the network trained
in this run by the library's kernels on converged a_k of L = 8, 12, 16
(paper_1509_08391_amd/warmstart/), and the time to accuracy against the
long-run reference slopes stored there; --m2-iters-plain and --m2-iters-mlp iterations.

The timed steps run with per-kernel HIP-event timing (which launches the
sweeps eagerly); one more step after them replays the captured sweep graphs,
the library's default path, and is reported as graph_replay.  health: chains
flagged by the recompute's health tests and the largest drift of the
incremental energy seen at a recompute.

cpu_baseline: the CPU oracle (FP64, OpenMP over chains) timed on restricted
sweeps of L=20 chains inside intervals of the benchmark's width, on all host
cores and on one.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

L = 20
N_INT = 128
SEED = 1509083910
PEAK_HBM_GBS = 8000.0
# Calibrated HBM bytes per heatbath launch (FETCH_SIZE x 2 + WRITE_SIZE x 1,
# rocprofv3 on this kernel version with 4 class links per thread;
# profiles/k_hb_L20x128_fp32_counters.md for the plain pass of the grouped
# order, profiles/k_hb_or_fused_L20x128_fp32_counters.md for the fused pass of
# the interleaved order); None once the kernel changes until the counters are
# taken again.
HB_TRAFFIC = {("fp32", 4, "grouped"): 374.8e6, ("fp32", 4, "interleaved"): 410.3e6}


WARMSTART = os.path.join(ROOT, "paper_1509_08391_amd", "warmstart")


def _a_ref():
    with open(os.path.join(WARMSTART, "aref_L20.json")) as f:
        return json.load(f)


def cpu_baseline(order, target_s=10.0):
    """The oracle (plain FP64 C, OpenMP over chains) on a bounded sample of the
    same workload: restricted sweeps (8 heatbath + 8 overrelaxation passes)
    of L=20 chains whose energies lie inside their intervals.  The states come
    from the seeded input generator (plaquette densities spread over the
    intervals' range u in [0.60, 0.664]); each chain is restricted to an
    interval of the benchmark's width 2 dE centred on its energy, at the
    reference a_k of the interval nearest that energy; one untimed sweep
    first.  All cores: one chain per thread; one core: a single chain."""
    import oracle
    from tests.inputs import random_state
    oracle.build(force=False)
    threads = oracle.num_threads()
    V6 = 6 * L ** 4
    dE = 0.0005 * V6
    ref = _a_ref()
    cen = np.array(ref["E_low"]) + 0.5 * dE
    o_order = {"interleaved": oracle.SWEEP_INTERLEAVED, "staggered": oracle.SWEEP_STAGGERED}.get(
        order, oracle.SWEEP_GROUPED)

    def run(nch, budget):
        th = np.ascontiguousarray(np.concatenate(
            [random_state(4, L, 1, seed=SEED + k, u_target=0.60 + 0.064 * (k + 0.5) / nch) for k in range(nch)]))
        E = np.array([oracle.energy(4, L, th[k]) for k in range(nch)])
        a = np.interp(E, cen, ref["a_ref"])
        lo, hi = E - dE, E + dE
        itv = np.arange(nch)
        E, _ = oracle.sweeps(4, L, th, a, lo, hi, itv, E, 1, 0, seed=SEED, order=o_order)
        done = 0
        t0 = time.perf_counter()
        while True:
            E, bits = oracle.sweeps(4, L, th, a, lo, hi, itv, E, 1, 1 + done, seed=SEED, order=o_order)
            done += 1
            if time.perf_counter() - t0 > budget:
                break
        dt = time.perf_counter() - t0
        assert np.all((E >= lo) & (E <= hi))
        return 2.0 * 4 * L ** 4 * nch * done / dt, done, dt

    v_all, n_all, t_all = run(threads, target_s)
    v_one, n_one, t_one = run(1, 0.5 * target_s)
    return {"value": v_all, "unit": "link updates/s", "cores": threads, "kind": "oracle",
            "one_core": v_one,
            "sample": f"restricted sweeps (8 heatbath + 8 overrelaxation passes, {order}) of L=20 chains inside "
                      f"intervals of width 2 dE = {2 * dE:.0f} at the reference a_k: {n_all} sweep(s) of {threads} "
                      f"chains, one per thread, in {t_all:.1f} s (all cores); {n_one} sweep(s) of one chain in "
                      f"{t_one:.1f} s (one core, {v_one:.3e} updates/s)"}


def rm_convergence(llr, n_plain, n_mlp):
    """The metric's second half: Robbins-Monro sweeps to |a^(n+1) - a^(n)| <
    1e-4 (the stopping rule of Sec. 2.4) on the full-pipeline interval set,
    from the cold start a^(0) = 1 and from the warm start of the network
    trained here with the library's kernels on the converged a_k of L = 8, 12,
    16 (warmstart/train_ak.json; predictions that are non-finite or outside
    the trained range fall back to a^(0) = 1).  Same seed, same GPU, N_RM =
    n_plain and n_mlp.  Also the time to accuracy against the long-run reference
    slopes (warmstart/aref_L20.json): the sweeps after which every a_k^(n)
    stays within tol of a_ref for all later n of the run."""
    with open(os.path.join(WARMSTART, "train_ak.json")) as f:
        pts = np.array(json.load(f)["points"])
    ref = _a_ref()
    a_ref = np.array(ref["a_ref"])
    u, il, a_tr = pts[:, 0], pts[:, 1], pts[:, 2]
    V6 = 6 * L ** 4
    dE = 0.0005 * V6
    E_low = 0.60 * V6 + dE * np.arange(N_INT)
    t0 = time.perf_counter()
    c0 = llr.Context(precision=llr.FP32, device=0)
    w, hist = c0.mlp_train(c0.mlp_init(SEED), u, il, a_tr, epochs=4000, lr=3e-3, bf16=True)
    fit_rms = float(np.sqrt(np.mean((c0.mlp_predict(w, u, il, bf16=True) - a_tr) ** 2)))
    c0.close()
    t_train = time.perf_counter() - t0
    margin = 0.1 * (a_tr.max() - a_tr.min())
    nsw = 2500
    out = {"n_rm": {"plain": n_plain, "mlp": n_mlp}, "eps": 1e-4, "training_points": int(len(pts)), "train_s": t_train,
           "fit_rms": fit_rms, "a_ref_uncertainty_max": 2 * float(np.max(ref["half_difference"]))}
    for name, n_iter in (("plain", n_plain), ("mlp", n_mlp)):
        ctx = llr.Context(precision=llr.FP32, device=0)
        ctx.set_params(n_th=500, n_a=2000, n_rm=n_iter, seed=SEED, replica_exchange=True, overlap=1.0,
                       recompute_every=10, eps=1e-4, approach_cap=20000)
        ctx.add_lattice(L, E_low, dE)
        ctx.bind_state()
        nf = 0
        if name == "mlp":
            a0, nf = ctx.mlp_warm_start(0, w, a_tr.min() - margin, a_tr.max() + margin)
            out["mlp_error_vs_a_ref"] = {"max": float(np.max(np.abs(a0 - a_ref))),
                                         "rms": float(np.sqrt(np.mean((a0 - a_ref) ** 2))), "fallbacks": int(nf)}
        else:
            a0 = np.full(N_INT, 1.0)
            ctx.set_a(0, a0)
        t1 = time.perf_counter()
        ctx.hot_start()
        ap = int(ctx.approach()[0])
        ctx.rm_begin()
        for it in range(n_iter):
            ctx.rm_step(1)
            if it % 5 == 4:
                print(f"# {name} start: RM iteration {it + 1}/{n_iter}, {time.perf_counter() - t1:.0f} s",
                      file=sys.stderr, flush=True)
        wall = time.perf_counter() - t1
        a_fin, conv, conv_sw = ctx.get_a(0)
        hist = ctx.get_history(0)
        ctx.close()
        ok = conv >= 0
        r = {"approach_sweeps": ap, "wall_s": wall,
             "intervals_converged": int(ok.sum()),
             "sweeps_to_stop_total": int(conv_sw[ok].sum()),
             "sweeps_to_stop_slowest": int(conv_sw[ok].max()) if ok.any() else None,
             "mean_iteration_of_stop": float(conv[ok].mean()) if ok.any() else None,
             "final_error_vs_a_ref": {"max": float(np.max(np.abs(a_fin - a_ref))),
                                      "rms": float(np.sqrt(np.mean((a_fin - a_ref) ** 2)))}}
        for tol in (1e-3, 3e-4):
            bad = np.abs(hist - a_ref[None, :]) >= tol          # rows n = 0..n_iter
            last_bad = np.where(bad.any(axis=1))[0]
            n_ok = 0 if last_bad.size == 0 else int(last_bad[-1]) + 1
            r[f"sweeps_to_within_{tol:g}_of_a_ref"] = ap + n_ok * nsw if n_ok <= n_iter else None
        out[name] = r
    p, m = out["plain"], out["mlp"]
    if p["sweeps_to_stop_total"] and m["sweeps_to_stop_total"]:
        out["stop_sweeps_ratio_plain_over_mlp"] = p["sweeps_to_stop_total"] / m["sweeps_to_stop_total"]
    return out


def link_updates(order, V, n_chains, n_sweeps, hb_acceptance):
    """Link updates done by n_sweeps sweeps of n_chains chains of V sites.
    Grouped order: every link gets one heatbath and one overrelaxation per
    sweep, 2 x 4V.  Interleaved order: 8 fused passes of V/2 class links, one
    update per link of an accepted heatbath class (the overrelaxation that
    follows on the same staples is a relabelled draw) and two (rejected
    proposal, overrelaxation) per link of a rejected one.  Staggered order:
    the grouped order's passes on every chain (half of them overrelaxation
    first), 2 x 4V."""
    if order in ("grouped", "staggered"):
        return 2.0 * 4 * V * n_chains * n_sweeps
    return (2.0 - hb_acceptance) * 8 * (V // 2) * n_chains * n_sweeps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--m2-iters-plain", type=int, default=40,
                    help="Robbins-Monro iterations of the convergence run from a^(0) = 1")
    ap.add_argument("--m2-iters-mlp", type=int, default=20,
                    help="Robbins-Monro iterations of the convergence run from the network's warm start")
    ap.add_argument("--no-m2", action="store_true", help="skip the plain-vs-network convergence runs")
    ap.add_argument("--order", choices=["grouped", "interleaved", "staggered"], default="grouped")
    ap.add_argument("--n-th", type=int, default=500)
    ap.add_argument("--n-a", type=int, default=2000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 5 plain device copies of 1 GiB (FP32) to calibrate the FETCH_SIZE and "
                         "WRITE_SIZE counters against a known byte count, then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the chains of this workload are "
              f"independent between replica exchanges and one MI355X holds all 128 of them.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1509_08391_amd import llr

    if args.copy_calibration:
        n = 1 << 28
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 5
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 6,
                          "copy_GBps_read_plus_write": 8 * n / dt / 1e9}))
        return

    V = L ** 4
    V6 = 6 * V
    dE = 0.0005 * V6
    E_low = 0.60 * V6 + dE * np.arange(N_INT)
    prec = llr.FP32 if args.precision == "fp32" else llr.FP64
    n_rm = args.warmup + args.steps + 1   # + one step replayed from HIP graphs after the timed region
    ctx = llr.Context(precision=prec, device=0)
    ctx.set_params(n_th=args.n_th, n_a=args.n_a, n_rm=n_rm, seed=SEED, replica_exchange=True, overlap=1.0,
                   recompute_every=10, eps=1e-4, approach_cap=20000)
    ctx.add_lattice(L, E_low, dE)
    ctx.bind_state()
    ctx.set_a(0, np.full(N_INT, 1.0))
    ctx.set_sweep_order({"grouped": llr.SWEEP_GROUPED, "interleaved": llr.SWEEP_INTERLEAVED,
                         "staggered": llr.SWEEP_STAGGERED}[args.order])
    t_setup = time.perf_counter()
    ctx.hot_start()
    ctx.approach_begin()
    done = False
    while not done:
        ap_sweeps, done = ctx.approach_continue(50)
        E, _ = ctx.get_energy(0)
        inside = int(np.sum((E >= E_low - 0.5 * dE) & (E <= E_low + 1.5 * dE)))
        print(f"# approach: {int(ap_sweeps[0])} sweeps, {inside}/{N_INT} chains inside, "
              f"{time.perf_counter() - t_setup:.1f} s", file=sys.stderr, flush=True)
        if ap_sweeps[0] >= 20000:
            raise SystemExit("approach did not finish within 20000 sweeps")
    t_setup = time.perf_counter() - t_setup
    tiles = ctx.autotune()
    print(f"# autotuned class links per thread: heatbath {tiles[0]}, overrelaxation {tiles[1]}",
          file=sys.stderr, flush=True)
    ctx.rm_begin()
    centres = E_low + 0.5 * dE
    for w in range(args.warmup):
        ctx.rm_step(1)
        print(f"# warmup step {w} done", file=sys.stderr, flush=True)
    ctx.set_timing(True)
    hp0, ha0, _, _ = ctx.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ctx.rm_step(1)
        a, _, _ = ctx.get_a(0)
        bc, pk = ctx.beta_c(centres, a, dE, V6, 1.008, 1.012, h=1e-5, tol=1e-9)
        print(f"# step {s}: beta_c {bc:.6f} C_V/(6V) {pk / V6:.3e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = ctx.get_timing()
    hp, ha, rp, ra = ctx.stats()
    ctx.set_timing(False)
    # the same work with the sweeps replayed from the captured HIP graphs (the
    # library's default path; per-kernel event timing launches them eagerly)
    torch.cuda.synchronize()
    tg0 = time.perf_counter()
    ctx.rm_step(1)
    a, _, _ = ctx.get_a(0)
    ctx.beta_c(centres, a, dE, V6, 1.008, 1.012, h=1e-5, tol=1e-9)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - tg0
    rates = ctx.rates()
    health_flags, drift = ctx.health()

    nsw = args.n_th + args.n_a
    dt = t1 - t0
    hb_acc_timed = float((ha - ha0).sum() / max((hp - hp0).sum(), 1))
    updates = link_updates(args.order, V, N_INT, nsw * args.steps, hb_acc_timed)
    value = updates / dt
    esz = 4 if prec == llr.FP32 else 8
    # algorithmic bytes of one heatbath pass: the pass reads the whole lattice
    # once (4V angles for V/2 class links = 8 angles per class link) and
    # writes one proposal per class link: 9 angles per class link (one
    # update); the fused pass of the interleaved order writes two (the
    # overrelaxed candidate and the overrelaxed old angle): 10 angles per
    # class link for its two updates
    # In the staggered order the heatbath and overrelaxation passes of the two
    # chain halves overlap on two streams and one event pair spans a sweep's
    # 16 launches: the figure is then the class passes' average, 9 angles per
    # class link for either kind of pass, over the sweep's class-pass time.
    per_link = 10 if args.order == "interleaved" else 9
    bytes_per_hb_launch = N_INT * (V // 2) * per_link * esz
    hb_avg_s = tm["hb_ms"] / max(tm["hb_n"], 1) / 1e3
    achieved = bytes_per_hb_launch / hb_avg_s / 1e9 if hb_avg_s > 0 else 0.0
    or_avg_s = tm["or_ms"] / max(tm["or_n"], 1) / 1e3
    kernel = {"grouped": "heatbath class pass (k_hb)",
              "interleaved": "heatbath + overrelaxation class pass (k_hb, fused)",
              "staggered": "class passes of both chain halves on two streams (k_hb, k_or), per pass"}[args.order]
    out = {
        "metric": "link updates/s at 20^4x128 intervals; RM sweeps to |da_k|<1e-4, plain vs MLP",
        "value": value,
        "unit": "link updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == llr.FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": "LLR 4D compact U(1), L=20, 128 intervals u in [0.60,0.664], dE=480, "
                               "replica exchange (w=2dE), N_TH=500, N_A=2000; step = one Robbins-Monro "
                               "iteration (2500 sweeps) + beta_c reconstruction",
                   "L": L, "intervals": N_INT, "sweeps_per_step": nsw, "tiles": list(tiles),
                   "sweep_order": args.order,
                   "precision": "fp32 angles, fp64 energy/test/RM" if prec == llr.FP32 else "fp64"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": HB_TRAFFIC.get((args.precision, tiles[0], args.order)),
                     "kernel": kernel,
                     "bytes_per_launch": bytes_per_hb_launch, "avg_launch_us": hb_avg_s * 1e6,
                     "overrelaxation_avg_launch_us": or_avg_s * 1e6 if args.order != "staggered" else None},
        "acceptance": {"heatbath_class": hb_acc_timed, "overrelaxation": rates["or_acceptance"],
                       "replica_exchange": float(ra / max(rp, 1))},
        "approach_sweeps": int(ap_sweeps[0]),
        "graph_replay": {"ms_per_step": t_graph * 1e3, "link_updates_per_s": updates / args.steps / t_graph},
        "health": {"chains_flagged": int(np.count_nonzero(health_flags)),
                   "max_recompute_drift": float(drift.max())},
    }
    ctx.close()
    if not args.no_m2 and args.precision == "fp32":
        out["rm_sweeps_plain_vs_mlp"] = rm_convergence(llr, args.m2_iters_plain, args.m2_iters_mlp)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.order)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
