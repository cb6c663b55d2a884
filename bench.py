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
every colour, 16 launches per sweep: 2 x 4V updates per sweep) or interleaved
(heatbath then overrelaxation per colour, one fused launch per colour).  In
the interleaved order the overrelaxation reflects the heatbath draw just made
on the same staples, which is again a von Mises draw: an accepted heatbath
class gives its links one update, a rejected one gives the rejected proposal
and one overrelaxation.  Its count is (2 - acceptance) x V/2 per class pass,
with the heatbath class acceptance measured over the timed steps.
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
HB_TRAFFIC = {("fp32", 4, "grouped"): 374.0e6, ("fp32", 4, "interleaved"): 408.0e6}


def cpu_baseline(order, target_s=12.0):
    """The oracle (plain FP64 C, OpenMP over chains) on a bounded sample of the
    same workload: one L=20 chain per thread from the oracle's hot start,
    sweeps (heatbath + overrelaxation, in the given order) until ~target_s
    seconds of CPU work."""
    import oracle
    oracle.build(force=False)
    threads = oracle.num_threads()
    nch = threads
    th = oracle.hot_start(4, L, nch, SEED)
    E = np.array([oracle.energy(4, L, th[i]) for i in range(nch)])
    a = np.full(nch, 1.0)
    lo, hi = np.full(nch, -1e9), np.full(nch, 1e9)
    done = 0
    t0 = time.perf_counter()
    while True:
        E, _ = oracle.sweeps(4, L, th, a, lo, hi, np.arange(nch), E, 1, done, mode=oracle.MODE_RESTRICTED,
                             seed=SEED, order=oracle.SWEEP_INTERLEAVED if order == "interleaved"
                             else oracle.SWEEP_GROUPED)
        done += 1
        if time.perf_counter() - t0 > target_s:
            break
    dt = time.perf_counter() - t0
    upd = 2.0 * 4 * L ** 4 * nch * done
    return {"value": upd / dt, "unit": "link updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} restricted sweep(s) (8 heatbath + 8 overrelaxation passes, {order}) of {nch} "
                      f"L=20 chains, one per thread, from the oracle's hot start; {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--order", choices=["grouped", "interleaved"], default="grouped")
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
    n_rm = args.warmup + args.steps
    ctx = llr.Context(precision=prec, device=0)
    ctx.set_params(n_th=args.n_th, n_a=args.n_a, n_rm=n_rm, seed=SEED, replica_exchange=True, overlap=1.0,
                   recompute_every=10, eps=1e-4, approach_cap=20000)
    ctx.add_lattice(L, E_low, dE)
    ctx.bind_state()
    ctx.set_a(0, np.full(N_INT, 1.0))
    ctx.set_sweep_order(llr.SWEEP_INTERLEAVED if args.order == "interleaved" else llr.SWEEP_GROUPED)
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

    nsw = args.n_th + args.n_a
    dt = t1 - t0
    hb_acc_timed = float((ha - ha0).sum() / max((hp - hp0).sum(), 1))
    if args.order == "grouped":
        updates = 2.0 * 4 * V * N_INT * nsw * args.steps
    else:
        # 8 fused passes per sweep of V/2 class links each: 1 update per link
        # of an accepted class, 2 (proposal + overrelaxation) of a rejected one
        updates = (2.0 - hb_acc_timed) * 8 * (V // 2) * N_INT * nsw * args.steps
    value = updates / dt
    esz = 4 if prec == llr.FP32 else 8
    # algorithmic bytes of one heatbath pass: the pass reads the whole lattice
    # once (4V angles for V/2 class links = 8 angles per class link) and
    # writes one proposal per class link: 9 angles per class link (one
    # update); the fused pass of the interleaved order writes two (the
    # overrelaxed candidate and the overrelaxed old angle): 10 angles per
    # class link for its two updates
    per_link = 10 if args.order == "interleaved" else 9
    bytes_per_hb_launch = N_INT * (V // 2) * per_link * esz
    hb_avg_s = tm["hb_ms"] / max(tm["hb_n"], 1) / 1e3
    achieved = bytes_per_hb_launch / hb_avg_s / 1e9 if hb_avg_s > 0 else 0.0
    or_avg_s = tm["or_ms"] / max(tm["or_n"], 1) / 1e3
    out = {
        "metric": "link updates/s at 20^4x128 intervals",
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
                     "kernel": "heatbath class pass (k_hb)" if args.order == "grouped"
                               else "heatbath + overrelaxation class pass (k_hb, fused)",
                     "bytes_per_launch": bytes_per_hb_launch, "avg_launch_us": hb_avg_s * 1e6,
                     "overrelaxation_avg_launch_us": or_avg_s * 1e6},
        "acceptance": {"heatbath_class": hb_acc_timed,
                       "replica_exchange": float(ra / max(rp, 1))},
        "approach_sweeps": int(ap_sweeps[0]),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.order)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
