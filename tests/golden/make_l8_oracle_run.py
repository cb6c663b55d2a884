"""Writes tests/golden/l8_oracle_run_fp64.json: the FP64 oracle's full run of
the L=8 case (32 intervals from u = 0.55 with dE = 0.005 6V, N_TH = 200,
N_A = 500, N_RM = 50, a^(0) = 1, hot start, seed 1509083910) and its
reconstruction of <u>(beta), C_V(beta) on beta in [0.98, 1.04] and of beta_c.
Calls only the oracle (Algorithm 1; eqs. (kk3a), (l19)-(l20))."""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle  # noqa: E402


def main():
    L, d = 8, 4
    V6 = 6 * L ** 4
    dE = 0.005 * V6
    E_low = 0.55 * V6 + dE * np.arange(32)
    seed = 1509083910
    t0 = time.time()
    r = oracle.llr_run(d, L, E_low, dE, 1.0, n_th=200, n_a=500, n_rm=50, seed=seed, approach_cap=20000)
    cen = E_low + 0.5 * dE
    beta = np.linspace(0.98, 1.04, 61)
    lr, u, cv = oracle.reconstruct(cen, r["a"], dE, V6, beta)
    bc, pk = oracle.beta_c(cen, r["a"], dE, V6, 0.98, 1.04)
    out = {"L": L, "n_intervals": 32, "dE": dE, "E_low": E_low.tolist(), "seed": seed,
           "n_th": 200, "n_a": 500, "n_rm": 50, "a": r["a"].tolist(), "a_hist": r["a_hist"].tolist(),
           "conv_iter": r["conv_iter"].tolist(), "approach_sweeps": r["approach_sweeps"],
           "beta": beta.tolist(), "u_mean": u.tolist(), "cv": cv.tolist(), "ln_rho": lr.tolist(),
           "beta_c": bc, "cv_peak": pk, "oracle_seconds": time.time() - t0, "threads": oracle.num_threads()}
    with open(os.path.join(HERE, "l8_oracle_run_fp64.json"), "w") as f:
        json.dump(out, f)
    print("done", time.time() - t0)


if __name__ == "__main__":
    main()
