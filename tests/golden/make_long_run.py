"""Writes long_run_cube256_L15.json: the FP64 oracle's state after 500 iterations of
Algorithm 2 on the 256 x 256 x 15 workload (0.5 N visibilities per channel in 4 blocks,
iSNR 40 dB), started from zero, with the step sizes of Sec. 3.4 (kappa3 from the oracle's
power iteration).  Calls only the oracle and the seeded input generators; the GPU test
compares the library's FP64 iteration with it on sampled pixels and on per-channel
norms.  Run from the repository root:  python tests/golden/make_long_run.py"""
import json
import multiprocessing
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import pd  # noqa: E402

CASE, ITERS, SAMPLES = "cube256_L15", 500, 2048
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "long_run_cube256_L15.json")


def main(workers: int = 6):
    cfg = W.CONFIGS[CASE]
    inp = W.make_problem_inputs(cfg)
    with ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("spawn")) as ex:
        op, _ = pd.build_problem(cfg, inp, "density", pool=ex)
        nrm, _, _ = pd.op_norm_phi(op, W.synth.power_start(cfg), max_it=100, tol=1e-8)
        kappa3 = 0.98 / nrm
        L, ny, nx = cfg.L, cfg.ny, cfg.nx
        prm = pd.Params(mu=0.01, tau=0.33, kappa3=kappa3, w=np.ones(L))
        st = pd.zero_state(op)
        beta = {}
        t0 = time.time()
        for k in range(1, ITERS + 1):
            st = pd.pd_iteration(st, op, prm, (1.0, 1.0 / op.D, kappa3), pool=ex)
            if k in (1, 10, 100, ITERS):
                beta[str(k)] = st.beta
            if k % 25 == 0:
                print(f"iteration {k}: beta {st.beta:.3e} ({time.time() - t0:.0f} s)", flush=True)
    rng = np.random.default_rng(2024)
    idx = np.sort(rng.choice(L * ny * nx, SAMPLES, replace=False))
    out = {"_source": "written by tests/golden/make_long_run.py from the FP64 oracle (Algorithm 2, "
                      "zero start, non-adaptive bounds)",
           "case": CASE, "iterations": ITERS, "mu": prm.mu, "tau": prm.tau, "kappa2": 1.0 / op.D,
           "kappa3": kappa3, "w": [1.0] * L,
           "sample_idx": idx.tolist(), "X_samples": st.X.reshape(-1)[idx].tolist(),
           "X_norm": [float(np.linalg.norm(st.X[l])) for l in range(L)],
           "P_norm": [float(np.linalg.norm(st.P[l])) for l in range(L)],
           "A_norm": [float(np.linalg.norm(st.A[:, l])) for l in range(L)],
           "v_norm": [float(np.linalg.norm(v)) for v in st.v],
           "rho": [float(r) for rr in st.extra["rho"] for r in rr],
           "beta": beta}
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(OUT)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 6)
