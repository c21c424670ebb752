"""Reconstruction quality against the sampling rate: a synthetic analogue of the
paper's Sec. 4.3 study (aSNR of LR, JAS, LRJAS, HyperSARA and SARA for SR in
[0.01, 1], InSNR in {20, 40} dB, L in {15, 60}).

For every (L, InSNR, SR) a seeded synthetic cube is drawn (10 extended sources,
so the cube's rank is below L; curved power-law spectra with emission lines), its
visibilities are simulated with the library's Phi on a Gaussian-density uv
coverage scaled per channel, and noise is added at the given InSNR.  Each method
then runs on the GPU from a zero state; every (re)weighted problem is solved
until the relative variation beta of Algorithm 2 falls below `--tol` (checked every
100 iterations, at most `--iters` iterations per problem):

* LR, JAS, LRJAS: one PD solve with all weights 1 (Sec. 4.2, eq:min-lr,
  eq:min-js and eq:min-problem with unit weights);
* HyperSARA: Algorithm 1: the unit-weight problem (as LRJAS), then `--reweights`
  reweighted problems (the paper uses 10), each warm-started;
* SARA: the weighted l1 prior applied to every channel independently, weights 1
  (the paper's SARA is also reweighted; reweighting per-channel l1 weights is
  not modelled here).

mu is mu_hat of Sec. 2.3 (the dirty cube), kappa3 comes from the power
iteration, tau = 0.33.  aSNR (Sec. 4.3) is the mean over channels of
20 log10(||x_l|| / ||x_l - x_hat_l||).

    python asnr_sweep.py [--L 15] [--isnr 40 20] [--sr 0.01 0.05 0.1 0.2 0.3] [--out file.json]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METHODS = ("lr", "jas", "lrjas", "hypersara", "sara")


def asnr(X_true: np.ndarray, X_hat: np.ndarray) -> float:
    """Mean over channels of 20 log10(||x_l|| / ||x_l - x_hat_l||) (Sec. 4.3)."""
    L = X_true.shape[0]
    t = X_true.reshape(L, -1)
    e = t - X_hat.reshape(L, -1)
    return float(np.mean(20.0 * np.log10(np.linalg.norm(t, axis=1) / np.linalg.norm(e, axis=1))))


def sweep_config(L: int, sr: float, isnr: float, n: int = 256, seed: int = 31):
    import workloads as W
    # 10 extended sources (widths 3-12 px, peaks log-uniform in [1e-3, 1]) on a 256^2 grid: the
    # cube's leading singular value is O(10^2), as for an extended image of unit peak
    return W.WorkloadConfig(f"sr{sr}_L{L}_in{isnr}", n, n, L, 1.4, 2.78, 10, True, max(1, int(round(sr * n * n))),
                            None, 4, float(isnr), seed, n_lines=2, src_sigma=(3.0, 12.0))


def run_point(cfg, methods, iters: int, reweights: int, tol: float = 1e-5, dtype: str = "f32", log=print):
    """aSNR of each method on one synthetic problem; returns {method: aSNR}."""
    import torch

    import workloads as W
    from paper_1806_04596_amd.workload import build_problem

    inp = W.make_problem_inputs(cfg)
    prob, _, _ = build_problem(cfg, inp, W.make_measurements, dtype=dtype)
    x0 = torch.as_tensor(W.synth.power_start(cfg), dtype=prob.tdtype, device=prob.device).contiguous()
    nrm, _, _ = prob.op_norm(x0, max_it=200, tol=1e-6)
    kappa3 = 1.0 / nrm
    mu, _ = prob.dirty_mu(want_cube=False)
    zeros = dict(X=prob.empty_cube().zero_(), Xt=prob.empty_cube().zero_(), P=prob.empty_cube().zero_(),
                 A=prob.empty_coef().zero_(), v=prob.empty_vis().zero_())
    out = {}
    chk = min(100, iters)
    for m in methods:
        prior = {"hypersara": "lrjas"}.get(m, m)
        prob.pd_init(mu=mu, tau=0.33, kappa3=kappa3, kappa2=1.0 / 9.0, prior=prior)
        prob.set_state(**zeros)
        t0 = time.perf_counter()
        X, rep = prob.solve(0, iters, beta_tol=tol, check_every=chk)
        n_it = rep["iterations"]
        if m == "hypersara" and reweights > 0:
            # reweights 1..K, warm-started from the unit-weight solution
            X, rep = prob.solve(reweights, iters, beta_tol=tol, check_every=chk)
            n_it += rep["iterations"]
        torch.cuda.synchronize()
        out[m] = asnr(inp["X0"], X.double().cpu().numpy())
        log(f"  {cfg.name} {m:10s} aSNR {out[m]:7.2f} dB  ({n_it} iterations, {time.perf_counter() - t0:.2f} s)")
    prob.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--L", type=int, nargs="+", default=[15])
    ap.add_argument("--isnr", type=float, nargs="+", default=[40.0, 20.0])
    ap.add_argument("--sr", type=float, nargs="+", default=[0.01, 0.02, 0.05, 0.1, 0.2, 0.3])
    ap.add_argument("--n", type=int, default=256, help="image edge (pixels)")
    ap.add_argument("--iters", type=int, default=3000, help="iteration cap per (re)weighted problem")
    ap.add_argument("--tol", type=float, default=1e-5, help="stop a problem when beta falls below this")
    ap.add_argument("--reweights", type=int, default=10)
    ap.add_argument("--methods", nargs="+", default=list(METHODS), choices=METHODS)
    ap.add_argument("--out", default=None, help="write the results as JSON")
    args = ap.parse_args()
    rows = []
    for L in args.L:
        for isnr in args.isnr:
            for sr in args.sr:
                cfg = sweep_config(L, sr, isnr, n=args.n)
                res = run_point(cfg, args.methods, args.iters, args.reweights, tol=args.tol)
                rows.append({"L": L, "isnr_db": isnr, "sr": sr, "aSNR_db": {k: round(v, 2) for k, v in res.items()}})
                print(json.dumps(rows[-1]), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"n": args.n, "iters": args.iters, "tol": args.tol, "reweights": args.reweights, "rows": rows}, f,
                      indent=1)


if __name__ == "__main__":
    main()
