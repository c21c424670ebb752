"""Long-run FP64 parity of Algorithm 2: the library's batched FP64 iteration (graph
replay) against the FP64 oracle after many iterations from a zero start, at the
FP64 bar.

* 64 x 64 x 4 (2048 visibilities per channel, iSNR 60 dB): 200 iterations, the
  oracle run in the test; every output compared element by element.
* 256 x 256 x 15 (0.5 N visibilities per channel in 4 blocks, iSNR 40 dB): 500
  iterations; the oracle's result (too slow to recompute in a test) is stored in
  tests/golden/long_run_cube256_L15.json by tests/golden/make_long_run.py, which
  calls only the oracle: sampled pixels of X, per-channel norms of X, P, A and v,
  the residual norms rho of every block and beta along the run.  The primal
  quantities are held to the FP64 bar; the duals, which integrate the rounding of
  every iteration, to t times that bar on their driving terms.

Both sides use the same data (formed by the oracle) and the same step sizes."""
import json
import os

import numpy as np
import pytest

import workloads as W
from gpu_cases import TOL, check_rel, gpu_case, host, oracle_case, rel, split, to_dev
from oracle import nufft, pd

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
GOLD = os.path.join(os.path.dirname(__file__), "golden", "long_run_cube256_L15.json")


def _zero_start(prob, w, kappa2, kappa3):
    import torch
    cube = torch.zeros(prob.L, prob.ny, prob.nx, dtype=prob.tdtype, device=prob.device)
    prob.set_state(X=cube, Xt=cube.clone(), P=cube.clone(), A=torch.zeros(prob.D, *cube.shape, dtype=prob.tdtype,
                                                                           device=prob.device),
                   v=torch.zeros(prob.M, dtype=prob.cdtype, device=prob.device))
    prob.pd_init(mu=0.01, tau=0.33, kappa3=kappa3, kappa1=1.0, kappa2=kappa2, w=w)


def test_pd_200_iterations_f64_vs_oracle():
    name, n = "cube64_L4", 200
    cfg, inp, op = oracle_case(name)
    prob, _, _ = gpu_case(name, "f64")
    nrm, _, _ = pd.op_norm_phi(op, W.synth.power_start(cfg), max_it=100, tol=1e-8)
    k3 = 0.98 / nrm
    w = np.ones(cfg.L)
    prm = pd.Params(mu=0.01, tau=0.33, kappa3=k3, w=w)
    st = pd.zero_state(op)
    for _ in range(n):
        st = pd.pd_iteration(st, op, prm, (1.0, 1.0 / op.D, k3))
    _zero_start(prob, w, 1.0 / op.D, k3)
    prob.iterate(n)
    g = {k: host(v) for k, v in prob.get_state().items()}
    beta, rho, _ = prob.stats()
    tol = TOL["f64"]
    for k in ("X", "Xt", "P"):
        e = max(rel(g[k][l], getattr(st, k)[l]) for l in range(cfg.L))
        print(f"{name} {n} iterations {k}: max per-channel rel err {e:.2e}", flush=True)
        assert e <= tol, (k, e)
    e = max(rel(g["A"][d, l], st.A[d, l]) for d in range(op.D) for l in range(cfg.L))
    print(f"{name} {n} iterations A: {e:.2e}", flush=True)
    assert e <= tol
    vg = split(g["v"], prob.counts)
    for l in range(cfg.L):
        check_rel(vg[l], st.v[l], tol, f"v[{l}]")
    check_rel(rho, np.concatenate(st.extra["rho"]), tol, "rho")
    # beta = ||X_t - X_{t-1}|| / ||X_t|| is a difference of consecutive iterates: the bar on
    # X (relative to ||X||) bounds its absolute error by 2 tol, whatever beta's size
    print(f"{name} {n} iterations beta: {beta:.15e} (oracle {st.beta:.15e})", flush=True)
    assert abs(beta - st.beta) <= 2 * tol


def test_pd_500_iterations_f64_vs_stored_oracle_run():
    if not os.path.exists(GOLD):
        pytest.skip("tests/golden/long_run_cube256_L15.json not generated")
    ref = json.load(open(GOLD))
    name = ref["case"]
    cfg, _, op = oracle_case(name)
    prob, _, _ = gpu_case(name, "f64")
    w = np.asarray(ref["w"])
    _zero_start(prob, w, ref["kappa2"], ref["kappa3"])
    beta = {}
    done = 0
    for k in sorted(int(s) for s in ref["beta"]):
        prob.iterate(k - done)
        done = k
        beta[k] = prob.stats()[0]
    assert done == ref["iterations"]
    g = {k: host(v) for k, v in prob.get_state().items()}
    _, rho, _ = prob.stats()
    tol = TOL["f64"]
    t = done
    idx = np.asarray(ref["sample_idx"])
    e = rel(g["X"].reshape(-1)[idx], np.asarray(ref["X_samples"]))
    print(f"{name} {t} iterations: sampled X rel err {e:.2e}", flush=True)
    assert e <= tol
    e = np.max(np.abs(np.array([np.linalg.norm(g["X"][l]) for l in range(cfg.L)]) - np.asarray(ref["X_norm"]))
               / np.asarray(ref["X_norm"]))
    print(f"{name} {t} iterations: per-channel norm of X rel err {e:.2e}", flush=True)
    assert e <= tol
    check_rel(rho, np.asarray(ref["rho"]), tol, "rho")
    # beta = ||X_t - X_{t-1}|| / ||X_t|| is a difference of consecutive iterates: the bar
    # on X (relative to ||X||) bounds its absolute error by 2 tol, whatever beta's size
    for k, b in beta.items():
        print(f"{name} beta at {k}: {b:.15e} (oracle {ref['beta'][str(k)]:.15e})", flush=True)
        assert abs(b - ref["beta"][str(k)]) <= 2 * tol, (k, b, ref["beta"][str(k)])
    # The duals of Algorithm 2 are running sums of their driving terms, projected: P of
    # Xt, A of Psi^dag Xt, v of U Phi Xt.  On the components the projections leave alone
    # they integrate the rounding differences of every iteration instead of contracting
    # them (the primal X does contract), so after t iterations a dual differs from the
    # oracle's by up to t times the FP64 bar on its driving term:
    # ||dDual|| / ||Dual|| <= t * tol * ||drive|| / ||Dual||.
    Xt = g["Xt"]
    drive = {"P": [np.linalg.norm(Xt[l]) for l in range(cfg.L)],
             "A": [3.0 * np.linalg.norm(Xt[l]) for l in range(cfg.L)],     # ||Psi^dag|| = sqrt(D) = 3
             "v": [np.linalg.norm(op.u[l] * nufft.phi(Xt[l], op.uv[l], op.theta[l])) for l in range(cfg.L)]}
    for key, vals in (("P", [np.linalg.norm(g["P"][l]) for l in range(cfg.L)]),
                      ("A", [np.linalg.norm(g["A"][:, l]) for l in range(cfg.L)]),
                      ("v", [np.linalg.norm(v) for v in split(g["v"], prob.counts)])):
        refn = np.asarray(ref[f"{key}_norm"])
        err = np.abs(np.asarray(vals) - refn) / refn
        bound = t * tol * np.asarray(drive[key]) / refn
        print(f"{name} {t} iterations: per-channel norm of {key} rel err {err.max():.2e} "
              f"(bound {bound.min():.2e} .. {bound.max():.2e})", flush=True)
        assert np.all(err <= bound), key
