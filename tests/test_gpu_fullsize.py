"""Parity at full size: the benchmark's 512x512x60 uneven cube (16.3 M
visibilities, 8 blocks per channel) and the 1024x1024x32 cube (33.5 M
visibilities, 4 blocks per channel), in FP32, built and launched exactly as the
benchmark builds them (automatic tile, batched kernels, graph replay).

The data y_raw, theta and eps of every channel are formed once by the oracle
(FP64) and handed to the library, so both sides solve the same problem.
Channel-separable outputs (Phi, Phi^dagger, Psi^dagger, Psi, the data-fidelity
dual) are compared element by element with the oracle on sampled channels
(the smallest, a middle and the largest); the channel-coupled nuclear dual and
one whole PD iteration are compared on the whole cube.  The 1024 cube runs with the
nuclear prox's Gram matrix as a BF16 split (FP32 accumulation, FP64 eigen-solve);
every test prints its relative errors, the per-operator error table of that
precision pattern.  The oracle's
per-channel work runs in a process pool (channels are independent)."""
import multiprocessing
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

import workloads as W
from oracle import nufft, pd, prox, wavelets
from gpu_cases import TOL, check_rel, host, rel, split, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _workers():
    return max(1, min(12, (os.cpu_count() or 2) - 1))


@pytest.fixture(scope="module")
def pool():
    with ProcessPoolExecutor(max_workers=_workers(), mp_context=multiprocessing.get_context("spawn")) as ex:
        yield ex


# the 1024 x 1024 x 32 cube runs in the mixed-precision pattern: FP32 operators, the
# Gram matrix of the nuclear prox as a BF16 split with FP32 accumulation, FP64 eigen-solve
GRAM = {"cube512_L60": "f64", "cube1024_L32": "bf16_split"}


def _report(CFG, what, err):
    print(f"{CFG.name} [{GRAM[CFG.name]} Gram] {what}: rel err {err:.2e}", flush=True)


@pytest.fixture(scope="module", params=["cube512_L60", "cube1024_L32"])
def big(request, pool):
    from paper_1806_04596_amd.workload import build_problem
    CFG = W.CONFIGS[request.param]
    inp = W.make_problem_inputs(CFG)
    counts = np.array([len(u) for u in inp["uv"]])
    S = sorted({int(np.argmin(counts)), CFG.L // 2, int(np.argmax(counts))})
    op, y_raw = pd.build_problem(CFG, inp, pool=pool)
    prob, X0, hd = build_problem(CFG, inp, W.make_measurements, dtype="f32",
                                 data={"y_raw": y_raw, "theta": op.theta, "eps": op.eps},
                                 gram_mode=GRAM[CFG.name])
    print(f"{CFG.name} full size: sampled channels {S}, M = {prob.M}", flush=True)
    yield {"cfg": CFG, "inp": inp, "prob": prob, "S": S, "op": op, "y_raw": y_raw}
    prob.close()


def test_phi_full_size(big):
    prob, S, op, inp = big["prob"], big["S"], big["op"], big["inp"]
    rng = np.random.default_rng(40)
    X = inp["X0"] + 0.05 * inp["X0"].max() * rng.standard_normal(inp["X0"].shape)
    Y = split(host(prob.phi(to_dev(prob, X))), prob.counts)
    for l in S:
        ref = nufft.phi(X[l], op.uv[l], op.theta[l])
        _report(big["cfg"], f"Phi channel {l}", check_rel(Y[l], ref, TOL["f32"], f"Phi channel {l}"))


def test_phi_adj_full_size(big):
    CFG = big["cfg"]
    prob, S, op = big["prob"], big["S"], big["op"]
    rng = np.random.default_rng(41)
    y = rng.standard_normal(prob.M) + 1j * rng.standard_normal(prob.M)
    X = host(prob.phi_adj(to_dev(prob, y, complex_=True)))
    ys = split(y, prob.counts)
    for l in S:
        ref = nufft.phi_adj(ys[l], op.uv[l], op.theta[l], CFG.ny, CFG.nx)
        _report(CFG, f"Phi^dag channel {l}", check_rel(X[l], ref, TOL["f32"], f"Phi^dag channel {l}"))


def test_psi_full_size(big):
    CFG = big["cfg"]
    prob, S = big["prob"], big["S"]
    rng = np.random.default_rng(42)
    X = rng.standard_normal((CFG.L, CFG.ny, CFG.nx))
    C = host(prob.psi_adj(to_dev(prob, X)))
    ref = wavelets.psi_adj(X[S])
    for j, l in enumerate(S):
        e = max(check_rel(C[d, l], ref[d, j], TOL["f32"], f"Psi^dag basis {d} channel {l}") for d in range(9))
        _report(CFG, f"Psi^dag channel {l} (max over bases)", e)
    Cr = rng.standard_normal((9, CFG.L, CFG.ny, CFG.nx)).astype(np.float32)
    Xs = host(prob.psi(to_dev(prob, Cr)))
    ref = wavelets.psi(Cr[:, S].astype(np.float64))
    for j, l in enumerate(S):
        _report(CFG, f"Psi channel {l}", check_rel(Xs[l], ref[j], TOL["f32"], f"Psi channel {l}"))


def test_dual_nuclear_full_size(big):
    CFG = big["cfg"]
    prob, inp = big["prob"], big["inp"]
    rng = np.random.default_rng(43)
    X = inp["X0"] + 0.01 * inp["X0"].max() * rng.standard_normal(inp["X0"].shape)
    P = 0.05 * inp["X0"].max() * rng.standard_normal(X.shape)
    s = np.linalg.svd(X.reshape(CFG.L, -1).T, compute_uv=False)
    w = np.sort(rng.uniform(0.0, 0.5 * s[0], CFG.L))
    Pd = host(prob.dual_nuclear(to_dev(prob, P), to_dev(prob, X), w))
    ref = prox.dual_nuclear(P, X, w, "gram")
    _report(CFG, "nuclear dual P (whole cube)", check_rel(Pd, ref, TOL["f32"], "P"))


def test_dual_data_full_size(big):
    prob, S, op, inp = big["prob"], big["S"], big["op"], big["inp"]
    rng = np.random.default_rng(44)
    Xt = inp["X0"] + 0.05 * inp["X0"].max() * rng.standard_normal(inp["X0"].shape)
    v = 0.05 * (rng.standard_normal(prob.M) + 1j * rng.standard_normal(prob.M))
    vd = host(prob.dual_data(to_dev(prob, v, complex_=True), to_dev(prob, Xt)))
    vg, vs = split(vd, prob.counts), split(v, prob.counts)
    for l in S:
        vbar = vs[l] + op.u[l] * nufft.phi(Xt[l], op.uv[l], op.theta[l])
        bp = op.block_ptr[l]
        vr = np.empty_like(vbar)
        for b in range(len(bp) - 1):
            sl = slice(bp[b], bp[b + 1])
            vr[sl], _ = prox.dual_data_block(vbar[sl], op.y[l][sl], op.u[l][sl], op.eps[l][b])
        _report(big["cfg"], f"data dual v channel {l}", check_rel(vg[l], vr, TOL["f32"], f"v channel {l}"))


def _kappa3(op):
    return 1.0 / (max(len(t) for t in op.theta) * max(float(np.max(t)) for t in op.theta if len(t)) ** 2)


def test_pd_iteration_full_size_vs_oracle(big, pool):
    """One graph-replayed FP32 iteration of Algorithm 2 on the whole cube, from a shared
    state, against one oracle iteration: X, X~, P, A element by element per channel, v per
    channel, and the residual norms rho of every block."""
    CFG = big["cfg"]
    prob, op, inp = big["prob"], big["op"], big["inp"]
    st = W.make_state(CFG, inp["X0"], prob.counts)
    w = np.linspace(0.2, 1.0, CFG.L)
    k3 = _kappa3(op)
    prm = pd.Params(mu=0.01, tau=0.33, kappa3=k3, w=w)
    ost = pd.State(X=st["X"], Xt=st["Xt"], P=st["P"], A=st["A"], v=st["v"],
                   eps=[e.copy() for e in op.eps], vartheta=[np.zeros(len(e), np.int64) for e in op.eps])
    ref = pd.pd_iteration(ost, op, prm, (1.0, 1.0 / 9.0, k3), pool=pool)
    prob.set_state(X=to_dev(prob, st["X"]), Xt=to_dev(prob, st["Xt"]), P=to_dev(prob, st["P"]),
                   A=to_dev(prob, st["A"]), v=to_dev(prob, np.concatenate(st["v"]), complex_=True))
    prob.pd_init(mu=0.01, tau=0.33, kappa3=k3, kappa2=1.0 / 9.0, w=w)
    prob.iterate(1)
    g = prob.get_state()
    tol = TOL["f32"]
    for k in ("X", "Xt", "P"):
        a = host(g[k])
        err = max(rel(a[l], getattr(ref, k)[l]) for l in range(CFG.L))
        _report(CFG, f"one iteration {k} (max per channel)", err)
        assert err <= tol, (k, err)
    A = host(g["A"])
    err = max(rel(A[d, l], ref.A[d, l]) for d in range(9) for l in range(CFG.L))
    _report(CFG, "one iteration A (max per basis and channel)", err)
    assert err <= tol
    vg = split(host(g["v"]), prob.counts)
    err = max(rel(vg[l], ref.v[l]) for l in range(CFG.L))
    _report(CFG, "one iteration v (max per channel)", err)
    assert err <= tol
    _, rho, _ = prob.stats()
    err = rel(rho, np.concatenate(ref.extra["rho"]))
    _report(CFG, "one iteration rho", err)
    assert err <= tol


def test_pd_iteration_full_size_properties(big):
    """Graph replay (as timed by the benchmark) equals the eager iteration bit
    for bit; X >= 0; X~ = 2X - X_prev exactly; beta = ||X - X_prev|| / ||X||;
    the FP32 iteration agrees with the FP64 instantiation to 1e-5."""
    CFG = big["cfg"]
    import torch
    from paper_1806_04596_amd.workload import build_problem
    prob, inp, op = big["prob"], big["inp"], big["op"]
    amp = float(inp["X0"].max())
    g = torch.Generator(device="cpu").manual_seed(45)

    def r(*shape):
        return torch.randn(*shape, generator=g, dtype=torch.float64)
    X = (torch.as_tensor(inp["X0"]) * (1 + 0.2 * r(*inp["X0"].shape))).clamp_min(0)
    st = {"X": X, "Xt": X + 0.02 * amp * r(*X.shape), "P": 0.05 * amp * r(*X.shape),
          "A": 0.05 * amp * r(9, *X.shape), "v": 0.05 * torch.complex(r(prob.M), r(prob.M))}
    kappa3 = 1.0 / prob.op_norm(to_dev(prob, W.synth.power_start(CFG)), max_it=30, tol=1e-6)[0]

    def run(p, eager):
        dev = {k: t.to(p.device, p.cdtype if k == "v" else p.tdtype).contiguous() for k, t in st.items()}
        p.set_state(**dev)
        p.pd_init(mu=0.01, tau=0.33, kappa3=kappa3, kappa2=1.0 / 9.0)
        if eager:
            p.profile_phases(1)
        else:
            p.iterate(1)
        out = p.get_state()
        return out, p.stats()[0], dev["X"]

    a, beta_a, Xp = run(prob, eager=False)
    b, beta_b, _ = run(prob, eager=True)
    for k in a:
        assert torch.equal(a[k], b[k]), k
    assert beta_a == beta_b
    assert bool((a["X"] >= 0).all())
    assert torch.equal(a["Xt"], 2 * a["X"] - Xp)
    bref = float((a["X"].double() - Xp.double()).norm() / a["X"].double().norm())
    assert abs(beta_a - bref) <= 1e-6 * bref
    p64, _, _ = build_problem(CFG, inp, W.make_measurements, dtype="f64",
                              data={"y_raw": big["y_raw"], "theta": op.theta, "eps": op.eps})
    c, _, _ = run(p64, eager=False)
    for k in ("X", "Xt", "P", "A"):
        err = rel(host(a[k]), host(c[k]))
        assert err <= TOL["f32"], (k, err)
    p64.close()
