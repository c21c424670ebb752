#!/usr/bin/env python3
"""Benchmark of the HyperSARA primal-dual hot path on one MI355X.

A step is one iteration of Algorithm 2 (all operators: Phi, Phi^dagger, the
SARA dictionary, the nuclear, l2,1 and data-fidelity duals, the primal update)
over the whole synthetic 512 x 512 x 60 cube with uneven channels (workload
"cube512_L60"), batched in FP32 and replayed from a captured HIP graph.  Prints one JSON
line: the metric, its value and unit, the per-phase times, the roofline of the dominant
kernel, the FP64 comparison and the CPU-oracle baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--workload", default="cube512_L60")
    p.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-channels", type=int, default=16, help="channels of the oracle's CPU sample")
    p.add_argument("--phase-iters", type=int, default=5)
    p.add_argument("--tune-cache", default=None,
                   help="autotuner cache (JSON lines); default: the package's tuning_cache.jsonl")
    p.add_argument("--gram-mode", default="f64", choices=["f64", "f32", "bf16_split"])
    p.add_argument("--norm-iters", type=int, default=1000,
                   help="power iterations for the step-size norm (relative tolerance 1e-10)")
    p.add_argument("--precision", action="store_true",
                   help="per-operator error of the FP32 context against the FP64 one on the whole cube")
    p.add_argument("--drift-iters", type=int, default=0,
                   help="also run both contexts this many PD iterations from zero and report the drift")
    p.add_argument("--phases-only", action="store_true",
                   help="only the eager per-phase timing (for rocprofv3 kernel traces and counters)")
    p.add_argument("--calib-copy", action="store_true",
                   help="also run a 1 GiB device-to-device copy: the counter reference of known size")
    p.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                   help="offline: turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE) into "
                        "profiles/traffic.json and exit")
    return p.parse_args()


def algorithmic_bytes(cfg, M: int, r: int = 4):
    """Compulsory HBM bytes per iteration of each phase (r = bytes per real).

    N pixels, L channels, c = 2r bytes per complex.  The image is real, so its
    transform is conjugate-symmetric and only the half plane kx in [0, Kx/2] is
    compulsory: Hc = ny (nx + 1) cells per channel after the row pass and
    Gc = 2 ny (nx + 1) ~ 2N cells of the oversampled grid.
    """
    N, L, D, nb = cfg.N, cfg.L, 9, 8
    c = 2 * r
    Hc, Gc = cfg.ny * (cfg.nx + 1), 2 * cfg.ny * (cfg.nx + 1)
    lev = sum(0.25 ** k for k in range(4))            # fraction of pixels touched over 4 levels
    return {
        # read x, write and read the ny half-spectrum rows, write the half-plane grid
        "fft_fwd": L * (N * r + 2 * Hc * c + Gc * c),
        # grid read + per visibility: cell(4) frac(2r) theta(r) u(r) y(c) v(c) bin(4) write v(c)
        "degrid": L * Gc * c + M * (4 + 2 * r + r + r + c + c + 4 + c),
        "roots": 0,
        # v read/write, bin (the factor of each bin comes from the root solver)
        "dual_apply": M * (2 * c + 4),
        # per visibility cell, frac, v, theta; grid written once
        "grid": M * (4 + 2 * r + c + r) + L * Gc * c,
        "fft_adj": L * (Gc * c + 2 * Hc * c + N * r),
        "gram": 2 * L * N * r,
        "eig": 0,
        "backproject": 3 * L * N * r,
        # fused level kernels: X~ read once at level 1; per basis every level writes its four
        # subbands (sum N * lev) and levels 2..4 read the previous low-pass (N * (lev - 1))
        "psi_adj": L * N * r * (1 + nb * lev + nb * (lev - 1)),
        # read A (D bases), the 8 analysis outputs and Xt, write A
        "l21": L * N * r * (D + nb + 1 + D),
        # per basis each level reads its four subbands (N * lev) and levels 4..2 write the next
        # low-pass (N * (lev - 1)); the finest level adds the Dirac term and writes the sum once
        "psi": L * N * r * (nb * lev + nb * (lev - 1) + 2),
        # read X, P, At, D; write X, Xt
        "primal": 6 * L * N * r,
    }


def source_hash(*names) -> str:
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1806_04596_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# kernel that dominates each phase (the one the counters are read for)
PHASE_KERNEL = {"grid": "k_grid_pull", "degrid": "k_degrid_dual", "fft_fwd": "k_fft_cols_fwd",
                "fft_adj": "k_fft_cols_adj", "psi": "k_idwt_level", "psi_adj": "k_dwt_level", "eig": "k_eig",
                "l21": "k_l21", "primal": "k_primal", "gram": "k_gram", "backproject": "k_backproject"}
COPY_KERNEL = "__amd_rocclr_copyBuffer"
CALIB_BYTES = 1 << 30


def _counter_means(path: str, counter: str):
    """Mean counter value (KiB) per dispatch, by kernel (short name), from a rocprofv3 counter CSV."""
    import csv
    sums, counts = {}, {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            full = r["Kernel_Name"].replace("void ", "").split("(")[0]
            name = full.split("<")[0].split("::")[-1]
            if "<" in full:   # keep the element type apart: the FP64 comparator runs the same kernels
                name += "<" + full.split("<", 1)[1].split(",")[0].split(">")[0].strip() + ">"
            sums[name] = sums.get(name, 0.0) + float(r["Counter_Value"])
            counts[name] = counts.get(name, 0) + 1
    return {k: sums[k] / counts[k] for k in sums}, counts


def write_traffic(fetch_csv: str, write_csv: str, workload: str):
    """profiles/traffic.json: HBM bytes per launch of each phase's kernel on `workload`, each
    counter scaled by what it reads for a device-to-device copy of CALIB_BYTES (read once,
    write once)."""
    fm, fc = _counter_means(fetch_csv, "FETCH_SIZE")
    wm, wc = _counter_means(write_csv, "WRITE_SIZE")
    if COPY_KERNEL not in fm or COPY_KERNEL not in wm:
        raise SystemExit("the counter runs must include the copy reference (bench.py --calib-copy)")
    # the copy may be split over several dispatches: the reference is the total over one copy
    f_scale = CALIB_BYTES / (fm[COPY_KERNEL] * 1024 * fc[COPY_KERNEL] / 3)
    w_scale = CALIB_BYTES / (wm[COPY_KERNEL] * 1024 * wc[COPY_KERNEL] / 3)
    out = {"_reference": {"kernel": COPY_KERNEL, "bytes": CALIB_BYTES, "fetch_scale": f_scale, "write_scale": w_scale,
                          "workload": workload,
                          "note": "counter KiB per dispatch x 1024 x scale = HBM bytes per dispatch"}}
    for phase, kern0 in PHASE_KERNEL.items():
        kern = kern0 + "<float>"      # the FP32 problem the bench times
        if kern in fm and kern in wm:
            fb, wb = fm[kern] * 1024 * f_scale, wm[kern] * 1024 * w_scale
            out[phase] = {"kernel": kern, "fetch_bytes_per_launch": round(fb), "write_bytes_per_launch": round(wb),
                          "bytes_per_launch": round(fb + wb), "dispatches": fc[kern],
                          "src_hash": source_hash(PHASE_SRC[phase])}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


def traffic_from_profiles(kernel_phase: str, src_file: str, workload: str):
    """Measured HBM bytes per launch of a phase's kernel from committed rocprofv3
    counter summaries (profiles/traffic.json); None if absent, stale (kernel source
    changed since) or taken on another workload."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
        if t.get("_reference", {}).get("workload") != workload:
            return None
        ent = t.get(kernel_phase)
        if not ent or ent.get("src_hash") != source_hash(src_file):
            return None
        return ent["bytes_per_launch"]
    except Exception:
        return None


PHASE_SRC = {"fft_fwd": "k_nufft.hip", "degrid": "k_nufft.hip", "roots": "k_nufft.hip", "dual_apply": "k_nufft.hip",
             "grid": "k_nufft.hip", "fft_adj": "k_nufft.hip", "gram": "k_nuclear.hip", "eig": "k_nuclear.hip",
             "backproject": "k_nuclear.hip", "psi_adj": "k_wavelet.hip", "l21": "k_wavelet.hip",
             "psi": "k_wavelet.hip", "primal": "k_misc.hip"}


def cpu_baseline(cfg, inputs, n_ch: int):
    """The FP64 oracle, as it stands, timed for one PD iteration on the first n_ch
    channels of the same workload, its per-channel work mapped over a process pool of
    the host cores this run may use (at most 16); median of 3 runs, scaled by L/n_ch
    to the full cube's iterations per second."""
    import multiprocessing
    import statistics
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    import workloads as W
    from oracle import pd

    n_ch = max(1, min(n_ch, cfg.L))
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    sub = cfg.scaled(L=n_ch)
    inp = {"X0": inputs["X0"][:n_ch], "uv": inputs["uv"][:n_ch], "block_ptr": inputs["block_ptr"][:n_ch],
           "noise": inputs["noise"][:n_ch]}
    import contextlib
    lim = threadpool_limits(limits=cores) if threadpool_limits else contextlib.nullcontext()
    with lim, ProcessPoolExecutor(max_workers=cores, mp_context=multiprocessing.get_context("spawn")) as ex:
        op, _ = pd.build_problem(sub, inp, "density", pool=ex)
        st = W.make_state(sub, inp["X0"], [len(u) for u in inp["uv"]])
        prm = pd.Params(mu=0.01, tau=0.33)
        k3 = 1.0 / (max(len(t) for t in op.theta) * max(float(t.max()) for t in op.theta) ** 2)
        times = []
        for _ in range(3):
            ost = pd.State(X=st["X"], Xt=st["Xt"], P=st["P"], A=st["A"], v=st["v"],
                           eps=[e.copy() for e in op.eps], vartheta=[np.zeros(len(e), np.int64) for e in op.eps])
            t0 = time.perf_counter()
            pd.pd_iteration(ost, op, prm, (1.0, 1.0 / 9.0, k3), pool=ex)
            times.append(time.perf_counter() - t0)
    dt = statistics.median(times)
    scale = cfg.L / n_ch
    m_sub = sum(len(u) for u in inp["uv"])
    return {"value": 1.0 / (dt * scale), "unit": "iters/s", "cores": cores, "kind": "oracle",
            "sample": f"one PD iteration on channels 0..{n_ch - 1} of {cfg.name} ({m_sub} visibilities), "
                      f"per-channel work over {cores} worker processes, median of 3 runs = {dt:.2f} s "
                      f"(runs {', '.join(f'{t:.2f}' for t in times)} s), scaled by L/{n_ch} = {scale:.2f} "
                      f"to the full cube"}


def precision_report(prob, p64, cfg, X0, mu, tau, kappa3, drift_iters):
    """Error of the FP32 context (its Gram mode included) against the FP64 context, per
    operator on the whole cube: every input drawn in FP64 on the device (seeded), rounded
    to FP32, and the same FP32 values given to both sides.  Relative errors: the whole
    output and the largest per-channel one.  Then both contexts iterate from a zero state
    and the relative error of X is reported along the run (the drift)."""
    import numpy as np
    import torch
    dev = prob.device
    g = torch.Generator(device=dev).manual_seed(77)
    L = cfg.L

    def rnd(*shape, cplx=False):
        if cplx:
            x = torch.complex(torch.randn(*shape, generator=g, device=dev, dtype=torch.float64),
                              torch.randn(*shape, generator=g, device=dev, dtype=torch.float64))
            x32 = x.to(torch.complex64).contiguous()
            return x32, x32.to(torch.complex128).contiguous()
        x32 = torch.randn(*shape, generator=g, device=dev, dtype=torch.float64).float().contiguous()
        return x32, x32.double().contiguous()

    def errs(a32, a64, chan_axis=0, counts=None):
        a, b = a32.to(a64.dtype), a64
        tot = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
        if counts is not None:
            off = np.concatenate([[0], np.cumsum(counts)])
            per = [float(torch.linalg.vector_norm(a[off[l]:off[l + 1]] - b[off[l]:off[l + 1]]) /
                         torch.linalg.vector_norm(b[off[l]:off[l + 1]])) for l in range(L) if counts[l]]
        else:
            per = [float(torch.linalg.vector_norm(a.select(chan_axis, l) - b.select(chan_axis, l)) /
                         torch.linalg.vector_norm(b.select(chan_axis, l))) for l in range(L)]
        return {"rel": tot, "max_per_channel": max(per)}

    amp = float(X0.max())
    rep = {}
    x32, x64 = rnd(L, cfg.ny, cfg.nx)
    X32 = (X0.float() * (1 + 0.05 * x32)).contiguous()
    X64 = X32.double()
    rep["phi"] = errs(prob.phi(X32), p64.phi(X64), counts=prob.counts)
    y32, y64 = rnd(prob.M, cplx=True)
    rep["phi_adj"] = errs(prob.phi_adj(y32), p64.phi_adj(y64))
    rep["psi_adj"] = errs(prob.psi_adj(x32), p64.psi_adj(x64), chan_axis=1)
    c32, c64 = rnd(9, L, cfg.ny, cfg.nx)
    rep["psi"] = errs(prob.psi(c32), p64.psi(c64))
    a32, a64 = rnd(9, L, cfg.ny, cfg.nx)
    a32.mul_(0.05 * amp), a64.mul_(0.05 * amp)
    rep["dual_l21"] = errs(prob.dual_l21(a32, X32, mu), p64.dual_l21(a64, X64, mu), chan_axis=1)
    s = torch.linalg.svdvals(X64.reshape(L, -1).T).cpu().numpy()
    w = np.sort(np.random.default_rng(78).uniform(0.0, 0.5 * s[0], L))
    p32, p64_ = rnd(L, cfg.ny, cfg.nx)
    p32.mul_(0.05 * amp), p64_.mul_(0.05 * amp)
    rep["dual_nuclear"] = errs(prob.dual_nuclear(p32, X32, w), p64.dual_nuclear(p64_, X64, w))
    _, sig32 = prob.prox_nuclear(X32.clone(), w)
    _, sig64 = p64.prox_nuclear(X64.clone(), w)
    rep["singular_values"] = {"rel": float(np.linalg.norm(sig32 - sig64) / np.linalg.norm(sig64)),
                              "max_rel": float(np.max(np.abs(sig32 - sig64) / np.abs(sig64)))}
    v32, v64 = rnd(prob.M, cplx=True)
    v32.mul_(0.05), v64.mul_(0.05)
    rep["dual_data"] = errs(prob.dual_data(v32, X32), p64.dual_data(v64, X64), counts=prob.counts)
    torch.cuda.synchronize()
    if drift_iters > 0:
        for p in (prob, p64):
            z = torch.zeros(L, cfg.ny, cfg.nx, dtype=p.tdtype, device=dev)
            p.set_state(X=z, Xt=z.clone(), P=z.clone(), A=torch.zeros(9, L, cfg.ny, cfg.nx, dtype=p.tdtype, device=dev),
                        v=torch.zeros(p.M, dtype=p.cdtype, device=dev))
            p.pd_init(mu=mu, tau=tau, kappa3=kappa3)
        trace, done = [], 0
        for k in sorted({1, 10, 100, drift_iters}):
            if k > drift_iters:
                continue
            prob.iterate(k - done)
            p64.iterate(k - done)
            done = k
            e = errs(prob.get_state()["X"], p64.get_state()["X"])
            trace.append({"iteration": k, "X_rel": e["rel"], "X_max_per_channel": e["max_per_channel"],
                          "beta_f32": prob.stats()[0], "beta_f64": p64.stats()[0]})
        rep["drift_from_zero"] = trace
    torch.cuda.synchronize()
    return rep


def calib_copy():
    """Three device-to-device copies of CALIB_BYTES (the counter reference)."""
    import torch
    src = torch.empty(CALIB_BYTES, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def main():
    args = parse()
    if args.traffic_from:
        write_traffic(*args.traffic_from, args.workload)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus above 1 is not supported"}))
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as W
    from paper_1806_04596_amd.workload import build_problem

    cfg = W.CONFIGS[args.workload]
    t_setup = time.perf_counter()
    inputs = W.make_problem_inputs(cfg)
    # the data are formed once, with the FP64 instantiation's Phi, and shared by the FP32
    # problem, so that the FP32-vs-FP64 comparison runs on one problem.  The FP64 problem is
    # the plain comparator: the same kernels in FP64, launched channel by channel, default
    # decomposition, eager iterations (no graph)
    p64, _, host_data = build_problem(cfg, inputs, W.make_measurements, dtype="f64", per_channel=True)
    data = {"y_raw": host_data["y_raw"], "theta": host_data["theta"], "eps": host_data["eps"]}
    if args.no_fp64:
        p64.close()
        p64 = None
    prob, X0, _ = build_problem(cfg, inputs, W.make_measurements, dtype="f32", data=data, autotune=True,
                                tune_cache=args.tune_cache, gram_mode=args.gram_mode)
    info = prob.info()
    x0 = torch.as_tensor(W.synth.power_start(cfg), dtype=prob.tdtype, device=prob.device).contiguous()
    nrm, _, it_norm = prob.op_norm(x0, max_it=args.norm_iters, tol=1e-10)   # FP64 power iteration
    kappa3 = 1.0 / nrm
    mu, tau = 0.01, 0.33
    prob.pd_init(mu=mu, tau=tau, kappa3=kappa3)
    setup_s = time.perf_counter() - t_setup
    stream = prob.stream
    if args.phases_only:
        prob.profile_phases(1)
        phases = prob.profile_phases(args.phase_iters)
        torch.cuda.synchronize()
        if args.calib_copy:
            calib_copy()
        print(json.dumps({"phases_ms": {k: round(v, 4) for k, v in phases.items()}, "workload": cfg.name,
                          "tuning": prob.tuning(), "setup_s": round(setup_s, 1)}), flush=True)
        return

    # warm-up (the first call captures one iteration into a HIP graph)
    prob.iterate(args.warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    prob.iterate(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    value = args.steps / wall
    beta, _, _ = prob.stats()
    dg = prob.diag()

    # Phi and Phi^dagger throughput (library stream, HIP events)
    X = prob.get_state()["X"]
    Y = prob.phi(X)
    reps = 10
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(reps):
            prob.phi(X, Y)
        e1.record(stream)
    torch.cuda.synchronize()
    t_phi = e0.elapsed_time(e1) / reps / 1e3
    Xa = prob.empty_cube()
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(reps):
            prob.phi_adj(Y, Xa)
        e1.record(stream)
    torch.cuda.synchronize()
    t_adj = e0.elapsed_time(e1) / reps / 1e3

    # per-phase durations (HIP events between phases, same stream, eager launches)
    phases = prob.profile_phases(args.phase_iters)
    torch.cuda.synchronize()
    ab = algorithmic_bytes(cfg, prob.M)
    # the longest phase that spreads over the whole chip (the eigen-solve is one
    # work-group, latency-bound, and overlapped with the other branches in the graph)
    dom = max((k for k in phases if ab.get(k, 0) > 0), key=lambda k: phases[k])
    ach = ab[dom] / (phases[dom] * 1e-3) / 1e9 if ab[dom] > 0 else 0.0
    traffic = traffic_from_profiles(dom, PHASE_SRC[dom], cfg.name)
    roofline = {"bound": "hbm", "kernel": f"{PHASE_KERNEL.get(dom, dom)} ({dom} phase)", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": traffic,
                "algorithmic_bytes": int(ab[dom]), "avg_ms": round(phases[dom], 4)}
    iter_bytes = sum(ab.values())

    # FP64 comparison: same kernels in FP64 from the FP32 run's current state
    fp64 = None
    if not args.no_fp64:
        st = prob.get_state()
        torch.cuda.synchronize()
        del Y, Xa
        p64.pd_init(mu=mu, tau=tau, kappa3=kappa3)
        s64 = {k: v.to(torch.complex128 if v.is_complex() else torch.float64) for k, v in st.items()}
        p64.set_state(**s64)
        prob.set_state(**st)
        p64.iterate(1)
        prob.iterate(1)
        g32, g64 = prob.get_state()["X"].double(), p64.get_state()["X"]
        rel = float(torch.linalg.vector_norm(g32 - g64) / torch.linalg.vector_norm(g64))
        p64.iterate(2)
        torch.cuda.synchronize()
        n64 = max(5, args.steps // 5)
        t0 = time.perf_counter()
        p64.iterate(n64)
        torch.cuda.synchronize()
        v64 = n64 / (time.perf_counter() - t0)
        fp64 = {"kind": "plain FP64: per-channel launches, default decomposition, eager (no graph)",
                "iters_per_s": round(v64, 3), "fp32_speedup": round(value / v64, 3),
                "one_iter_rel_err_fp32_vs_fp64": rel}
        if args.precision or args.drift_iters:
            X0d = torch.as_tensor(X0, device=prob.device) if not torch.is_tensor(X0) else X0.to(prob.device)
            fp64["precision"] = precision_report(prob, p64, cfg, X0d, mu, tau, kappa3, args.drift_iters)
        del p64
    if args.calib_copy:
        calib_copy()
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, inputs, args.cpu_channels)

    out = {
        "metric": "PD iters/s + Φ/Φ† vis/s, batched FP32 vs plain FP64 at ≤1e-5 rel err",
        "value": round(value, 3), "unit": "iters/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 4), "gpu_ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.nx}x{cfg.ny} image, L={cfg.L} channels, "
                               f"{prob.M} visibilities (uneven per channel), {cfg.n_blocks} blocks/channel, "
                               f"Dirac+db1-db8 x 4 levels, KB 8x8 2x oversampled, FP32 batched graph replay",
                   "n_vis": prob.M, "gram_mode": args.gram_mode, "tuning": prob.tuning()},
        "phi_vis_per_s": round(prob.M / t_phi, 1), "phi_adj_vis_per_s": round(prob.M / t_adj, 1),
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "iteration_algorithmic_GB": round(iter_bytes / 1e9, 3),
        "iteration_effective_GBs": round(iter_bytes / (ms_per_step * 1e-3) / 1e9, 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64": fp64,
        "beta_last": beta, "eig_sweeps_last": dg["eig_sweeps"], "op_norm_iters": it_norm,
        "setup_s": round(setup_s, 1),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
