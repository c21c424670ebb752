"""Shared builders for the GPU parity tests.

Both sides start from the same seeded draws (workloads).  The data y_raw,
theta and eps are formed once, by the oracle (its FP64 Phi and the noise
recipe), and handed to the library, so both sides solve the same problem;
each side computes its own density preconditioner and visibility order.
"""
from __future__ import annotations

import functools

import numpy as np

import workloads as W
from oracle import pd

TOL = {"f64": 1e-12, "f32": 1e-5}


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rel_per_channel(a, b) -> float:
    return max(rel(a[l], b[l]) for l in range(len(b)))


_yraw = {}


@functools.lru_cache(maxsize=None)
def oracle_case(name: str, precond: str = "density", **over):
    cfg = W.CONFIGS[name].scaled(**over) if over else W.CONFIGS[name]
    inp = W.make_problem_inputs(cfg)
    oprob, y_raw = pd.build_problem(cfg, inp, precond)
    _yraw[(name, precond, tuple(sorted(over.items())))] = y_raw
    return cfg, inp, oprob


def oracle_data(name: str, precond: str = "density", **over):
    """The oracle's y_raw, theta and eps of a case (to hand to the library)."""
    _, _, op = oracle_case(name, precond, **over)
    y_raw = _yraw[(name, precond, tuple(sorted(over.items())))]
    return {"y_raw": y_raw, "theta": op.theta, "eps": op.eps}


_gpu_cache = {}


def gpu_case(name: str, dtype: str, precond: str = "density", tile: int = 0, gram_mode: str = "f64",
             per_channel: bool = False, **over):
    key = (name, dtype, precond, tile, gram_mode, per_channel, tuple(sorted(over.items())))
    if key not in _gpu_cache:
        from paper_1806_04596_amd.workload import build_problem
        cfg, inp, _ = oracle_case(name, precond, **over)
        prob, X0, host = build_problem(cfg, inp, W.make_measurements, dtype=dtype, precond=precond, tile=tile,
                                       data=oracle_data(name, precond, **over), gram_mode=gram_mode,
                                       per_channel=per_channel)
        _gpu_cache[key] = (prob, X0, host)
    return _gpu_cache[key]


def to_dev(prob, a, complex_=False):
    import torch
    dt = prob.cdtype if complex_ else prob.tdtype
    return torch.as_tensor(np.ascontiguousarray(a), device=prob.device).to(dt).contiguous()


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


def split(v, counts):
    off = np.concatenate([[0], np.cumsum(counts)])
    return [v[off[l]:off[l + 1]] for l in range(len(counts))]


def check_rel(a, b, tol, what=""):
    err = rel(a, b)
    assert err <= tol, f"{what}: rel err {err:.3e} > {tol:.1e}"
    return err


def check_rel_pc(a, b, tol, what=""):
    err = rel_per_channel(a, b)
    assert err <= tol, f"{what}: per-channel rel err {err:.3e} > {tol:.1e}"
    return err
