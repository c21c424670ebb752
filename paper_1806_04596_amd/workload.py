"""Build a GPU ``Problem`` from seeded synthetic draws (sky, uv, noise).

The data y_raw, theta and eps are either given by the caller or formed here:
noiseless visibilities from this library's own Phi (theta = 1), then the noise
recipe (``make_measurements``) passed in by the caller, so this package does
not depend on any test-side module.  The density preconditioner comes from the
library's own host routine.
"""
from __future__ import annotations

import numpy as np

from .problem import Problem, density_precond


def build_problem(cfg, inputs: dict, make_measurements, dtype: str = "f32", precond: str = "density",
                  tile: int = 0, device: int = 0, levels: int = 4, n_db: int = 8, data=None, **desc):
    """Returns (Problem, X0 device tensor, host dict of y_raw/theta/eps).

    data: optional dict of per-channel lists y_raw, theta, eps given by the caller
    (then nothing is simulated here); channels missing from data["channels"] (all
    when that key is absent) take the listed entries in order.  desc: further
    Problem options (gram_mode, ...)."""
    uvs, bps = inputs["uv"], inputs["block_ptr"]
    chans = []
    for l in range(cfg.L):
        m = len(uvs[l])
        pre = density_precond(uvs[l], cfg.nx, cfg.ny) if (precond == "density" and m > 0) else None
        chans.append(dict(uv=uvs[l], y_raw=np.zeros(m, complex), theta=np.ones(m), block_ptr=bps[l],
                          eps=np.ones(len(bps[l]) - 1), precond=pre))
    prob = Problem(cfg.nx, cfg.ny, chans, dtype=dtype, levels=levels, n_db=n_db, tile=tile, device=device, **desc)
    torch = prob.torch
    X0 = torch.as_tensor(inputs["X0"], dtype=prob.tdtype, device=prob.device).contiguous()
    sel = list(range(cfg.L))
    if data is not None:
        sel = list(data.get("channels", range(cfg.L)))
        y_raw, theta, eps = data["y_raw"], data["theta"], data["eps"]
        given = set(sel)
        rest = [l for l in range(cfg.L) if l not in given]
    else:
        rest = sel
    if rest:
        # the remaining channels: noiseless data from this library's Phi, then the noise recipe
        y0 = prob.phi(X0).cpu().numpy().astype(np.complex128)
        off = np.concatenate([[0], np.cumsum(prob.counts)])
        y0_list = [y0[off[l]:off[l + 1]] for l in rest]
        yr, th, ep = make_measurements(y0_list, [inputs["noise"][l] for l in rest], [bps[l] for l in rest],
                                       cfg.isnr_db)
    out = {"y_raw": [None] * cfg.L, "theta": [None] * cfg.L, "eps": [None] * cfg.L}
    if data is not None:
        for j, l in enumerate(sel):
            out["y_raw"][l], out["theta"][l], out["eps"][l] = y_raw[j], theta[j], eps[j]
    for j, l in enumerate(rest):
        out["y_raw"][l], out["theta"][l], out["eps"][l] = yr[j], th[j], ep[j]
    for l in range(cfg.L):
        prob.set_data(l, out["y_raw"][l], out["theta"][l], out["eps"][l])
    out["precond"] = [c["precond"] for c in chans]
    return prob, X0, out
