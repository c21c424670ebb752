"""Build a GPU ``Problem`` from seeded synthetic draws (sky, uv, noise).

The noiseless visibilities are simulated with this library's own Phi
(theta = 1) and the density preconditioner with its own host routine; the
noise recipe (``make_measurements``) is passed in by the caller so this
package does not depend on any test-side module.
"""
from __future__ import annotations

import numpy as np

from .problem import Problem, density_precond


def build_problem(cfg, inputs: dict, make_measurements, dtype: str = "f32", precond: str = "density",
                  tile: int = 0, device: int = 0, levels: int = 4, n_db: int = 8):
    """Returns (Problem, X0 device tensor, host dict of y_raw/theta/eps)."""
    uvs, bps = inputs["uv"], inputs["block_ptr"]
    chans = []
    for l in range(cfg.L):
        m = len(uvs[l])
        pre = density_precond(uvs[l], cfg.nx, cfg.ny) if (precond == "density" and m > 0) else None
        chans.append(dict(uv=uvs[l], y_raw=np.zeros(m, complex), theta=np.ones(m), block_ptr=bps[l],
                          eps=np.ones(len(bps[l]) - 1), precond=pre))
    prob = Problem(cfg.nx, cfg.ny, chans, dtype=dtype, levels=levels, n_db=n_db, tile=tile, device=device)
    torch = prob.torch
    X0 = torch.as_tensor(inputs["X0"], dtype=prob.tdtype, device=prob.device).contiguous()
    y0 = prob.phi(X0).cpu().numpy().astype(np.complex128)
    off = np.concatenate([[0], np.cumsum(prob.counts)])
    y0_list = [y0[off[l]:off[l + 1]] for l in range(cfg.L)]
    y_raw, theta, eps = make_measurements(y0_list, inputs["noise"], bps, cfg.isnr_db)
    for l in range(cfg.L):
        prob.set_data(l, y_raw[l], theta[l], eps[l])
    return prob, X0, {"y_raw": y_raw, "theta": theta, "eps": eps, "precond": [c["precond"] for c in chans]}
