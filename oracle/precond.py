"""Sampling-density preconditioner U (Sec. 3.3) -- plain definition.

The paper sets U_l^b diagonal, strictly positive and inversely proportional to
the density of the Fourier sampling around each probed mode, without giving
the construction.  Reading taken (integer, hence exactly reproducible):
the uv plane of channel l is cut into the nx x ny cells of the image's own
Fourier grid (cell width 1/nx cycles/pixel); n_m counts the visibilities of
channel l (all blocks) in the cell of visibility m, cell = (floor(u nx) mod nx,
floor(v ny) mod ny); U_m = 1 / n_m.

Parity: pinned against a dictionary count (tests/test_oracle_misc.py).
"""
from __future__ import annotations

import numpy as np


def density_counts(uv: np.ndarray, nx: int, ny: int) -> np.ndarray:
    cx = np.mod(np.floor(uv[:, 0] * nx).astype(np.int64), nx)
    cy = np.mod(np.floor(uv[:, 1] * ny).astype(np.int64), ny)
    key = cy * nx + cx
    _, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
    return cnt[inv]


def density_precond(uv: np.ndarray, nx: int, ny: int) -> np.ndarray:
    return 1.0 / density_counts(uv, nx, ny).astype(np.float64)
