"""Definition of the visibility order used by the library (host logic, integer).

This is not a passage of the paper but a data layout of the GPU design; the
oracle holds its plain definition so the library's plan can be checked bit
for bit.  For channel l with oversampled grid Kx x Ky and square tile T:

* t = (u Kx, v Ky) (exact: K is a power of two and u is float32-representable);
  cell c = (floor(t_x) mod Kx, floor(t_y) mod Ky);
* tile = (c_y // T) * (Kx // T) + (c_x // T);
* region (0..8) = 3 * row_class + col_class, where for the in-tile offset o,
  class 0 if o < J/2 - 1, class 2 if o >= T - J/2, else 1 -- the visibilities
  whose kernel footprint reaches into the previous / next tile;
* bin = block * C + class_of(U), with C the number of distinct preconditioner
  values of the channel and class_of the rank of U_m among them (ascending);
* order = stable sort by (tile, region, bin), ties kept in input order.
"""
from __future__ import annotations

import numpy as np

J = 8


def cells(uv: np.ndarray, nx: int, ny: int):
    Kx, Ky = 2 * nx, 2 * ny
    cx = np.mod(np.floor(uv[:, 0] * Kx).astype(np.int64), Kx)
    cy = np.mod(np.floor(uv[:, 1] * Ky).astype(np.int64), Ky)
    return cx, cy


def region_class(o: np.ndarray, T: int) -> np.ndarray:
    cls = np.ones_like(o)
    cls[o < J // 2 - 1] = 0
    cls[o >= T - J // 2] = 2
    return cls


def bins(u: np.ndarray | None, block_ptr: np.ndarray, M: int):
    blk = np.zeros(M, dtype=np.int64)
    for b in range(len(block_ptr) - 1):
        blk[block_ptr[b]:block_ptr[b + 1]] = b
    if u is None:
        return blk, 1, np.array([1.0])
    vals, cls = np.unique(u, return_inverse=True)
    C = len(vals)
    return blk * C + cls, C, vals


def order(uv: np.ndarray, u: np.ndarray | None, block_ptr: np.ndarray, nx: int, ny: int, T: int):
    """Returns (perm, region_ptr): perm[k] = input index of the k-th visibility;
    region_ptr[(tile*9 + region)] = first position of that (tile, region)."""
    M = uv.shape[0]
    Kx, Ky = 2 * nx, 2 * ny
    cx, cy = cells(uv, nx, ny)
    tile = (cy // T) * (Kx // T) + (cx // T)
    reg = 3 * region_class(cy % T, T) + region_class(cx % T, T)
    b, _, _ = bins(u, block_ptr, M)
    key_major = tile * 9 + reg
    perm = np.lexsort((np.arange(M), b, key_major))
    ntr = (Kx // T) * (Ky // T) * 9
    counts = np.bincount(key_major, minlength=ntr)
    region_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return perm.astype(np.int64), region_ptr
