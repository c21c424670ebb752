"""Definition of the visibility order used by the library (host logic, integer).

This is not a passage of the paper but a data layout of the GPU design; the
oracle holds its plain definition so the library's plan can be checked bit
for bit.  For channel l with oversampled grid Kx x Ky and square tile T:

* t = (u Kx, v Ky) (exact: K is a power of two and u is float32-representable);
  cell c = (floor(t_x) mod Kx, floor(t_y) mod Ky), fraction f = t - floor(t);
* Hermitian half plane (the image is real, so its transform at -t is the
  conjugate of that at t): when c_x + f_x > Kx/2 the visibility is reflected
  to -t.  Its taps floor(t) - 3 .. floor(t) + 4 mirror to the taps of cell
  ceil(-t) - 1 = (Kx - 1 - c_x, Ky - 1 - c_y) with fraction 1 - f in (0, 1];
  every cell then has c_x in [0, Kx/2];
* tile = (c_y // T) * (nx // T + 1) + (c_x // T) (nx // T + 1 tiles cover
  kx in [0, Kx/2]);
* region (0..8) = 3 * row_class + col_class, where for the in-tile offset o,
  class 0 if o < J/2 - 1, class 2 if o >= T - J/2, else 1 -- the visibilities
  whose kernel footprint reaches into the previous / next tile;
* bins: the (block, preconditioner value) pairs that occur; bin = the number
  of such pairs in the earlier blocks + the rank of U_m among the distinct
  values of its own block (ascending), so there are at most M + B of them;
* order = stable sort by (tile, region, bin, cell within the tile in raster
  order), ties kept in input order.
"""
from __future__ import annotations

import numpy as np

J = 8


def cells(uv: np.ndarray, nx: int, ny: int):
    """Half-plane cells (cx, cy) and the reflection flag of each visibility."""
    Kx, Ky = 2 * nx, 2 * ny
    tx, ty = uv[:, 0] * Kx, uv[:, 1] * Ky
    fx, fy = tx - np.floor(tx), ty - np.floor(ty)
    cx = np.mod(np.floor(tx).astype(np.int64), Kx)
    cy = np.mod(np.floor(ty).astype(np.int64), Ky)
    refl = (cx > nx) | ((cx == nx) & (fx > 0))
    cx = np.where(refl, Kx - 1 - cx, cx)
    cy = np.where(refl, Ky - 1 - cy, cy)
    return cx, cy, refl


def region_class(o: np.ndarray, T: int) -> np.ndarray:
    cls = np.ones_like(o)
    cls[o < J // 2 - 1] = 0
    cls[o >= T - J // 2] = 2
    return cls


def bins(u: np.ndarray | None, block_ptr: np.ndarray, M: int):
    """Bin of every visibility, the bin pointer of each block and each bin's value."""
    out = np.zeros(M, dtype=np.int64)
    ptr, vals = [0], []
    for b in range(len(block_ptr) - 1):
        s = slice(block_ptr[b], block_ptr[b + 1])
        if u is None:
            v, cls = (np.array([1.0]), np.zeros(block_ptr[b + 1] - block_ptr[b], np.int64)) \
                if block_ptr[b + 1] > block_ptr[b] else (np.zeros(0), np.zeros(0, np.int64))
        else:
            v, cls = np.unique(u[s], return_inverse=True)
        out[s] = ptr[-1] + cls
        ptr.append(ptr[-1] + len(v))
        vals.append(v)
    return out, np.array(ptr, dtype=np.int64), (np.concatenate(vals) if vals else np.zeros(0))


def order(uv: np.ndarray, u: np.ndarray | None, block_ptr: np.ndarray, nx: int, ny: int, T: int):
    """The plan's visibility order: by (tile, region, bin, cell within the tile in
    raster order, input index).  Returns (perm, region_ptr): perm[k] = input index
    of the k-th visibility;
    region_ptr[(tile*9 + region)] = first position of that (tile, region)."""
    M = uv.shape[0]
    Kx, Ky = 2 * nx, 2 * ny
    cx, cy, _ = cells(uv, nx, ny)
    tx = nx // T + 1
    tile = (cy // T) * tx + (cx // T)
    reg = 3 * region_class(cy % T, T) + region_class(cx % T, T)
    b, _, _ = bins(u, block_ptr, M)
    key_major = tile * 9 + reg
    cell_in_tile = (cy % T) * T + (cx % T)   # raster order of the cell within its tile
    perm = np.lexsort((np.arange(M), cell_in_tile, b, key_major))
    ntr = tx * (Ky // T) * 9
    counts = np.bincount(key_major, minlength=ntr)
    region_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return perm.astype(np.int64), region_ptr
