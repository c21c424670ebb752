"""Pins of the preconditioner density and of the visibility-order definition."""
from collections import Counter
from fractions import Fraction
import math

import numpy as np

import workloads as W
from oracle import binning, precond


def test_density_counts_vs_dictionary_count():
    cfg = W.CONFIGS["cube64_L5"]
    uvs, _ = W.synth.make_uv(cfg)
    for uv in uvs[:2]:
        n = precond.density_counts(uv, cfg.nx, cfg.ny)
        keys = [(int(np.floor(a * cfg.nx)) % cfg.nx, int(np.floor(b * cfg.ny)) % cfg.ny) for a, b in uv]
        cnt = Counter(keys)
        assert np.array_equal(n, [cnt[k] for k in keys])
        assert np.array_equal(precond.density_precond(uv, cfg.nx, cfg.ny), 1.0 / n)


def test_order_definition_properties():
    cfg = W.CONFIGS["cube64_L5"]
    uvs, bps = W.synth.make_uv(cfg)
    T = 16
    for uv, bp in zip(uvs[:2], bps[:2]):
        u = precond.density_precond(uv, cfg.nx, cfg.ny)
        perm, rptr = binning.order(uv, u, bp, cfg.nx, cfg.ny, T)
        M = len(uv)
        assert np.array_equal(np.sort(perm), np.arange(M))
        cx, cy, _ = binning.cells(uv, cfg.nx, cfg.ny)
        tile = (cy // T) * (cfg.nx // T + 1) + cx // T
        reg = 3 * binning.region_class(cy % T, T) + binning.region_class(cx % T, T)
        key = tile * 9 + reg
        assert np.all(np.diff(key[perm]) >= 0)
        for k in range(len(rptr) - 1):
            seg = perm[rptr[k]:rptr[k + 1]]
            assert np.all(key[seg] == k)
        # regions: offsets within the tile
        assert np.all((cx % T)[reg % 3 == 0] < 3) and np.all((cx % T)[reg % 3 == 2] >= T - 4)
        # within a (tile, region): by bin, then by the cell's raster position in the
        # tile, then by input index (strictly increasing tuples)
        b, _, _ = binning.bins(u, bp, M)
        for k in range(len(rptr) - 1):
            seg = perm[rptr[k]:rptr[k + 1]]
            keys = [(int(b[m]), int((cy[m] % T) * T + cx[m] % T), int(m)) for m in seg]
            assert all(keys[i] < keys[i + 1] for i in range(len(keys) - 1))


def test_region_reaches_neighbour_exactly():
    # a visibility at in-tile offset o has taps o-3 .. o+4; it reaches the
    # previous tile iff o < 3 and the next tile iff o >= T - 4
    T = 16
    o = np.arange(T)
    cls = binning.region_class(o, T)
    assert np.array_equal(cls == 0, o - 3 < 0)
    assert np.array_equal(cls == 2, o + 4 >= T)


def test_half_plane_cells_by_exact_arithmetic():
    """Each visibility's half-plane cell is floor(p) of p = t mod K if that has
    kx <= Kx/2, else (the transform of a real image at -t is the conjugate of
    that at t) the cell whose 8 taps are the mirror images of the taps of t,
    ceil(p) - 1 of p = -t mod K; computed here in exact rational arithmetic."""
    nx, ny = 16, 16
    Kx, Ky = 2 * nx, 2 * ny
    rng = np.random.default_rng(5)
    uv = rng.uniform(-1.2, 1.2, (400, 2)).astype(np.float32).astype(np.float64)
    # on nodes, on the reflection line kx = Kx/2 and next to it, at 0
    uv = np.concatenate([uv, [[0.5, 0.25], [-0.5, -0.25], [0.5 + 2.0 ** -20, 0.1], [0.5 - 2.0 ** -20, 0.1],
                              [0.0, 0.0], [0.0, 0.5], [1 / 32, -1 / 32], [-1 / 32, 1 / 32]]])
    cx, cy, refl = binning.cells(uv, nx, ny)
    for m, (a, b) in enumerate(uv):
        px, py = (Fraction(a) * Kx) % Kx, (Fraction(b) * Ky) % Ky
        r = px > nx
        if r:
            px, py = (-px) % Kx, (-py) % Ky
        assert bool(refl[m]) == r, m
        if r:
            want = (math.ceil(px) - 1, math.ceil(py) - 1)
            want = (want[0], want[1] % Ky)
            # the taps of the mirror cell are the negated taps of t
            t0x, t0y = math.floor(Fraction(a) * Kx), math.floor(Fraction(b) * Ky)
            taps = {((-(t0x - 3 + i)) % Kx, (-(t0y - 3 + j)) % Ky) for i in range(8) for j in range(8)}
            assert taps == {((want[0] - 3 + i) % Kx, (want[1] - 3 + j) % Ky) for i in range(8) for j in range(8)}
        else:
            want = (int(px // 1), int(py // 1))
        assert (int(cx[m]), int(cy[m])) == want, m
        assert 0 <= cx[m] <= nx
