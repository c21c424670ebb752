"""Pins of the preconditioner density and of the visibility-order definition."""
from collections import Counter

import numpy as np

import workloads as W
from oracle import binning, precond


def test_density_counts_vs_dictionary_count():
    cfg = W.CONFIGS["t2"]
    uvs, _ = W.synth.make_uv(cfg)
    for uv in uvs[:2]:
        n = precond.density_counts(uv, cfg.nx, cfg.ny)
        keys = [(int(np.floor(a * cfg.nx)) % cfg.nx, int(np.floor(b * cfg.ny)) % cfg.ny) for a, b in uv]
        cnt = Counter(keys)
        assert np.array_equal(n, [cnt[k] for k in keys])
        assert np.array_equal(precond.density_precond(uv, cfg.nx, cfg.ny), 1.0 / n)


def test_order_definition_properties():
    cfg = W.CONFIGS["t2"]
    uvs, bps = W.synth.make_uv(cfg)
    T = 16
    for uv, bp in zip(uvs[:2], bps[:2]):
        u = precond.density_precond(uv, cfg.nx, cfg.ny)
        perm, rptr = binning.order(uv, u, bp, cfg.nx, cfg.ny, T)
        M = len(uv)
        assert np.array_equal(np.sort(perm), np.arange(M))
        cx, cy = binning.cells(uv, cfg.nx, cfg.ny)
        Kx = 2 * cfg.nx
        tile = (cy // T) * (Kx // T) + cx // T
        reg = 3 * binning.region_class(cy % T, T) + binning.region_class(cx % T, T)
        key = tile * 9 + reg
        assert np.all(np.diff(key[perm]) >= 0)
        for k in range(len(rptr) - 1):
            seg = perm[rptr[k]:rptr[k + 1]]
            assert np.all(key[seg] == k)
        # regions: offsets within the tile
        assert np.all((cx % T)[reg % 3 == 0] < 3) and np.all((cx % T)[reg % 3 == 2] >= T - 4)


def test_region_reaches_neighbour_exactly():
    # a visibility at in-tile offset o has taps o-3 .. o+4; it reaches the
    # previous tile iff o < 3 and the next tile iff o >= T - 4
    T = 16
    o = np.arange(T)
    cls = binning.region_class(o, T)
    assert np.array_equal(cls == 0, o - 3 < 0)
    assert np.array_equal(cls == 2, o + 4 >= T)
