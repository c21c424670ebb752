"""FP64 SARA dictionary: Dirac basis + Daubechies db1..db8 (Sec. 2.3).

The paper defines Psi^dagger = (Psi_1, ..., Psi_D)^dagger as the concatenation
of the Dirac basis and the first eight Daubechies wavelet bases; it gives no
decomposition depth, boundary handling or normalisation.  Readings taken:

* each Daubechies basis is the orthonormal, critically sampled, periodised
  separable 2-D Mallat transform (the dual variables A_d are N x L, so every
  Psi_d^dagger must map R^N to R^N);
* depth 4 levels (workload parameter);
* the concatenation is not renormalised, so Psi Psi^dagger = D I and
  ||Psi^dagger||_S^2 = D = 9 exactly;
* filters: db-K low-pass h of length 2K from Daubechies' spectral
  factorisation of P_K(y) = sum_{k<K} C(K-1+k, k) y^k keeping the roots inside
  the unit circle (minimum phase), normalised so that sum h = sqrt(2);
  high-pass g[n] = (-1)^n h[2K-1-n];
* one level on a length-n signal: a[k] = sum_n h[n] x[(2k+n) mod n_len],
  d[k] = sum_n g[n] x[(2k+n) mod n_len]; low half then high half;
  rows (x direction) first, then columns; the LL quadrant is transformed at
  the next level.

Parity: pinned by filter identities, closed-form db2/db3, perfect
reconstruction, Parseval and vanishing moments (tests/test_oracle_wavelets.py).
"""
from __future__ import annotations

from functools import lru_cache
from math import comb

import numpy as np


@lru_cache(maxsize=None)
def daubechies(K: int) -> np.ndarray:
    """Low-pass filter of db-K (2K taps) by spectral factorisation."""
    if K < 1:
        raise ValueError("K >= 1")
    # P_K(y) = sum_{k<K} C(K-1+k, k) y^k; np.roots wants the highest power first
    coeffs = [comb(K - 1 + k, k) for k in range(K)]
    yroots = np.roots(coeffs[::-1]) if K > 1 else np.array([])
    # y = sin^2(w/2) = (2 - z - 1/z)/4  ->  z^2 - (2 - 4y) z + 1 = 0
    zr = []
    for y in yroots:
        b = 1.0 - 2.0 * y
        s = np.sqrt(b * b - 1.0 + 0j)
        z1, z2 = b + s, b - s
        zr.append(z1 if abs(z1) < 1 else z2)
    poly = np.array([1.0 + 0j])
    for _ in range(K):
        poly = np.convolve(poly, [0.5, 0.5])
    for r in zr:
        poly = np.convolve(poly, [1.0, -r]) / (1.0 - r)
    h = np.sqrt(2.0) * poly.real
    return h


def highpass(h: np.ndarray) -> np.ndarray:
    n = np.arange(len(h))
    return ((-1.0) ** n) * h[::-1]


def _analysis_1d(x: np.ndarray, h: np.ndarray, g: np.ndarray) -> np.ndarray:
    """One periodised analysis level along the last axis: [..., n] -> [..., a | d]."""
    n = x.shape[-1]
    idx = (2 * np.arange(n // 2)[:, None] + np.arange(len(h))[None, :]) % n
    xs = x[..., idx]  # [..., n/2, taps]
    return np.concatenate([xs @ h, xs @ g], axis=-1)


def _synthesis_1d(c: np.ndarray, h: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Adjoint (= inverse) of _analysis_1d along the last axis."""
    n = c.shape[-1]
    a, d = c[..., : n // 2], c[..., n // 2:]
    x = np.zeros_like(c)
    k = np.arange(n // 2)
    for j in range(len(h)):
        x[..., (2 * k + j) % n] += h[j] * a + g[j] * d
    return x


def dwt2(x: np.ndarray, K: int, levels: int) -> np.ndarray:
    """Psi_d^dagger for db-K on images [..., ny, nx] (Mallat layout, in a new array)."""
    h = daubechies(K)
    g = highpass(h)
    c = np.array(x, dtype=np.float64, copy=True)
    ny, nx = c.shape[-2:]
    for lev in range(levels):
        my, mx = ny >> lev, nx >> lev
        sub = c[..., :my, :mx]
        sub = _analysis_1d(sub, h, g)                                    # rows (x)
        sub = np.swapaxes(_analysis_1d(np.swapaxes(sub, -1, -2), h, g), -1, -2)  # columns (y)
        c[..., :my, :mx] = sub
    return c


def idwt2(c: np.ndarray, K: int, levels: int) -> np.ndarray:
    """Psi_d for db-K: adjoint (and inverse) of dwt2."""
    h = daubechies(K)
    g = highpass(h)
    x = np.array(c, dtype=np.float64, copy=True)
    ny, nx = x.shape[-2:]
    for lev in reversed(range(levels)):
        my, mx = ny >> lev, nx >> lev
        sub = x[..., :my, :mx]
        sub = np.swapaxes(_synthesis_1d(np.swapaxes(sub, -1, -2), h, g), -1, -2)  # columns
        sub = _synthesis_1d(sub, h, g)                                           # rows
        x[..., :my, :mx] = sub
    return x


def psi_adj(X: np.ndarray, levels: int = 4, n_db: int = 8) -> np.ndarray:
    """Psi^dagger X: [L][ny][nx] -> [D][L][ny][nx]; d = 0 Dirac, d = K for db-K."""
    out = [np.array(X, dtype=np.float64, copy=True)]
    for K in range(1, n_db + 1):
        out.append(dwt2(X, K, levels))
    return np.stack(out)


def psi(C: np.ndarray, levels: int = 4) -> np.ndarray:
    """Psi C = sum_d Psi_d C_d: [D][L][ny][nx] -> [L][ny][nx]."""
    X = np.array(C[0], dtype=np.float64, copy=True)
    for K in range(1, C.shape[0]):
        X += idwt2(C[K], K, levels)
    return X
