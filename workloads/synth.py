"""Synthetic wideband workloads shaped like the paper's simulations (Section 4.1).

The paper's own inputs (the W28 image and a VLA uv-coverage) are not
available, so seeded stand-ins with the same shapes are drawn here:

* sky cube: sum of Gaussian sources with power-law (optionally curved)
  spectra, i.e. a linear mixture X = S H^T as in eq:model;
* uv points: Gaussian-density random Fourier sampling at the reference
  frequency, scaled by nu_l/nu_0 per channel, rounded to float32-representable
  values so that FP32 and FP64 consumers see identical coordinates;
* noise: unit complex Gaussian draws, scaled from the input SNR;
* l2 bounds: chi-square based (mean + 2 std of the whitened noise norm).

Coordinates are in cycles per pixel.  Nothing here evaluates the measurement
operator: ``make_measurements`` takes noiseless visibilities from the caller.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np


@dataclass(frozen=True)
class WorkloadConfig:
    name: str
    nx: int
    ny: int
    L: int
    f_lo: float            # GHz, first channel (= reference frequency nu_0)
    f_hi: float            # GHz, last channel
    n_src: int
    curved: bool           # curved power law (alpha + beta log(nu/nu0))
    m_per_chan: int        # fixed visibilities per channel (when m_range is None)
    m_range: tuple | None  # (lo, hi) fractions of N for uniform per-channel counts
    n_blocks: int
    isnr_db: float
    seed: int
    n_lines: int = 0       # emission lines added to each source spectrum (own random stream)
    src_sigma: tuple = (1.0, 3.0)   # range of the Gaussian source widths (pixels)

    @property
    def N(self) -> int:
        return self.nx * self.ny

    def freqs(self) -> np.ndarray:
        if self.L == 1:
            return np.array([self.f_lo])
        return np.linspace(self.f_lo, self.f_hi, self.L)

    def scaled(self, **kw) -> "WorkloadConfig":
        return replace(self, **kw)


# The five workloads (64^2 x 4 FP64, 256^2 x 15 FP64, 512^2 x 60 uneven FP32,
# the same cube for autograd, 1024^2 x 32 mixed precision).
CONFIGS = {
    "cube64_L4": WorkloadConfig("cube64_L4", 64, 64, 4, 1.0, 2.0, 20, False, 2048, None, 1, 60.0, 1),
    "cube256_L15": WorkloadConfig("cube256_L15", 256, 256, 15, 1.4, 2.8, 50, True, 32768, None, 4, 40.0, 2),
    "cube512_L60": WorkloadConfig("cube512_L60", 512, 512, 60, 1.4, 2.8, 50, True, 0, (0.2, 2.0), 8, 40.0, 3),
    "cube512_L60_autograd": WorkloadConfig("cube512_L60_autograd", 512, 512, 60, 1.4, 2.8, 50, True, 0, (0.2, 2.0), 8, 40.0, 4),
    "cube1024_L32": WorkloadConfig("cube1024_L32", 1024, 1024, 32, 1.4, 2.8, 50, True, 1048576, None, 4, 40.0, 5),
    # small cases used by parity tests: several tiles, ragged block sizes
    "cube32_L3": WorkloadConfig("cube32_L3", 32, 32, 3, 1.0, 2.0, 6, False, 700, None, 3, 40.0, 11),
    "cube64_L5": WorkloadConfig("cube64_L5", 64, 64, 5, 1.4, 2.8, 12, True, 0, (0.2, 2.0), 4, 40.0, 12),
    "cube128x64_L4": WorkloadConfig("cube128x64_L4", 128, 64, 4, 1.4, 2.8, 15, True, 0, (0.2, 2.0), 3, 30.0, 13),
}


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([seed, stream]))


def make_sky(cfg: WorkloadConfig) -> np.ndarray:
    """Sky cube X0 of shape [L][ny][nx] (float64, non-negative)."""
    rng = _rng(cfg.seed, 1)
    nu = cfg.freqs() / cfg.f_lo
    cy = cfg.ny / 2 + rng.uniform(-0.4, 0.4, cfg.n_src) * cfg.ny
    cx = cfg.nx / 2 + rng.uniform(-0.4, 0.4, cfg.n_src) * cfg.nx
    sig = rng.uniform(cfg.src_sigma[0], cfg.src_sigma[1], cfg.n_src)
    peak = 10.0 ** rng.uniform(-3.0, 0.0, cfg.n_src)
    alpha = rng.normal(-0.7, 0.2, cfg.n_src)
    curv = rng.normal(0.0, 0.1, cfg.n_src) if cfg.curved else np.zeros(cfg.n_src)
    yy = np.arange(cfg.ny)[:, None]
    xx = np.arange(cfg.nx)[None, :]
    S = np.empty((cfg.n_src, cfg.ny, cfg.nx))
    for q in range(cfg.n_src):
        S[q] = peak[q] * np.exp(-((yy - cy[q]) ** 2 + (xx - cx[q]) ** 2) / (2 * sig[q] ** 2))
    H = nu[:, None] ** (alpha[None, :] + curv[None, :] * np.log(nu)[:, None])  # [L][Q]
    if cfg.n_lines > 0:
        # Gaussian emission lines on the continua (Sec. 4.1 adds lines of varied
        # positions and amplitudes); drawn from a stream of their own
        rl = _rng(cfg.seed, 6)
        ch = np.arange(cfg.L)[:, None]
        for q in range(cfg.n_src):
            pos = rl.uniform(0, cfg.L - 1, cfg.n_lines)
            amp = rl.uniform(0.2, 1.0, cfg.n_lines) * H[:, q].max()
            wid = rl.uniform(0.5, 2.0, cfg.n_lines)
            H[:, q] += (amp[None, :] * np.exp(-0.5 * ((ch - pos[None, :]) / wid[None, :]) ** 2)).sum(axis=1)
    X = np.tensordot(H, S, axes=(1, 0))
    return np.ascontiguousarray(X)


def _counts(cfg: WorkloadConfig, rng: np.random.Generator) -> np.ndarray:
    if cfg.m_range is None:
        return np.full(cfg.L, cfg.m_per_chan, dtype=np.int64)
    lo, hi = cfg.m_range
    return np.floor(rng.uniform(lo, hi, cfg.L) * cfg.N).astype(np.int64)


def make_uv(cfg: WorkloadConfig):
    """Per-channel (uv [M_l][2] float64 of float32 values, block_ptr int64)."""
    rng = _rng(cfg.seed, 2)
    nu = cfg.freqs() / cfg.f_lo
    s = 0.5 / (3.0 * nu[-1])
    counts = _counts(cfg, rng)
    pool_n = int(counts.max()) if cfg.m_range is None else 2 * cfg.N
    base = rng.normal(0.0, s, (pool_n, 2))
    uvs, bptrs = [], []
    for l in range(cfg.L):
        m = int(counts[l])
        uv = (base[:m] * nu[l]).astype(np.float32).astype(np.float64)
        uvs.append(np.ascontiguousarray(uv))
        B = cfg.n_blocks
        bptrs.append(np.array([(b * m) // B for b in range(B + 1)], dtype=np.int64))
    return uvs, bptrs


def make_noise(cfg: WorkloadConfig, counts) -> list:
    """Unit-variance complex Gaussian draws per channel ([M_l] complex128)."""
    rng = _rng(cfg.seed, 3)
    out = []
    for m in counts:
        w = (rng.standard_normal(m) + 1j * rng.standard_normal(m)) / np.sqrt(2.0)
        out.append(w)
    return out


def make_problem_inputs(cfg: WorkloadConfig):
    """Sky cube, uv coverage, block pointers and noise draws for ``cfg``."""
    X0 = make_sky(cfg)
    uvs, bptrs = make_uv(cfg)
    noise = make_noise(cfg, [len(u) for u in uvs])
    return {"X0": X0, "uv": uvs, "block_ptr": bptrs, "noise": noise}


def make_measurements(y0_list, noise_list, block_ptrs, isnr_db: float):
    """Noisy data from noiseless visibilities y0 (computed by the caller).

    sigma_l = ||y0_l|| / sqrt(M_l) * 10^(-iSNR/20); y_raw = y0 + sigma_l w;
    natural weights theta = 1/sigma_l; l2 bounds from the chi-square law of
    the whitened noise norm: eps_b = sqrt(M_b + 2 sqrt(M_b)).
    """
    y_raw, theta, eps = [], [], []
    for y0, w, bp in zip(y0_list, noise_list, block_ptrs):
        m = len(y0)
        sig = np.linalg.norm(y0) / np.sqrt(m) * 10.0 ** (-isnr_db / 20.0) if m else 1.0
        if not np.isfinite(sig) or sig <= 0:
            sig = 1.0
        y_raw.append(y0 + sig * w)
        theta.append(np.full(m, 1.0 / sig))
        mb = np.diff(bp).astype(np.float64)
        eps.append(np.sqrt(mb + 2.0 * np.sqrt(mb)))
    return y_raw, theta, eps


def make_state(cfg: WorkloadConfig, X0: np.ndarray, counts, n_bases: int = 9, seed_stream: int = 4,
               scale_dual: float = 0.05):
    """A generic primal-dual state (X, X_tilde, P, A, v) for one-iteration tests.

    X is a perturbed non-negative copy of the sky, X_tilde a further perturbed
    copy (it may be negative), and the duals are small random arrays.
    Returned as float64 / complex128.
    """
    rng = _rng(cfg.seed, seed_stream)
    amp = max(float(X0.max()), 1e-3)
    X = np.maximum(X0 * (1 + 0.2 * rng.standard_normal(X0.shape)) + 0.01 * amp * rng.standard_normal(X0.shape), 0)
    Xt = X + 0.02 * amp * rng.standard_normal(X0.shape)
    P = scale_dual * amp * rng.standard_normal(X0.shape)
    A = scale_dual * amp * rng.standard_normal((n_bases,) + X0.shape)
    v = [scale_dual * (rng.standard_normal(m) + 1j * rng.standard_normal(m)) for m in counts]
    return {"X": X, "Xt": Xt, "P": P, "A": A, "v": v}


def power_start(cfg: WorkloadConfig, seed_stream: int = 5) -> np.ndarray:
    """Seeded start cube for power iterations ([L][ny][nx], float64)."""
    rng = _rng(cfg.seed, seed_stream)
    return rng.standard_normal((cfg.L, cfg.ny, cfg.nx))
