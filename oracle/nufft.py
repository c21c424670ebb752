"""FP64 measurement operator Phi_l = Theta_l G_l F Z (Sec. 2.1, eq:inverse).

Readings taken where the paper is silent (it names only "a convolution
kernel", "the FFT matrix" and "Z accounts for the oversampling and corrects
for possible imperfections in the interpolation"):

* pixel p = (i - nx/2, j - ny/2) for array index [j][i] (row j = y);
  u = (u, v) in cycles per pixel; exact target is the NUDFT
  y_m = theta_m sum_p x_p exp(-2 pi i (u_m p_x + v_m p_y))  (sign of eq:RIdata1);
* oversampling 2 per dimension: grid Kx = 2 nx, Ky = 2 ny;
* Kaiser-Bessel kernel of width J = 8, phi(t) = I0(beta sqrt(1-(2t/J)^2))/I0(beta)
  for |t| <= J/2, beta = pi sqrt((J/s)^2 (s-1/2)^2 - 0.8) with s = 2 (Beatty et al. 2005);
* taps k = floor(t) - J/2 + 1 ... floor(t) + J/2 (the |t-k| = J/2 endpoint on the
  right of t is included), grid index k mod K;
* Z: multiply by s(p) = 1/(phihat(p_x/Kx) phihat(p_y/Ky)) and place pixel p at grid
  index p mod K; phihat is the closed-form continuous Fourier transform of phi;
* F: unnormalised forward DFT  ghat[k] = sum_q g[q] exp(-2 pi i k.q/K);
* adjoint for real images: Re(Z^T F^H G^T Theta y)  (real part as in eq:proj-plus).

Parity: pinned against brute-force NUDFT, dense matrices, the dot test and a
quadrature of phihat (tests/test_oracle_nufft.py).
"""
from __future__ import annotations

import numpy as np
from scipy import special

J = 8
OVERSAMP = 2


def kb_beta(J: int = J, sigma: float = float(OVERSAMP)) -> float:
    return float(np.pi * np.sqrt((J / sigma) ** 2 * (sigma - 0.5) ** 2 - 0.8))


BETA = kb_beta()


def kb_kernel(t, J: int = J, beta: float = BETA) -> np.ndarray:
    """phi(t), normalised to phi(0) = 1, zero outside |t| <= J/2."""
    t = np.asarray(t, dtype=np.float64)
    arg = 1.0 - (2.0 * t / J) ** 2
    out = np.zeros_like(t)
    m = arg >= 0.0
    out[m] = special.i0(beta * np.sqrt(arg[m])) / special.i0(beta)
    return out


def kb_ft(xi, J: int = J, beta: float = BETA) -> np.ndarray:
    """Continuous Fourier transform of kb_kernel: int phi(t) exp(-2 pi i xi t) dt."""
    xi = np.asarray(xi, dtype=np.float64)
    z = beta ** 2 - (np.pi * J * xi) ** 2
    out = np.empty_like(xi)
    pos = z > 0
    r = np.sqrt(np.abs(z))
    out[pos] = J * np.sinh(r[pos]) / r[pos]
    neg = z < 0
    out[neg] = J * np.sin(r[neg]) / r[neg]
    out[z == 0] = J
    return out / special.i0(beta)


def deapod(n: int) -> np.ndarray:
    """Z's per-dimension scaling 1/phihat(p/K) for pixels p = 0..n-1 (centred)."""
    K = OVERSAMP * n
    p = np.arange(n) - n // 2
    return 1.0 / kb_ft(p / K)


def _zero_pad(x: np.ndarray) -> np.ndarray:
    """Z: scale and place image [ny][nx] onto the oversampled grid [Ky][Kx]."""
    ny, nx = x.shape
    Ky, Kx = OVERSAMP * ny, OVERSAMP * nx
    g = np.zeros((Ky, Kx), dtype=np.complex128)
    qy = (np.arange(ny) - ny // 2) % Ky
    qx = (np.arange(nx) - nx // 2) % Kx
    g[np.ix_(qy, qx)] = x * deapod(ny)[:, None] * deapod(nx)[None, :]
    return g


def _crop(g: np.ndarray, ny: int, nx: int) -> np.ndarray:
    """Z^T: take the image support back from the grid and apply the scaling."""
    Ky, Kx = g.shape
    qy = (np.arange(ny) - ny // 2) % Ky
    qx = (np.arange(nx) - nx // 2) % Kx
    return g[np.ix_(qy, qx)] * deapod(ny)[:, None] * deapod(nx)[None, :]


def _taps(t: np.ndarray, K: int):
    """Per-visibility tap indices (mod K) and weights along one dimension: [J][M]."""
    f = np.floor(t)
    k = f[None, :] - (J // 2 - 1) + np.arange(J)[:, None]
    w = kb_kernel(t[None, :] - k)
    return np.mod(k.astype(np.int64), K), w


def degrid(ghat: np.ndarray, uv: np.ndarray) -> np.ndarray:
    """G: interpolate the oversampled spectrum at the visibility frequencies."""
    Ky, Kx = ghat.shape
    kx, wx = _taps(uv[:, 0] * Kx, Kx)
    ky, wy = _taps(uv[:, 1] * Ky, Ky)
    out = np.zeros(uv.shape[0], dtype=np.complex128)
    for jy in range(J):
        row = np.zeros(uv.shape[0], dtype=np.complex128)
        for jx in range(J):
            row += wx[jx] * ghat[ky[jy], kx[jx]]
        out += wy[jy] * row
    return out


def grid(z: np.ndarray, uv: np.ndarray, Ky: int, Kx: int) -> np.ndarray:
    """G^T: spread visibilities onto the oversampled grid (sum over taps)."""
    kx, wx = _taps(uv[:, 0] * Kx, Kx)
    ky, wy = _taps(uv[:, 1] * Ky, Ky)
    acc = np.zeros(Ky * Kx, dtype=np.complex128)
    for jy in range(J):
        for jx in range(J):
            lin = ky[jy] * Kx + kx[jx]
            w = wy[jy] * wx[jx]
            acc += np.bincount(lin, weights=w * z.real, minlength=Ky * Kx)
            acc += 1j * np.bincount(lin, weights=w * z.imag, minlength=Ky * Kx)
    return acc.reshape(Ky, Kx)


def fft_grid(x: np.ndarray) -> np.ndarray:
    """F Z x for one channel image."""
    return np.fft.fft2(_zero_pad(x))


def phi(x: np.ndarray, uv: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """Phi_l x = Theta_l G_l F Z x for one channel (eq:inverse)."""
    return theta * degrid(fft_grid(x), uv)


def phi_adj(y: np.ndarray, uv: np.ndarray, theta: np.ndarray, ny: int, nx: int) -> np.ndarray:
    """Re Phi_l^dagger y = Re Z^T F^H G^T Theta y (adjoint as written in the dual problem)."""
    Ky, Kx = OVERSAMP * ny, OVERSAMP * nx
    g = grid(theta * y, uv, Ky, Kx)
    img = np.fft.ifft2(g) * (Ky * Kx)  # F^H = K * ifft
    return _crop(img, ny, nx).real


def phi_cube(X: np.ndarray, uvs, thetas) -> list:
    """Wideband Phi(X) = [Phi_l x_l]_l (block diagonal over channels)."""
    return [phi(X[l], uvs[l], thetas[l]) for l in range(X.shape[0])]


def phi_adj_cube(ys, uvs, thetas, ny: int, nx: int) -> np.ndarray:
    return np.stack([phi_adj(ys[l], uvs[l], thetas[l], ny, nx) for l in range(len(ys))])


# ---------------------------------------------------------------- exact references

def nudft(x: np.ndarray, uv: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """Brute-force non-uniform DFT: the exact quantity Phi approximates (eq:RIdata1)."""
    ny, nx = x.shape
    py = np.arange(ny) - ny // 2
    px = np.arange(nx) - nx // 2
    ex = np.exp(-2j * np.pi * uv[:, 0:1] * px[None, :])  # [M][nx]
    ey = np.exp(-2j * np.pi * uv[:, 1:2] * py[None, :])  # [M][ny]
    return theta * np.einsum("mj,ji,mi->m", ey, x, ex)


def dense_matrices(ny: int, nx: int, uv: np.ndarray):
    """Dense G [M][K], F [K][K], Z [K][N] for tiny sizes (row-major flattening)."""
    Ky, Kx = OVERSAMP * ny, OVERSAMP * nx
    K, N, M = Ky * Kx, ny * nx, uv.shape[0]
    Z = np.zeros((K, N))
    qy = (np.arange(ny) - ny // 2) % Ky
    qx = (np.arange(nx) - nx // 2) % Kx
    sy, sx = deapod(ny), deapod(nx)
    for j in range(ny):
        for i in range(nx):
            Z[qy[j] * Kx + qx[i], j * nx + i] = sy[j] * sx[i]
    Fy = np.exp(-2j * np.pi * np.outer(np.arange(Ky), np.arange(Ky)) / Ky)
    Fx = np.exp(-2j * np.pi * np.outer(np.arange(Kx), np.arange(Kx)) / Kx)
    F = np.kron(Fy, Fx)
    G = np.zeros((M, K))
    kx, wx = _taps(uv[:, 0] * Kx, Kx)
    ky, wy = _taps(uv[:, 1] * Ky, Ky)
    for m in range(M):
        for jy in range(J):
            for jx in range(J):
                G[m, ky[jy, m] * Kx + kx[jx, m]] += wy[jy, m] * wx[jx, m]
    return G, F, Z
