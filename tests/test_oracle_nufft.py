"""Pins of the FP64 NUFFT oracle against the mathematics it approximates (Sec. 2.1)."""
import numpy as np
import pytest
from scipy import integrate, special

from oracle import nufft as nu
from oracle import pd


def _uv_cases(rng, m):
    uv = rng.uniform(-0.5, 0.5, (m, 2))
    uv[0] = [0.0, 0.0]                       # the origin
    uv[1] = [0.25, -0.125]                   # exactly on grid nodes (t integer)
    uv[2] = [0.4999, -0.5]                   # |u| near 1/2
    uv[3] = [-0.5, 0.5]
    uv[4] = [1.3, -2.2]                      # outside the principal period
    return uv.astype(np.float32).astype(np.float64)


# measured relative l2 error of this kernel (J = 8, 2x oversampling) vs the exact
# NUDFT on these cases: ~5e-8; the threshold is 10x that and never above 1e-6.
NUFFT_TOL = 5e-7


def test_nufft_vs_brute_force_nudft():
    rng = np.random.default_rng(7)
    for (ny, nx) in [(16, 16), (16, 32)]:
        for ch in range(2):
            x = rng.standard_normal((ny, nx))
            uv = _uv_cases(rng, 50)
            th = rng.uniform(0.5, 2.0, 50)
            a = nu.phi(x, uv, th)
            b = nu.nudft(x, uv, th)
            err = np.linalg.norm(a - b) / np.linalg.norm(b)
            assert err < NUFFT_TOL, err


def test_periodicity_in_u():
    # The NUDFT is 1-periodic in u for integer pixel positions; the NUFFT's
    # tap indices are taken mod K, so shifting u by an integer is exact.
    rng = np.random.default_rng(8)
    x = rng.standard_normal((16, 16))
    uv = _uv_cases(rng, 20)
    th = np.ones(20)
    shifted = uv + np.array([3.0, -2.0])
    assert np.allclose(nu.phi(x, uv, th), nu.phi(x, shifted, th), rtol=0, atol=1e-10 * np.abs(nu.phi(x, uv, th)).max())


def test_dense_matrix_product_equals_operator():
    rng = np.random.default_rng(1)
    ny, nx = 8, 16
    x = rng.standard_normal((ny, nx))
    uv = _uv_cases(rng, 30)
    G, F, Z = nu.dense_matrices(ny, nx, uv)
    th = rng.uniform(0.5, 2, 30)
    dense = th * (G @ (F @ (Z @ x.ravel())))
    op = nu.phi(x, uv, th)
    assert np.linalg.norm(op - dense) <= 1e-14 * np.linalg.norm(dense)
    # adjoint: Re Z^T F^H G^T Theta y
    y = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    dense_adj = (Z.T @ (F.conj().T @ (G.T @ (th * y)))).real.reshape(ny, nx)
    assert np.linalg.norm(nu.phi_adj(y, uv, th, ny, nx) - dense_adj) <= 1e-13 * np.linalg.norm(dense_adj)


def test_dot_test():
    rng = np.random.default_rng(2)
    ny, nx = 32, 32
    x = rng.standard_normal((ny, nx))
    uv = _uv_cases(rng, 300)
    th = rng.uniform(0.5, 2, 300)
    y = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    Phix = nu.phi(x, uv, th)
    lhs = np.vdot(y, Phix).real          # <Phi x, y> over R (real images)
    rhs = float(np.sum(nu.phi_adj(y, uv, th, ny, nx) * x))
    assert abs(lhs - rhs) <= 1e-14 * np.linalg.norm(Phix) * np.linalg.norm(y)


@pytest.mark.parametrize("xi", [0.0, 0.05, 0.125, 0.2, 0.25])
def test_kernel_fourier_transform_closed_form(xi):
    f = lambda t: nu.kb_kernel(t) * np.cos(2 * np.pi * xi * t)
    q, _ = integrate.quad(f, -4, 4, epsabs=1e-16, epsrel=1e-14, limit=400, points=[0.0])
    assert abs(q - nu.kb_ft(xi)) <= 1e-12 * abs(q)


def test_kernel_shape():
    assert nu.kb_kernel(0.0) == 1.0
    assert nu.kb_kernel(4.0) == pytest.approx(1.0 / special.i0(nu.BETA), rel=1e-15)
    assert nu.kb_kernel(4.0 + 1e-9) == 0.0
    t = np.linspace(-4, 4, 101)
    assert np.array_equal(nu.kb_kernel(t), nu.kb_kernel(-t))
    assert nu.BETA == pytest.approx(np.pi * np.sqrt(35.2), rel=1e-15)


def test_taps_cover_support():
    # every tap with |t - k| < J/2 is used exactly once (J taps per dimension)
    rng = np.random.default_rng(3)
    t = rng.uniform(-100, 100, 1000)
    k, w = nu._taps(t, 1 << 20)
    base = np.floor(t)
    d = t[None, :] - (base[None, :] - 3 + np.arange(8)[:, None])
    assert np.all(d < 4) and np.all(d >= -4)


def test_op_norm_power_iteration_vs_dense_svd():
    rng = np.random.default_rng(4)
    ny, nx = 8, 8
    uv = _uv_cases(rng, 40)
    th = rng.uniform(0.5, 2, 40)
    u = 1.0 / rng.integers(1, 4, 40)
    G, F, Z = nu.dense_matrices(ny, nx, uv)
    Phi = (np.sqrt(u) * th)[:, None] * (G @ F @ Z)
    real_map = np.vstack([Phi.real, Phi.imag])      # x real -> (Re, Im) of U^1/2 Phi x
    smax = np.linalg.svd(real_map, compute_uv=False)[0]
    prob = pd.Problem(nx=nx, ny=ny, uv=[uv], y=[np.zeros(40, complex)], theta=[th], u=[u],
                      eps=[np.array([1.0])], block_ptr=[np.array([0, 40])])
    val, _, _ = pd.op_norm_phi(prob, rng.standard_normal((1, ny, nx)), max_it=5000, tol=1e-14)
    assert val == pytest.approx(smax ** 2, rel=1e-9)
