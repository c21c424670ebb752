"""Pins of the SARA dictionary oracle (Sec. 2.3): filter identities, closed forms, PR."""
import numpy as np
import pytest

from oracle import wavelets as wv


@pytest.mark.parametrize("K", range(1, 9))
def test_filter_identities(K):
    h = wv.daubechies(K)
    g = wv.highpass(h)
    assert len(h) == 2 * K
    assert h.sum() == pytest.approx(np.sqrt(2), abs=1e-14)
    for m in range(K):                     # orthonormality to even shifts
        assert np.dot(h[: len(h) - 2 * m], h[2 * m:]) == pytest.approx(float(m == 0), abs=1e-14)
    n = np.arange(2 * K, dtype=np.float64)
    for p in range(K):                     # K vanishing moments of the high-pass
        scale = np.sum(np.abs(n ** p * g))
        assert abs(np.sum(n ** p * g)) <= 1e-12 * scale
    # K vanishing moments is exactly the order of the zero of H at omega = pi
    assert abs(np.sum(((-1.0) ** n) * h)) < 1e-14


def test_db1_is_haar():
    assert np.allclose(wv.daubechies(1), [2 ** -0.5, 2 ** -0.5], rtol=0, atol=1e-16)


def test_db2_closed_form():
    s3 = np.sqrt(3.0)
    ref = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * np.sqrt(2.0))
    assert np.allclose(wv.daubechies(2), ref, rtol=0, atol=1e-15)


def test_db3_closed_form():
    s10 = np.sqrt(10.0)
    r = np.sqrt(5 + 2 * s10)
    ref = np.array([1 + s10 + r, 5 + s10 + 3 * r, 10 - 2 * s10 + 2 * r,
                    10 - 2 * s10 - 2 * r, 5 + s10 - 3 * r, 1 + s10 - r]) / (16 * np.sqrt(2.0))
    assert np.allclose(wv.daubechies(3), ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("shape", [(64, 64), (32, 64), (16, 16)])
def test_perfect_reconstruction_and_parseval(shape):
    rng = np.random.default_rng(0)
    X = rng.standard_normal((2,) + shape)
    for K in range(1, 9):
        C = wv.dwt2(X, K, 4)
        assert np.abs(wv.idwt2(C, K, 4) - X).max() < 1e-13
        assert np.linalg.norm(C) == pytest.approx(np.linalg.norm(X), rel=1e-14)


def test_constant_image_has_no_details():
    X = np.full((1, 32, 32), 3.5)
    for K in range(1, 9):
        C = wv.dwt2(X, K, 4)
        ll = C[0, :2, :2].copy()
        C[0, :2, :2] = 0
        assert np.abs(C).max() < 1e-12
        assert np.allclose(ll, 3.5 * 2 ** 4)     # each level multiplies the mean by 2


def test_haar_one_level_by_hand():
    x = np.array([[1.0, 3.0], [5.0, 7.0]])
    c = wv.dwt2(x, 1, 1)
    # rows: a = (x0 + x1)/sqrt2, d = (x0 - x1)/sqrt2 ; then columns
    r = np.array([[4 / np.sqrt(2), -2 / np.sqrt(2)], [12 / np.sqrt(2), -2 / np.sqrt(2)]])
    ref = np.array([[(r[0, 0] + r[1, 0]) / np.sqrt(2), (r[0, 1] + r[1, 1]) / np.sqrt(2)],
                    [(r[0, 0] - r[1, 0]) / np.sqrt(2), (r[0, 1] - r[1, 1]) / np.sqrt(2)]])
    assert np.allclose(c, ref, atol=1e-15)


def test_psi_is_adjoint_and_norm_is_D():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((3, 32, 32))
    C = rng.standard_normal((9, 3, 32, 32))
    lhs = np.sum(wv.psi_adj(X) * C)
    rhs = np.sum(X * wv.psi(C))
    assert lhs == pytest.approx(rhs, rel=1e-13)
    # Psi Psi^dag = D I, so the power iteration on it returns exactly D = 9
    x = rng.standard_normal((1, 32, 32))
    for _ in range(3):
        y = wv.psi(wv.psi_adj(x))
        lam = np.linalg.norm(y) / np.linalg.norm(x)
        x = y
    assert lam == pytest.approx(9.0, rel=1e-13)
