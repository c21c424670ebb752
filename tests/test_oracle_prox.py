"""Pins of the proximity operators and dual updates (Sec. 3.3, eq:md, Algorithm 2)."""
import numpy as np
import pytest
from scipy import optimize

from oracle import prox


# ----------------------------------------------------------------------- l2,1

def test_l21_rowwise_closed_form_and_optimality():
    rng = np.random.default_rng(0)
    Z = rng.standard_normal((3, 6, 4, 5))      # [D][L][ny][nx], rows along axis 1
    t = rng.uniform(0.5, 3.0, (3, 4, 5))
    P = prox.prox_l21(Z, t, axis=1)
    for d in range(3):
        for y in range(4):
            for x in range(5):
                z = Z[d, :, y, x]
                p = P[d, :, y, x]
                n = np.sqrt(np.sum(z * z))
                if n <= t[d, y, x]:
                    assert np.all(p == 0)
                else:   # optimality: z - p = t p/||p||
                    assert np.allclose(z - p, t[d, y, x] * p / np.linalg.norm(p), atol=1e-14)


def test_l21_single_channel_is_soft_threshold():
    rng = np.random.default_rng(1)
    z = rng.standard_normal((1, 1, 50))
    P = prox.prox_l21(z, 0.7, axis=1)
    assert np.allclose(P[0, 0], np.sign(z[0, 0]) * np.maximum(np.abs(z[0, 0]) - 0.7, 0))


def test_l21_dual_is_projection_onto_balls_moreau():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((2, 5, 3, 3))
    C = rng.standard_normal((2, 5, 3, 3))
    wbar = rng.uniform(0.1, 1.0, (2, 3, 3))
    mu, D = 0.3, 9.0
    out = prox.dual_l21(A, C, wbar, mu, D)
    Z = A + C
    r = mu * D * wbar
    n = np.sqrt(np.sum(Z * Z, axis=1))
    proj = Z * np.minimum(1.0, r / np.maximum(n, 1e-300))[:, None]     # ball projection, radius r
    assert np.allclose(out, proj, atol=1e-14)
    # Moreau: prox_f(z) + prox_{f*}(z) = z
    assert np.allclose(out + prox.prox_l21(Z, r, axis=1), Z, atol=1e-14)


# ------------------------------------------------------------------- nuclear

def test_nuclear_svd_vs_gram_routes():
    rng = np.random.default_rng(3)
    L = 7
    X = rng.standard_normal((L, 16, 16)) @ np.diag(np.logspace(0, -6, 16))   # ill-conditioned
    w = np.sort(rng.uniform(0.0, 0.5, L))
    a, sa = prox.prox_nuclear_svd(X, w)
    b, sb = prox.prox_nuclear_gram(X, w)
    assert np.allclose(sa, sb, rtol=0, atol=1e-10 * sa[0])
    assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(a)
    P = rng.standard_normal(X.shape)
    da = prox.dual_nuclear(P, X, w, "svd")
    db = prox.dual_nuclear(P, X, w, "gram")
    assert np.linalg.norm(da - db) <= 1e-10 * np.linalg.norm(da)


def test_nuclear_rank_one_closed_form():
    rng = np.random.default_rng(4)
    a = rng.standard_normal(64); a /= np.linalg.norm(a)
    b = rng.standard_normal(3); b /= np.linalg.norm(b)
    sig = 2.5
    X = (sig * np.outer(a, b)).T.reshape(3, 8, 8)
    out, s = prox.prox_nuclear_svd(X, np.array([0.75, 1.0, 1.0]))
    ref = ((sig - 0.75) * np.outer(a, b)).T.reshape(3, 8, 8)
    assert np.allclose(out, ref, atol=1e-14)
    assert s[0] == pytest.approx(sig)


def test_nuclear_single_channel_is_vector_shrink():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((1, 4, 4))
    n = np.linalg.norm(x)
    out, _ = prox.prox_nuclear_gram(x, np.array([0.3]))
    assert np.allclose(out, x * max(n - 0.3, 0) / n, atol=1e-14)


def test_nuclear_orthogonal_invariance_and_moreau():
    rng = np.random.default_rng(6)
    L, N = 4, 36
    X = rng.standard_normal((L, 6, 6))
    w = np.full(L, 0.8)
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    R, _ = np.linalg.qr(rng.standard_normal((L, L)))
    M = X.reshape(L, -1).T
    out, _ = prox.prox_nuclear_svd(X, w)
    Mo = out.reshape(L, -1).T
    rot = (Q @ M @ R).T.reshape(X.shape)
    out_rot, _ = prox.prox_nuclear_svd(rot, w)
    assert np.allclose(out_rot.reshape(L, -1).T, Q @ Mo @ R, atol=1e-12)
    # Moreau: (I - S*)(Z) + S*(Z) = Z
    assert np.allclose(prox.dual_nuclear(np.zeros_like(X), X, w) + out, X, atol=1e-13)


def test_nuclear_dual_zero_singular_value_keeps_direction():
    X = np.zeros((3, 4, 4))
    X[0, 1, 1] = 2.0                  # rank one; sigma_2 = sigma_3 = 0
    out = prox.dual_nuclear(np.zeros_like(X), X, np.array([0.5, 0.5, 0.5]), "gram")
    assert np.allclose(out, X * 0.25, atol=1e-15)


# ------------------------------------------------------------- data fidelity

def _block(rng, m):
    y = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    c = y + 3 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    u = 1.0 / rng.integers(1, 5, m)
    return c, y, u


def test_ball_projection_identity_metric_closed_form():
    rng = np.random.default_rng(7)
    c, y, _ = _block(rng, 40)
    eps = 2.0
    q, _ = prox.proj_ball_precond(c, y, np.ones(40), eps)
    ref = y + (c - y) * min(1.0, eps / np.linalg.norm(c - y))
    assert np.allclose(q, ref, atol=1e-13)


def test_ball_projection_kkt_feasibility_idempotence():
    rng = np.random.default_rng(8)
    c, y, u = _block(rng, 64)
    eps = 1.5
    q, lam = prox.proj_ball_precond(c, y, u, eps)
    assert np.linalg.norm(q - y) == pytest.approx(eps, rel=1e-12)      # on the boundary
    # KKT: U (q - c) + lam (q - y) = 0 with lam > 0
    assert lam > 0
    assert np.linalg.norm(u * (q - c) + lam * (q - y)) <= 1e-12 * np.linalg.norm(u * (q - c))
    q2, lam2 = prox.proj_ball_precond(q, y, u, eps * (1 + 1e-12))
    assert np.allclose(q2, q) and lam2 == 0.0
    # variational inequality against random feasible points (metric U)
    for _ in range(20):
        z = y + (rng.standard_normal(64) + 1j * rng.standard_normal(64))
        z = y + (z - y) * eps * rng.uniform() / np.linalg.norm(z - y)
        assert np.real(np.vdot(z - q, u * (c - q))) <= 1e-10


@pytest.mark.parametrize("m", [1, 3, 8])
def test_ball_projection_vs_slsqp(m):
    rng = np.random.default_rng(10 + m)
    c, y, u = _block(rng, m)
    eps = 0.7
    q, _ = prox.proj_ball_precond(c, y, u, eps)
    cr = np.concatenate([c.real, c.imag]); yr = np.concatenate([y.real, y.imag]); ur = np.concatenate([u, u])
    res = optimize.minimize(lambda z: np.sum(ur * (z - cr) ** 2), yr, jac=lambda z: 2 * ur * (z - cr),
                            method="SLSQP", constraints=[{"type": "ineq", "fun": lambda z: eps ** 2 - np.sum((z - yr) ** 2),
                                                          "jac": lambda z: -2 * (z - yr)}],
                            options={"ftol": 1e-15, "maxiter": 1000})
    qs = res.x[:m] + 1j * res.x[m:]
    assert np.linalg.norm(q - qs) <= 1e-7 * max(1.0, np.linalg.norm(q))


def test_dual_data_block_is_moreau_of_projection():
    rng = np.random.default_rng(9)
    c, y, u = _block(rng, 30)
    vbar = u * c
    v, lam = prox.dual_data_block(vbar, y, u, 1.0)
    q, _ = prox.proj_ball_precond(c, y, u, 1.0)
    assert np.allclose(v, vbar - u * q)
    # equals U^{1/2}(I - P_E)(U^{-1/2} vbar) with P_E the Euclidean projection on the ellipsoid
    w = vbar / np.sqrt(u)
    z = np.sqrt(u) * q                      # P_E(w): z = U^{1/2} q
    assert np.allclose(np.sqrt(u) * (w - z), v)
    # inside the ball the dual vanishes
    v0, lam0 = prox.dual_data_block(u * y, y, u, 1.0)
    assert np.all(v0 == 0) and lam0 == 0.0


def test_positivity_projection():
    x = np.array([-1.0, 0.0, 2.0]) + 1j * np.array([5.0, -1.0, 3.0])
    assert np.array_equal(prox.proj_pos(x), [0.0, 0.0, 2.0])


def test_l1_dual_is_projection_onto_linf_ball():
    # Moreau: Z - soft_t(Z) is the projection of Z onto the l_inf ball of radius t
    rng = np.random.default_rng(31)
    A = rng.standard_normal((3, 2, 8, 8))
    S = rng.standard_normal((3, 2, 8, 8))
    wbar = rng.uniform(0.1, 1.0, (3, 2, 8, 8))     # one weight per channel and coefficient
    mu, D = 0.2, 3.0
    out = prox.dual_l1(A, S, wbar, mu, D)
    t = mu * wbar * D
    assert np.allclose(out, np.clip(A + S, -t, t), rtol=0, atol=1e-15)
    # and soft thresholding by hand on one element
    z, tt = 1.7, 0.5
    assert prox.soft_threshold(np.array([z, -z, 0.2]), tt).tolist() == [1.2, -1.2, 0.0]
