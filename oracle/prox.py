"""FP64 proximity operators and dual updates (Sec. 3.3, eq:md, Algorithm 2).

* proj_pos         : eq:proj-plus, componentwise projection onto R_+ (of Re x).
* prox_l21         : eq:prox-L21, row-wise soft-thresholding of length-L rows.
* dual_l21         : Algorithm 2, l2,1 dual: A <- (I - S^{l21}_{w mu ||Psi^dag||^2})(A + Psi_d^dag X~).
* prox_nuclear_*   : eq:prox-L*, singular-value soft-thresholding, by SVD (the
                     definition) and by the L x L Gram matrix (the route the
                     GPU takes).
* dual_nuclear     : Algorithm 2, nuclear dual: P <- (I - S*_w)(P + X~).
* proj_ball_precond: prox of the l2-ball indicator in the metric U (eq:prox),
                     i.e. the ellipsoid projection of Sec. 3.3, solved exactly.
* dual_data_block  : Algorithm 2, data-dual projection via the Moreau identity eq:md.

Readings (paper silent):
* the nuclear weights w_j pair with the singular values sorted in decreasing
  order; a zero singular value keeps its direction (factor 1 in the dual form);
* the l2,1 weights are one per coefficient row (D*N rows), the index set used
  in eq:weights-l21;
* the ellipsoid projection is solved exactly: the multiplier lambda is the root
  of the secular equation, found by safeguarded Newton/bisection.
"""
from __future__ import annotations

import numpy as np


def proj_pos(x: np.ndarray) -> np.ndarray:
    """eq:proj-plus: max(Re x, 0)."""
    return np.maximum(np.real(x), 0.0)


def prox_l21(Z: np.ndarray, t: np.ndarray | float, axis: int = 1) -> np.ndarray:
    """eq:prox-L21: rows (along ``axis``) shrunk by max(||z_n|| - t_n, 0)/||z_n||."""
    nrm = np.sqrt(np.sum(Z * Z, axis=axis, keepdims=True))
    t = np.expand_dims(np.asarray(t, dtype=np.float64), axis) if np.ndim(t) else t
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(nrm > 0, np.maximum(nrm - t, 0.0) / nrm, 0.0)
    return Z * f


def dual_l21(A: np.ndarray, PsiXt: np.ndarray, wbar: np.ndarray, mu: float, psi_norm2: float) -> np.ndarray:
    """The l2,1 dual update of Algorithm 2 for all d at once.

    A, PsiXt: [D][L][ny][nx]; a row is the length-L vector at fixed (d, y, x);
    wbar: [D][ny][nx].  Returns Z - S(Z) with Z = A + PsiXt and threshold
    mu * wbar * psi_norm2.
    """
    Z = A + PsiXt
    return Z - prox_l21(Z, mu * wbar * psi_norm2, axis=1)


def soft_threshold(Z: np.ndarray, t) -> np.ndarray:
    """Proximity operator of t * |.| (elementwise l1, the single-channel SARA prior)."""
    return np.sign(Z) * np.maximum(np.abs(Z) - t, 0.0)


def dual_l1(A: np.ndarray, PsiXt: np.ndarray, wbar: np.ndarray, mu: float, psi_norm2: float) -> np.ndarray:
    """The same dual for the SARA variant: the weighted l1 norm of each channel's
    coefficients in place of the l2,1 norm (Sec. 4.2, eq:min-sara; each channel is its
    own problem with its own weights).  A, PsiXt, wbar: [D][L][ny][nx].  Returns
    Z - soft(Z) with Z = A + PsiXt and threshold mu * wbar * psi_norm2, element by element."""
    Z = A + PsiXt
    return Z - soft_threshold(Z, mu * wbar * psi_norm2)


def _as_matrix(X: np.ndarray) -> np.ndarray:
    """Cube [L][ny][nx] -> N x L matrix (column l = channel l), as in Sec. 2.1."""
    L = X.shape[0]
    return X.reshape(L, -1).T


def _from_matrix(M: np.ndarray, shape) -> np.ndarray:
    return np.ascontiguousarray(M.T.reshape(shape))


def prox_nuclear_svd(X: np.ndarray, w: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """eq:prox-L*: U diag(max(s - w, 0)) V^T by the SVD of the N x L matrix."""
    M = _as_matrix(X)
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    sp = np.maximum(s - w[: len(s)], 0.0)
    return _from_matrix((U * sp) @ Vt, X.shape), s


def gram_eig(M: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Singular values (descending) and right singular vectors via C = M^T M."""
    C = M.T @ M
    lam, V = np.linalg.eigh(C)
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order]
    return np.sqrt(np.maximum(lam, 0.0)), V


def nuclear_dual_factor(s: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Factor of (I - S*_w) on each singular direction: min(1, w_j / s_j), 1 at s_j = 0."""
    with np.errstate(divide="ignore"):
        return np.where(s > 0, np.minimum(1.0, w / np.where(s > 0, s, 1.0)), 1.0)


def prox_nuclear_gram(X: np.ndarray, w: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """eq:prox-L* through the Gram matrix: X V diag(1 - min(1, w/s)) V^T."""
    M = _as_matrix(X)
    s, V = gram_eig(M)
    f = 1.0 - nuclear_dual_factor(s, w)
    return _from_matrix(M @ (V * f) @ V.T, X.shape), s


def dual_nuclear(P: np.ndarray, Xt: np.ndarray, w: np.ndarray, method: str = "svd") -> np.ndarray:
    """The nuclear dual of Algorithm 2: P <- (I - S*_w)(P + X~)."""
    Z = P + Xt
    if method == "svd":
        return Z - prox_nuclear_svd(Z, w)[0]
    M = _as_matrix(Z)
    s, V = gram_eig(M)
    return _from_matrix(M @ (V * nuclear_dual_factor(s, w)) @ V.T, Z.shape)


# ------------------------------------------------------------------ data fidelity

def secular_root(a: np.ndarray, u: np.ndarray, eps: float, tol: float = 1e-14, max_it: int = 200) -> float:
    """Root lambda > 0 of f(lam) = sum_i a_i / (u_i + lam)^2 - eps^2 (decreasing).

    a_i = |U(c - y)|_i^2 >= 0.  Safeguarded Newton on [0, sqrt(sum a)/eps].
    """
    e2 = eps * eps
    lo, hi = 0.0, np.sqrt(a.sum()) / eps
    lam = 0.5 * hi
    for _ in range(max_it):
        r = u + lam
        f = np.sum(a / r ** 2) - e2
        if abs(f) <= tol * e2:
            break
        if f > 0:
            lo = lam
        else:
            hi = lam
        fp = -2.0 * np.sum(a / r ** 3)
        step = lam - f / fp
        lam = step if (lo < step < hi) else 0.5 * (lo + hi)
        if hi - lo <= 1e-16 * max(hi, 1e-300):
            break
    return lam


def proj_ball_precond(c: np.ndarray, y: np.ndarray, u: np.ndarray, eps: float):
    """argmin_{||q - y|| <= eps} (q - c)^H U (q - c) (prox of the ball indicator, eq:prox).

    Equivalent to the Euclidean projection onto the ellipsoid E(y, eps) of Sec. 3.3
    after the change of variable z = U^{1/2} q.  Returns (q, lambda).
    """
    r = c - y
    if np.linalg.norm(r) <= eps:
        return c.copy(), 0.0
    if eps == 0.0:          # the ball is the single point y
        return y.copy(), np.inf
    a = (u * u) * (r.real ** 2 + r.imag ** 2)
    lam = secular_root(a, u, eps)
    return y + (u / (u + lam)) * r, lam


def dual_data_block(vbar: np.ndarray, y: np.ndarray, u: np.ndarray, eps: float):
    """The data-dual projection of Algorithm 2: v = U^{1/2}(I - P_E)(U^{-1/2} vbar) = vbar - U q, q = prox(U^{-1} vbar).

    Follows from eq:md with zeta = 1 and the metric U.  Returns (v, lambda).
    """
    q, lam = proj_ball_precond(vbar / u, y, u, eps)
    return vbar - u * q, lam
