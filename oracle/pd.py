"""FP64 adaptive preconditioned primal-dual (Algorithm 2) and the HyperSARA loop (Algorithm 1).

Readings taken (paper silent or ambiguous):
* one iteration consumes (X^{t-1}, X~^{t-1}, P, A_d, v_l^b) and returns the next
  state; dual updates use only iterate t-1 (Algorithm 2 runs them side by side);
* the primal step's data term: channel l's adjoint lands in column l (the selection
  k_l^dagger of the adjoint in the dual problem is implied);
* kappa1 = 1, kappa2 = 1/||Psi^dagger||_S^2 = 1/D, kappa3 = 1/||U^{1/2} Phi||_S^2
  (Sec. 3.4); the norm is the largest eigenvalue of x -> Re Phi^dag U Phi x over
  real images, by power iteration (max over channels: Phi is block diagonal);
* tau = 0.33 by default (the paper requires 0 < tau < 1/3);
* adaptive l2 bounds (Sec. 3.6) use the Appendix A constants and are off by
  default (simulation mode, Sec. 4.1);
* reweighting (Algorithm 1, eq:weights-l21, eq:weights-n): gamma and gamma_bar
  start at 1 and are multiplied by a fixed factor (0.8 by default) after each
  reweight; warm start of every variable.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import nufft, prox, wavelets


@dataclass
class Problem:
    nx: int
    ny: int
    uv: list            # per channel [M_l][2]
    y: list             # per channel naturally weighted data theta * y_raw, [M_l] complex
    theta: list         # per channel [M_l]
    u: list             # per channel preconditioner [M_l] (ones for U = I)
    eps: list           # per channel [B_l]
    block_ptr: list     # per channel [B_l + 1]
    levels: int = 4
    n_db: int = 8

    @property
    def L(self) -> int:
        return len(self.uv)

    @property
    def D(self) -> int:
        return 1 + self.n_db

    def phi(self, X):
        return nufft.phi_cube(X, self.uv, self.theta)

    def phi_adj(self, ys):
        return nufft.phi_adj_cube(ys, self.uv, self.theta, self.ny, self.nx)


@dataclass
class Params:
    mu: float
    tau: float = 0.33
    kappa1: float = 1.0
    kappa2: float | None = None
    kappa3: float | None = None
    wbar: np.ndarray | None = None   # [D][ny][nx] ([D][L][ny][nx] for the SARA prior)
    w: np.ndarray | None = None      # [L]
    adaptive_eps: bool = False
    lam1: float = 5e-4
    lam2: float = 0.01
    lam3: float = 0.618
    vartheta_bar: int = 100
    # prior of the minimisation task: "lrjas" (low rankness + joint average sparsity,
    # eq:min; with reweighting this is HyperSARA), "lr" (nuclear norm only, eq:min-lr),
    # "jas" (l2,1 only, eq:min-js) or "sara" (weighted l1 per channel, eq:min-sara)
    prior: str = "lrjas"


@dataclass
class State:
    X: np.ndarray
    Xt: np.ndarray
    P: np.ndarray
    A: np.ndarray
    v: list
    eps: list | None = None
    vartheta: list | None = None
    beta: float = 1.0
    t: int = 0
    extra: dict = field(default_factory=dict)


def zero_state(prob: Problem) -> State:
    shape = (prob.L, prob.ny, prob.nx)
    return State(
        X=np.zeros(shape), Xt=np.zeros(shape), P=np.zeros(shape),
        A=np.zeros((prob.D,) + shape), v=[np.zeros(len(y), dtype=np.complex128) for y in prob.y],
        eps=[np.array(e, dtype=np.float64) for e in prob.eps],
        vartheta=[np.zeros(len(e), dtype=np.int64) for e in prob.eps])


def op_norm_phi(prob: Problem, x0: np.ndarray, max_it: int = 1000, tol: float = 1e-10):
    """||U^{1/2} Phi||_S^2 by per-channel power iteration on x -> Re Phi_l^dag U_l Phi_l x.

    Returns (max over channels, per-channel values, iterations used).
    """
    vals, its = [], []
    for l in range(prob.L):
        x = x0[l] / np.linalg.norm(x0[l])
        lam_prev = 0.0
        lam = 0.0
        for it in range(1, max_it + 1):
            y = nufft.phi(x, prob.uv[l], prob.theta[l]) * prob.u[l]
            xn = nufft.phi_adj(y, prob.uv[l], prob.theta[l], prob.ny, prob.nx)
            lam = float(np.linalg.norm(xn))
            if lam == 0.0:
                break
            x = xn / lam
            if abs(lam - lam_prev) <= tol * lam:
                break
            lam_prev = lam
        vals.append(lam)
        its.append(it)
    return max(vals) if vals else 0.0, np.array(vals), its


def step_sizes(prob: Problem, prm: Params, phi_norm2: float):
    k2 = prm.kappa2 if prm.kappa2 is not None else 1.0 / prob.D
    k3 = prm.kappa3 if prm.kappa3 is not None else 1.0 / phi_norm2
    return prm.kappa1, k2, k3


def _map(pool, fn, items):
    """fn over independent per-channel items, in a process pool when one is given."""
    return list(pool.map(fn, items)) if pool is not None else [fn(a) for a in items]


def _psi_adj_chan(a):
    x, levels, n_db = a
    return wavelets.psi_adj(x, levels, n_db)


def _psi_chan(a):
    c, levels = a
    return wavelets.psi(c, levels)


def _data_channel(a):
    """Data-fidelity dual of one channel (Algorithm 2): dual step, per-block projection
    (eq:md), residual norms and the adaptive bounds (Sec. 3.6), then the adjoint."""
    (xt, v, uv, theta, u, y, bp, eps_prev, vth_prev, ny, nx, t, beta_prev, adaptive, lam1, lam2, lam3,
     vbar_iters) = a
    Phix = nufft.phi(xt, uv, theta)                               # Theta G F Z x~_l
    vbar = v + u * Phix                                           # dual step
    vl = np.empty_like(vbar)
    eps_new = np.array(eps_prev, dtype=np.float64, copy=True)
    vth_new = np.array(vth_prev, copy=True)
    lam_l, rho_l = [], []
    for b in range(len(bp) - 1):
        s = slice(bp[b], bp[b + 1])
        e_prev = eps_prev[b]
        vl[s], lam = prox.dual_data_block(vbar[s], y[s], u[s], e_prev)   # projection (eq:md)
        lam_l.append(lam)
        r = float(np.linalg.norm(y[s] - Phix[s]))                        # residual norm
        rho_l.append(r)
        if adaptive and (beta_prev < lam1) and (t - vth_new[b] > vbar_iters) \
                and (abs(r - e_prev) / e_prev > lam2):                   # bound-update test
            eps_new[b] = lam3 * r + (1 - lam3) * e_prev                  # new bound
            vth_new[b] = t                                               # its iteration
    adj = nufft.phi_adj(vl, uv, theta, ny, nx)                           # adjoint of the data dual
    return vl, adj, np.array(lam_l), np.array(rho_l), eps_new, vth_new


def pd_iteration(st: State, prob: Problem, prm: Params, kappa: tuple, return_parts: bool = False,
                 pool=None) -> State:
    """One iteration of Algorithm 2.  pool: optional executor; the per-channel work
    (analysis, synthesis, data fidelity) is then mapped over it, channel by channel."""
    k1, k2, k3 = kappa
    L = prob.L
    if prm.wbar is not None:
        wbar = prm.wbar
    elif prm.prior == "sara":
        wbar = np.ones((prob.D, L, prob.ny, prob.nx))
    else:
        wbar = np.ones((prob.D, prob.ny, prob.nx))
    w = prm.w if prm.w is not None else np.ones(L)
    Xt = st.Xt
    t = st.t + 1

    use_nuc = prm.prior in ("lrjas", "lr")
    use_sp = prm.prior in ("lrjas", "jas", "sara")
    # low rankness dual
    P = prox.dual_nuclear(st.P, Xt, w, method="svd") if use_nuc else st.P
    # joint average sparsity duals (or per-channel l1 for SARA) and their synthesis
    if use_sp:
        PsiXt = np.concatenate(_map(pool, _psi_adj_chan, [(Xt[l:l + 1], prob.levels, prob.n_db) for l in range(L)]),
                               axis=1)
        if prm.prior == "sara":
            A = prox.dual_l1(st.A, PsiXt, wbar, prm.mu, float(prob.D))
        else:
            A = prox.dual_l21(st.A, PsiXt, wbar, prm.mu, float(prob.D))
        At_sum = np.concatenate(_map(pool, _psi_chan, [(A[:, l:l + 1], prob.levels) for l in range(L)]), axis=0)
    else:
        A, At_sum = st.A, np.zeros_like(Xt)
    # data fidelity duals, per (l, b); channels are independent (Phi is block diagonal)
    eps_prev = st.eps if st.eps is not None else [np.array(e) for e in prob.eps]
    vth_prev = st.vartheta if st.vartheta is not None else [np.zeros(len(e), np.int64) for e in prob.eps]
    args = [(Xt[l], st.v[l], prob.uv[l], prob.theta[l], prob.u[l], prob.y[l], prob.block_ptr[l], eps_prev[l],
             vth_prev[l], prob.ny, prob.nx, t, st.beta, prm.adaptive_eps, prm.lam1, prm.lam2, prm.lam3,
             prm.vartheta_bar) for l in range(L)]
    res = _map(pool, _data_channel, args)
    v_new = [r_[0] for r_ in res]
    data_adj = np.stack([r_[1] for r_ in res]) if L else np.zeros_like(Xt)
    lams = [r_[2] for r_ in res]
    rho = [r_[3] for r_ in res]
    eps_new = [r_[4] for r_ in res]
    vth_new = [r_[5] for r_ in res]
    # primal update
    G = (k1 * P if use_nuc else 0.0) + k2 * At_sum + k3 * data_adj
    X = prox.proj_pos(st.X - prm.tau * G)
    Xt_new = 2.0 * X - st.X
    nx_ = np.linalg.norm(X)
    beta = float(np.linalg.norm(X - st.X) / nx_) if nx_ > 0 else 0.0
    out = State(X=X, Xt=Xt_new, P=P, A=A, v=v_new, eps=eps_new, vartheta=vth_new, beta=beta, t=t)
    out.extra = {"lambda": lams, "rho": rho}
    if return_parts:
        out.extra.update({"At_sum": At_sum, "data_adj": data_adj, "G": G})
    return out


def objective_parts(X: np.ndarray, prob: Problem, prm: Params):
    """Weighted nuclear norm, weighted l2,1 norm of Psi^dag X and per-block residual norms."""
    w = prm.w if prm.w is not None else np.ones(prob.L)
    s = np.linalg.svd(X.reshape(prob.L, -1).T, compute_uv=False)
    nuc = float(np.sum(w[: len(s)] * s))
    C = wavelets.psi_adj(X, prob.levels, prob.n_db)
    wbar = prm.wbar if prm.wbar is not None else np.ones((prob.D, prob.ny, prob.nx))
    l21 = float(np.sum(wbar * np.sqrt(np.sum(C * C, axis=1))))
    res = []
    for l in range(prob.L):
        r = prob.y[l] - nufft.phi(X[l], prob.uv[l], prob.theta[l])
        bp = prob.block_ptr[l]
        res.append(np.array([np.linalg.norm(r[bp[b]:bp[b + 1]]) for b in range(len(bp) - 1)]))
    return nuc, l21, res


def dirty_cube(prob: Problem) -> np.ndarray:
    """x_l^dirty = eta_l Re Phi_l^dag y_l, eta_l = 1/max(Phi_l^dag Phi_l delta) (Sec. 4.3)."""
    out = np.zeros((prob.L, prob.ny, prob.nx))
    delta = np.zeros((prob.ny, prob.nx))
    delta[prob.ny // 2, prob.nx // 2] = 1.0
    for l in range(prob.L):
        psf = nufft.phi_adj(nufft.phi(delta, prob.uv[l], prob.theta[l]), prob.uv[l], prob.theta[l], prob.ny, prob.nx)
        eta = 1.0 / psf.max() if psf.max() > 0 else 0.0
        out[l] = eta * nufft.phi_adj(prob.y[l], prob.uv[l], prob.theta[l], prob.ny, prob.nx)
    return out


def mu_of_cube(X: np.ndarray, levels: int = 4, n_db: int = 8) -> float:
    """||X||_* / ||Psi^dag X||_{2,1} of a cube [L][ny][nx] (Sec. 2.3): the nuclear norm of
    the N x L matrix (column l = channel l) over the sum of the l2 norms of the
    length-L rows of the coefficients."""
    L = X.shape[0]
    nuc = float(np.sum(np.linalg.svd(X.reshape(L, -1).T, compute_uv=False)))
    C = wavelets.psi_adj(X, levels, n_db)
    l21 = float(np.sum(np.sqrt(np.sum(C * C, axis=1))))
    return nuc / l21 if l21 > 0 else 0.0


def mu_hat(prob: Problem) -> float:
    """mu_hat = ||X_dirty||_* / ||Psi^dag X_dirty||_{2,1} (Sec. 2.3)."""
    return mu_of_cube(dirty_cube(prob), prob.levels, prob.n_db)


def reweight(X: np.ndarray, prob: Problem, gamma: float, gamma_bar: float, prior: str = "lrjas"):
    """eq:weights-l21 and eq:weights-n from the current estimate.  For the SARA prior
    (a sequence of weighted l1 problems per channel, Sec. 2.3 and eq:min-sara) the
    weights are per channel and per coefficient, gamma_bar / (gamma_bar + |coefficient|),
    and there are no nuclear weights."""
    C = wavelets.psi_adj(X, prob.levels, prob.n_db)
    if prior == "sara":
        return gamma_bar / (gamma_bar + np.abs(C)), None   # [D][L][ny][nx]
    rn = np.sqrt(np.sum(C * C, axis=1))                   # [D][ny][nx]
    wbar = gamma_bar / (gamma_bar + rn)
    s = np.linalg.svd(X.reshape(prob.L, -1).T, compute_uv=False)
    w = gamma / (gamma + s)
    return wbar, w


def solve(prob: Problem, prm: Params, kappa: tuple, n_reweights: int, iters_per: int,
          factor: float = 0.8, st: State | None = None):
    """Algorithm 1: reweighted sequence of Algorithm 2 solves with warm starts."""
    st = zero_state(prob) if st is None else st
    gamma = gamma_bar = 1.0
    prm = Params(**{**prm.__dict__})
    history = []
    for k in range(n_reweights + 1):
        for _ in range(iters_per):
            st = pd_iteration(st, prob, prm, kappa)
        history.append(st.beta)
        if k == n_reweights:
            break
        prm.wbar, prm.w = reweight(st.X, prob, gamma, gamma_bar, prm.prior)
        gamma *= factor
        gamma_bar *= factor
    return st, prm, history


def _phi_unit(a):
    x, uv = a
    return nufft.phi(x, uv, np.ones(len(uv)))


def build_problem(cfg, inputs: dict, precond: str = "density", pool=None) -> Problem:
    """Oracle-side problem from the seeded workload draws: y0 = G F Z X0 (theta = 1),
    noisy data and bounds from ``workloads.make_measurements``, natural weighting
    y = theta * y_raw (Sec. 2.1), preconditioner from the density (or U = I)."""
    from workloads import make_measurements
    from .precond import density_precond

    uvs = inputs["uv"]
    y0 = _map(pool, _phi_unit, [(inputs["X0"][l], uvs[l]) for l in range(cfg.L)])
    y_raw, theta, eps = make_measurements(y0, inputs["noise"], inputs["block_ptr"], cfg.isnr_db)
    if precond == "density":
        u = [density_precond(uvs[l], cfg.nx, cfg.ny) for l in range(cfg.L)]
    else:
        u = [np.ones(len(uvs[l])) for l in range(cfg.L)]
    return Problem(nx=cfg.nx, ny=cfg.ny, uv=uvs, y=[theta[l] * y_raw[l] for l in range(cfg.L)],
                   theta=theta, u=u, eps=eps, block_ptr=inputs["block_ptr"]), y_raw
