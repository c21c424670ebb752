"""Pins of the FP64 primal-dual oracle (Algorithm 2) and the HyperSARA loop (Algorithm 1)."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import nufft, pd, prox, wavelets

GOLD = os.path.join(os.path.dirname(__file__), "golden", "appendix_a_constants.json")


def _tiny_problem(seed=0, nx=16, ny=16, L=2, m=120, B=2, eps_scale=1.0, y_zero=False, precond=True):
    rng = np.random.default_rng(seed)
    uv = [rng.normal(0, 0.12, (m, 2)).astype(np.float32).astype(np.float64) for _ in range(L)]
    th = [np.full(m, 2.0) for _ in range(L)]
    X0 = np.zeros((L, ny, nx))
    X0[:, ny // 2, nx // 2] = [1.0, 0.7][:L]
    X0[:, 5, 9] = 0.4
    bp = [np.array([(b * m) // B for b in range(B + 1)]) for _ in range(L)]
    y = []
    for l in range(L):
        yl = nufft.phi(X0[l], uv[l], th[l]) + 0.05 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
        y.append(np.zeros(m, complex) if y_zero else yl)
    from oracle.precond import density_precond
    u = [density_precond(uv[l], nx, ny) if precond else np.ones(m) for l in range(L)]
    eps = [eps_scale * np.sqrt(np.diff(bp[l]) * 0.05 ** 2 * 2 * 1.3) for l in range(L)]
    return pd.Problem(nx=nx, ny=ny, uv=uv, y=y, theta=th, u=u, eps=eps, block_ptr=bp), X0


def test_golden_constants_match_defaults():
    g = json.load(open(GOLD))
    prm = pd.Params(mu=0.01)
    assert (prm.lam1, prm.lam2, prm.lam3, prm.vartheta_bar) == (g["lambda1"], g["lambda2"], g["lambda3"], g["vartheta_bar"])
    assert 0 < prm.tau < g["tau_upper_bound_exclusive"]
    prob, _ = _tiny_problem()
    assert prob.D == g["dictionary_size_D"]
    k = pd.step_sizes(prob, prm, 4.0)
    assert k == (g["kappa1"], 1.0 / 9.0, 0.25)
    # convergence condition of Sec. 3.4: tau (k1 + k2 ||Psi^dag||^2 + k3 ||U^1/2 Phi||^2) < 1
    assert prm.tau * (k[0] + k[1] * 9.0 + k[2] * 4.0) < 1.0


def test_one_iteration_pieces_and_positivity():
    prob, X0 = _tiny_problem(1)
    cfg = W.CONFIGS["cube32_L3"].scaled(nx=16, ny=16, L=2)
    st0 = W.make_state(cfg, X0, [len(y) for y in prob.y])
    st = pd.State(X=st0["X"], Xt=st0["Xt"], P=st0["P"], A=st0["A"], v=st0["v"],
                  eps=[e.copy() for e in prob.eps], vartheta=[np.zeros(2, np.int64)] * 2)
    prm = pd.Params(mu=0.05, tau=0.3)
    nrm, _, _ = pd.op_norm_phi(prob, W.synth.power_start(cfg), tol=1e-12)
    kap = pd.step_sizes(prob, prm, nrm)
    out = pd.pd_iteration(st, prob, prm, kap, return_parts=True)
    assert np.all(out.X >= 0)
    # recompute the primal gradient with the pieces and an independent U = I-free path check
    G = kap[0] * out.P + kap[1] * out.extra["At_sum"] + kap[2] * out.extra["data_adj"]
    assert np.allclose(out.X, np.maximum(st.X - prm.tau * G, 0))
    assert np.allclose(out.Xt, 2 * out.X - st.X)
    # dual residual rows have norm <= mu * D * wbar (l2,1 dual is a ball projection)
    rn = np.sqrt(np.sum(out.A ** 2, axis=1))
    assert np.all(rn <= prm.mu * 9.0 * (1 + 1e-12))
    # every data dual v = vbar - U q with ||q - y|| <= eps
    for l in range(prob.L):
        vbar = st.v[l] + prob.u[l] * nufft.phi(st.Xt[l], prob.uv[l], prob.theta[l])
        q = (vbar - out.v[l]) / prob.u[l]
        bp = prob.block_ptr[l]
        for b in range(len(bp) - 1):
            s = slice(bp[b], bp[b + 1])
            assert np.linalg.norm(q[s] - prob.y[l][s]) <= prob.eps[l][b] * (1 + 1e-10)


def test_zero_is_the_solution_when_data_inside_balls():
    # ||y_b|| <= eps_b for every block: X = 0 is feasible and minimises the
    # (non-negative) objective uniquely, so the iteration must go to 0.
    prob, X0 = _tiny_problem(2, y_zero=True)
    prm = pd.Params(mu=0.05)
    nrm, _, _ = pd.op_norm_phi(prob, np.random.default_rng(0).standard_normal((2, 16, 16)), tol=1e-10)
    kap = pd.step_sizes(prob, prm, nrm)
    st = pd.zero_state(prob)
    st.X = X0.copy()
    st.Xt = X0.copy()
    for _ in range(300):
        st = pd.pd_iteration(st, prob, prm, kap)
    assert np.linalg.norm(st.X) < 1e-6 * np.linalg.norm(X0)


@pytest.mark.slow
def test_constraints_approached_at_convergence():
    # Well-conditioned tiny problem (M > N, uniform uv, U = I): the primal-dual
    # iterates approach feasibility and the objective settles.  PD converges
    # sublinearly, so the bound is checked to 3 % after 1200 iterations and the
    # residual must keep shrinking towards the ball.
    rng = np.random.default_rng(3)
    nx = ny = 16; L = 2; m = 600
    uv = [rng.uniform(-0.5, 0.5, (m, 2)).astype(np.float32).astype(np.float64) for _ in range(L)]
    th = [np.ones(m)] * L
    X0 = np.zeros((L, ny, nx)); X0[:, 8, 8] = [1.0, 0.7]; X0[:, 5, 9] = 0.4
    bp = [np.array([0, 300, 600])] * L
    y = [nufft.phi(X0[l], uv[l], th[l]) + 0.05 * (rng.standard_normal(m) + 1j * rng.standard_normal(m)) for l in range(L)]
    eps = [np.sqrt(np.diff(bp[l]) * 0.05 ** 2 * 2 * 1.3) for l in range(L)]
    prob = pd.Problem(nx=nx, ny=ny, uv=uv, y=y, theta=th, u=[np.ones(m)] * L, eps=eps, block_ptr=bp)
    prm = pd.Params(mu=0.02)
    nrm, _, _ = pd.op_norm_phi(prob, rng.standard_normal((2, 16, 16)), tol=1e-10)
    kap = pd.step_sizes(prob, prm, nrm)
    st = pd.zero_state(prob)
    ratio, objs = {}, []
    for it in range(1, 1201):
        st = pd.pd_iteration(st, prob, prm, kap)
        if it in (600, 1200):
            _, _, res = pd.objective_parts(st.X, prob, prm)
            ratio[it] = max(float(np.max(r / e)) for r, e in zip(res, prob.eps))
        if it >= 1000 and it % 100 == 0:
            nuc, l21, _ = pd.objective_parts(st.X, prob, prm)
            objs.append(nuc + prm.mu * l21)
    assert ratio[1200] <= 1.03 and ratio[1200] < ratio[600]
    assert abs(objs[-1] - objs[0]) <= 2e-3 * objs[-1]
    assert st.beta < 1e-4
    assert np.all(st.X >= 0)


def test_adaptive_eps_update_rule():
    # adaptive bounds with constants from Appendix A: force the update conditions
    prob, X0 = _tiny_problem(4)
    prm = pd.Params(mu=0.05, adaptive_eps=True, vartheta_bar=0)
    st = pd.zero_state(prob)
    st.X = X0.copy(); st.Xt = X0.copy(); st.beta = 0.0; st.t = 5
    out = pd.pd_iteration(st, prob, prm, (1.0, 1 / 9, 1e-3))
    for l in range(prob.L):
        for b in range(len(prob.eps[l])):
            rho = out.extra["rho"][l][b]
            e0 = prob.eps[l][b]
            if abs(rho - e0) / e0 > prm.lam2:
                assert out.eps[l][b] == pytest.approx(0.618 * rho + 0.382 * e0)
                assert out.vartheta[l][b] == 6
            else:
                assert out.eps[l][b] == e0


def test_reweighting_formulas():
    prob, X0 = _tiny_problem(5)
    wbar, w = pd.reweight(X0, prob, gamma=0.5, gamma_bar=0.25)
    C = wavelets.psi_adj(X0)
    rn = np.sqrt((C ** 2).sum(axis=1))
    assert np.allclose(wbar, 0.25 / (0.25 + rn))
    s = np.linalg.svd(X0.reshape(2, -1).T, compute_uv=False)
    assert np.allclose(w, 0.5 / (0.5 + s))
    assert np.all(np.diff(w) >= 0)          # non-decreasing: S*_w is then the exact prox


def _rank_two_cube(ny, nx, h1, h2):
    """X = 1 h1^T + C h2^T with C the checkerboard (-1)^(i+j): the two spatial
    factors are orthogonal, have norm sqrt(N), and their coefficients in every
    Daubechies basis are known in closed form (a constant keeps only its coarsest
    low-pass band, each coefficient 2^levels; the checkerboard keeps only its
    finest diagonal band, each coefficient 2, since H(pi) = 0 and |G(pi)| = sqrt(2))."""
    one = np.ones((ny, nx))
    chk = (-1.0) ** np.add.outer(np.arange(ny), np.arange(nx))
    return np.einsum("l,yx->lyx", h1, one) + np.einsum("l,yx->lyx", h2, chk)


def test_mu_of_cube_closed_form_rank_two():
    """mu = ||X||_* / ||Psi^dag X||_{2,1} (Sec. 2.3) on a cube whose singular values
    and coefficient rows are known exactly.  With a = ||h1||, b = ||h2|| (h1 _|_ h2):
    singular values sqrt(N) a and sqrt(N) b; Dirac rows all have norm sqrt(a^2 + b^2);
    each of the 8 wavelet bases has N/256 coarse rows of norm 16 a and N/4 diagonal
    rows of norm 2 b (4 levels)."""
    ny, nx, L = 32, 64, 5
    N = ny * nx
    rng = np.random.default_rng(21)
    h1 = rng.standard_normal(L)
    h2 = rng.standard_normal(L)
    h2 -= h1 * (h1 @ h2) / (h1 @ h1)
    a, b = np.linalg.norm(h1), np.linalg.norm(h2)
    X = _rank_two_cube(ny, nx, h1, h2)
    nuc = np.sqrt(N) * (a + b)
    l21 = N * np.sqrt(a * a + b * b) + 8 * (N / 256) * 16 * a + 8 * (N / 4) * 2 * b
    assert pd.mu_of_cube(X) == pytest.approx(nuc / l21, rel=1e-12)
    # a Frobenius norm in place of the nuclear norm, or the l1 norm of the entries in place
    # of the l2,1 norm of the rows, would give a different value on this cube
    assert abs(np.sqrt(N) * np.hypot(a, b) / l21 - nuc / l21) > 1e-3 * nuc / l21


def test_dirty_cube_against_brute_force_adjoint():
    """x_dirty_l = Re Phi_l^dag y_l / max PSF_l (Sec. 4.3).  The exact adjoint of the
    NUDFT is Re sum_m theta_m y_m e^{+2 pi i u_m . p}, and the PSF of a unit source at
    the phase centre peaks there at sum_m theta_m^2 (its NUDFT is theta_m): both by
    brute force, to the interpolation kernel's accuracy."""
    prob, _ = _tiny_problem(6)
    Xd = pd.dirty_cube(prob)
    py = np.arange(prob.ny) - prob.ny // 2
    px = np.arange(prob.nx) - prob.nx // 2
    for l in range(prob.L):
        uv, th, y = prob.uv[l], prob.theta[l], prob.y[l]
        ey = np.exp(2j * np.pi * uv[:, 1:2] * py[None, :])
        ex = np.exp(2j * np.pi * uv[:, 0:1] * px[None, :])
        adj = np.einsum("m,my,mx->yx", th * y, ey, ex).real
        ref = adj / np.sum(th * th)
        assert np.linalg.norm(Xd[l] - ref) <= 2e-6 * np.linalg.norm(ref)
    # the PSF of a unit source at the phase centre peaks there, at sum theta^2
    delta = np.zeros((prob.ny, prob.nx)); delta[prob.ny // 2, prob.nx // 2] = 1.0
    psf = nufft.phi_adj(nufft.phi(delta, prob.uv[0], prob.theta[0]), prob.uv[0], prob.theta[0], prob.ny, prob.nx)
    assert np.unravel_index(np.argmax(psf), psf.shape) == (prob.ny // 2, prob.nx // 2)
    assert psf.max() == pytest.approx(np.sum(prob.theta[0] ** 2), rel=1e-6)


def test_mu_hat_is_mu_of_the_dirty_cube():
    prob, _ = _tiny_problem(7)
    assert pd.mu_hat(prob) == pd.mu_of_cube(pd.dirty_cube(prob), prob.levels, prob.n_db)


def test_solve_without_reweights_is_the_plain_iteration():
    """Algorithm 1 with no reweight is T iterations of Algorithm 2 from the given state."""
    prob, X0 = _tiny_problem(8)
    prm = pd.Params(mu=0.02)
    kap = (1.0, 1.0 / 9.0, 1e-3)
    st0 = pd.zero_state(prob)
    st0.X = X0.copy(); st0.Xt = X0.copy()
    st_ref = st0
    for _ in range(4):
        st_ref = pd.pd_iteration(st_ref, prob, prm, kap)
    st, prm_out, hist = pd.solve(prob, prm, kap, n_reweights=0, iters_per=4, st=st0)
    for k in ("X", "Xt", "P", "A"):
        assert np.array_equal(getattr(st, k), getattr(st_ref, k)), k
    assert prm_out.w is None and prm_out.wbar is None and hist == [st_ref.beta]


def test_solve_gamma_sequence_and_weights(monkeypatch):
    """The weights the k-th reweight hands to the next solve (eq:weights-l21 and
    eq:weights-n) with gamma = gamma_bar = factor^(k-1), on an estimate X = 1 h^T whose
    singular values (sqrt(N) ||h||, then zeros) and coefficient rows (Dirac rows
    ||h||, coarsest low-pass rows 16 ||h|| in each wavelet basis, every other row 0)
    are known exactly.  The PD iteration is replaced by a stub returning that X."""
    prob, _ = _tiny_problem(9, L=2)
    N = prob.nx * prob.ny
    h = np.array([0.8, 0.3])
    Xr = _rank_two_cube(prob.ny, prob.nx, h, np.zeros(2))
    seen = []

    def stub(st, prob_, prm_, kappa, return_parts=False):
        seen.append((None if prm_.w is None else prm_.w.copy(), None if prm_.wbar is None else prm_.wbar.copy()))
        out = pd.State(X=Xr.copy(), Xt=Xr.copy(), P=st.P, A=st.A, v=st.v, eps=st.eps, vartheta=st.vartheta,
                       beta=0.5, t=st.t + 1)
        return out

    monkeypatch.setattr(pd, "pd_iteration", stub)
    factor = 0.7
    pd.solve(prob, pd.Params(mu=0.1), (1.0, 1.0 / 9.0, 1e-3), n_reweights=3, iters_per=2, factor=factor)
    assert len(seen) == 8
    assert seen[0][0] is None and seen[1][0] is None          # unit weights before the first reweight
    hn = np.linalg.norm(h)
    s1 = np.sqrt(N) * hn
    coarse = np.zeros((prob.ny, prob.nx), bool)
    coarse[: prob.ny // 16, : prob.nx // 16] = True
    for k in (1, 2, 3):
        g = factor ** (k - 1)
        for call in (2 * k, 2 * k + 1):
            w, wbar = seen[call]
            assert w[0] == pytest.approx(g / (g + s1), rel=1e-12)
            assert np.allclose(w[1:], 1.0, rtol=0, atol=1e-12)     # zero singular values
            assert np.allclose(wbar[0], g / (g + hn), rtol=1e-12)      # Dirac rows
            for d in range(1, 9):
                assert np.allclose(wbar[d][coarse], g / (g + 16 * hn), rtol=1e-10)
                assert np.allclose(wbar[d][~coarse], 1.0, rtol=0, atol=1e-10)


def test_workload_measurements_and_bounds():
    cfg = W.CONFIGS["cube64_L5"]
    inp = W.make_problem_inputs(cfg)
    prob, y_raw = pd.build_problem(cfg, inp)
    for l in range(cfg.L):
        m = len(prob.uv[l])
        bp = inp["block_ptr"][l]
        assert bp[0] == 0 and bp[-1] == m and np.all(np.diff(bp) >= 0)
        mb = np.diff(bp)
        assert np.allclose(prob.eps[l], np.sqrt(mb + 2 * np.sqrt(mb)))
        # whitened noise of each block is inside its bound with high probability
        y0 = nufft.phi(inp["X0"][l], prob.uv[l], np.ones(m))
        wn = prob.theta[l] * (y_raw[l] - y0)
        assert np.linalg.norm(wn) ** 2 == pytest.approx(m, rel=0.2)


def _variant_state(prob, seed):
    rng = np.random.default_rng(seed)
    L, ny, nx = prob.L, prob.ny, prob.nx
    X = np.abs(rng.standard_normal((L, ny, nx)))
    return pd.State(X=X, Xt=X + 0.1 * rng.standard_normal(X.shape), P=0.1 * rng.standard_normal(X.shape),
                    A=0.1 * rng.standard_normal((prob.D, L, ny, nx)),
                    v=[0.1 * (rng.standard_normal(len(u)) + 1j * rng.standard_normal(len(u))) for u in prob.uv])


def test_prior_variants_reduce_to_special_cases():
    """LR = LRJAS with mu = 0 and JAS = LRJAS with zero nuclear weights (eq:min-lr,
    eq:min-js, Sec. 4.2), for the primal update; SARA = JAS for a single channel."""
    prob, _ = _tiny_problem(2)
    st = _variant_state(prob, 5)
    k = (1.0, 1.0 / 9.0, 1e-3)
    lr = pd.pd_iteration(st, prob, pd.Params(mu=0.3, prior="lr"), k)
    ref = pd.pd_iteration(st, prob, pd.Params(mu=0.0, prior="lrjas"), k)
    assert np.allclose(lr.X, ref.X, rtol=0, atol=1e-14) and np.array_equal(lr.A, st.A)
    jas = pd.pd_iteration(st, prob, pd.Params(mu=0.3, prior="jas"), k)
    ref = pd.pd_iteration(st, prob, pd.Params(mu=0.3, w=np.zeros(prob.L), prior="lrjas"), k)
    assert np.allclose(jas.X, ref.X, rtol=0, atol=1e-14) and np.array_equal(jas.P, st.P)
    prob1, _ = _tiny_problem(1, L=1)
    st1 = _variant_state(prob1, 6)
    sara = pd.pd_iteration(st1, prob1, pd.Params(mu=0.3, prior="sara"), k)
    jas1 = pd.pd_iteration(st1, prob1, pd.Params(mu=0.3, prior="jas"), k)
    assert np.allclose(sara.X, jas1.X, rtol=0, atol=1e-14) and np.allclose(sara.A, jas1.A, rtol=0, atol=1e-14)


def test_sara_is_each_channel_on_its_own():
    """SARA (eq:min-sara) is one weighted-l1 problem per channel: one iteration of the
    two-channel SARA problem equals the two one-channel iterations, each with its own
    weights (channel 1's weights differ from channel 0's)."""
    prob, _ = _tiny_problem(3)
    st = _variant_state(prob, 7)
    k = (1.0, 1.0 / 9.0, 1e-3)
    rng = np.random.default_rng(12)
    wbar = rng.uniform(0.2, 1.0, (9, prob.L, prob.ny, prob.nx))
    both = pd.pd_iteration(st, prob, pd.Params(mu=0.3, prior="sara", wbar=wbar), k)
    for l in range(prob.L):
        one = pd.Problem(nx=prob.nx, ny=prob.ny, uv=[prob.uv[l]], y=[prob.y[l]], theta=[prob.theta[l]],
                         u=[prob.u[l]], eps=[prob.eps[l]], block_ptr=[prob.block_ptr[l]])
        s1 = pd.State(X=st.X[l:l + 1], Xt=st.Xt[l:l + 1], P=st.P[l:l + 1], A=st.A[:, l:l + 1], v=[st.v[l]])
        r1 = pd.pd_iteration(s1, one, pd.Params(mu=0.3, prior="sara", wbar=wbar[:, l:l + 1]), k)
        assert np.allclose(both.X[l], r1.X[0], rtol=0, atol=1e-14)
        assert np.allclose(both.A[:, l], r1.A[:, 0], rtol=0, atol=1e-14)


def test_sara_reweighting_closed_form():
    """SARA's reweighted l1 (Sec. 2.3): weight gamma_bar / (gamma_bar + |coefficient|) per
    channel, on X = 1 h^T: Dirac coefficients h_l, coarsest low-pass 16 h_l, others 0."""
    prob, _ = _tiny_problem(4, L=2)
    h = np.array([0.9, -0.4])
    X = _rank_two_cube(prob.ny, prob.nx, h, np.zeros(2))
    wbar, w = pd.reweight(X, prob, 1.0, 0.5, prior="sara")
    assert w is None and wbar.shape == (9, 2, prob.ny, prob.nx)
    coarse = np.zeros((prob.ny, prob.nx), bool)
    coarse[: prob.ny // 16, : prob.nx // 16] = True
    for l in range(2):
        assert np.allclose(wbar[0, l], 0.5 / (0.5 + abs(h[l])), rtol=1e-12)
        for d in range(1, 9):
            assert np.allclose(wbar[d, l][coarse], 0.5 / (0.5 + 16 * abs(h[l])), rtol=1e-10)
            assert np.allclose(wbar[d, l][~coarse], 1.0, rtol=0, atol=1e-10)


def test_pooled_iteration_is_the_same_iteration():
    """Mapping the per-channel work over a process pool changes nothing."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    prob, X0 = _tiny_problem(10, L=2)
    st = pd.zero_state(prob)
    st.X = X0.copy(); st.Xt = X0 + 0.01
    prm = pd.Params(mu=0.02)
    kap = (1.0, 1.0 / 9.0, 1e-3)
    ref = pd.pd_iteration(st, prob, prm, kap)
    with ProcessPoolExecutor(max_workers=2, mp_context=multiprocessing.get_context("spawn")) as ex:
        got = pd.pd_iteration(st, prob, prm, kap, pool=ex)
    for k in ("X", "Xt", "P", "A"):
        assert np.array_equal(getattr(got, k), getattr(ref, k)), k
    for l in range(prob.L):
        assert np.array_equal(got.v[l], ref.v[l]) and np.array_equal(got.extra["rho"][l], ref.extra["rho"][l])
