"""Autograd wrappers of Phi, Re Phi^dagger, Psi^dagger and Psi, and the l2,1 term
with checkpointed per-channel recomputation.

Gradients must be the adjoint maps: checked by torch's gradcheck in FP64,
against the oracle's adjoints for a data-fidelity + l21 loss, and by central
finite differences on the full 512x512x60 cube (h = 1e-3).  The checkpointed
l2,1 term is checked against the oracle's value and subgradient, against the
gradient composed from the whole coefficient array, and for its memory."""
import numpy as np
import pytest

import workloads as W
from oracle import wavelets
from gpu_cases import TOL, gpu_case, host, oracle_case, rel, split, to_dev

pytestmark = pytest.mark.gpu


def _rand(torch, prob, shape, seed, complex_=False):
    g = torch.Generator(device="cpu").manual_seed(seed)
    if complex_:
        t = torch.complex(torch.randn(shape, generator=g, dtype=torch.float64),
                          torch.randn(shape, generator=g, dtype=torch.float64))
        return t.to(prob.device, prob.cdtype)
    return torch.randn(shape, generator=g, dtype=torch.float64).to(prob.device, prob.tdtype)


@pytest.mark.parametrize("op", ["phi", "phi_adj", "psi_adj", "psi"])
def test_gradcheck_f64(op):
    import torch
    from paper_1806_04596_amd import autograd as AG
    prob, _, _ = gpu_case("cube32_L3", "f64")
    shapes = {"phi": (prob.L, prob.ny, prob.nx), "phi_adj": (prob.M,), "psi_adj": (prob.L, prob.ny, prob.nx),
              "psi": (prob.D, prob.L, prob.ny, prob.nx)}
    x = _rand(torch, prob, shapes[op], 10, complex_=(op == "phi_adj")).requires_grad_(True)
    fn = getattr(AG, op)
    assert torch.autograd.gradcheck(lambda t: fn(prob, t), (x,), eps=1e-6, atol=1e-7, rtol=1e-6, fast_mode=True)
    assert torch.autograd.gradgradcheck(lambda t: fn(prob, t), (x,), eps=1e-6, atol=1e-7, rtol=1e-6,
                                        fast_mode=True)


def test_backward_is_the_adjoint_call():
    import torch
    from paper_1806_04596_amd import autograd as AG
    prob, _, _ = gpu_case("cube64_L5", "f32")
    x = _rand(torch, prob, (prob.L, prob.ny, prob.nx), 11).requires_grad_(True)
    gy = _rand(torch, prob, (prob.M,), 12, complex_=True)
    AG.phi(prob, x).backward(gy)
    assert torch.equal(x.grad, prob.phi_adj(gy.contiguous()))
    c = _rand(torch, prob, (prob.D, prob.L, prob.ny, prob.nx), 13).requires_grad_(True)
    gx = _rand(torch, prob, (prob.L, prob.ny, prob.nx), 14)
    AG.psi(prob, c).backward(gx)
    assert torch.equal(c.grad, prob.psi_adj(gx))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_loss_gradient_vs_oracle(dtype):
    """grad of 0.5||Phi X - y||^2 + lam sum_r ||(Psi^dag X)_r||_2 against the oracle's
    Re Phi^dag (Phi X - y) + lam Psi (C_r / ||C_r||)."""
    import torch
    from paper_1806_04596_amd import autograd as AG
    cfg, inp, op = oracle_case("cube64_L5")
    prob, _, _ = gpu_case("cube64_L5", dtype)
    rng = np.random.default_rng(20)
    X = inp["X0"] + 0.05 * np.abs(rng.standard_normal(inp["X0"].shape)) * inp["X0"].max()
    y = rng.standard_normal(prob.M) + 1j * rng.standard_normal(prob.M)
    lam = 0.3
    Xt = to_dev(prob, X).requires_grad_(True)
    yt = to_dev(prob, y, complex_=True)
    r = AG.phi(prob, Xt) - yt
    C = AG.psi_adj(prob, Xt)
    loss = 0.5 * (r.abs() ** 2).sum() + lam * C.pow(2).sum(dim=1).sqrt().sum()
    loss.backward()
    g = host(Xt.grad)
    ys = split(y, prob.counts)
    res = [a - b for a, b in zip(op.phi(X), ys)]
    Cr = wavelets.psi_adj(X, 4, 8)
    nr = np.sqrt(np.sum(Cr * Cr, axis=1, keepdims=True))
    ref = op.phi_adj(res) + lam * wavelets.psi(Cr / nr, 4)
    err = rel(g, ref)
    assert err <= TOL[dtype], err


def test_psi_on_channel_chunks_equals_whole_cube():
    """Psi^dagger and Psi of a chunk of channels are the whole-cube results of those
    channels, bit for bit (the same kernels with fewer channels)."""
    import torch
    prob, _, _ = gpu_case("cube64_L5", "f32")
    X = _rand(torch, prob, (prob.L, prob.ny, prob.nx), 40)
    Cf = prob.psi_adj(X)
    Cr = _rand(torch, prob, (prob.D, prob.L, prob.ny, prob.nx), 41)
    Xf = prob.psi(Cr)
    for l0, n in ((0, 1), (1, 2), (3, 2), (0, prob.L)):
        assert torch.equal(prob.psi_adj(X[l0:l0 + n].contiguous()), Cf[:, l0:l0 + n])
        assert torch.equal(prob.psi(Cr[:, l0:l0 + n].contiguous()), Xf[l0:l0 + n])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("chunk", [1, 2, 5])
@pytest.mark.parametrize("weighted", [False, True])
def test_checkpointed_l21_vs_oracle(dtype, chunk, weighted):
    """The checkpointed l2,1 term sum_r wbar_r ||(Psi^dag X)_r|| and its gradient
    wbar_r Psi (C_r / ||C_r||) against the oracle, for chunks of 1, 2 and all 5
    channels, with and without weights; zero rows (a zero pixel in every channel)
    take the zero subgradient on both sides."""
    import torch
    from paper_1806_04596_amd import autograd as AG
    cfg, inp, op = oracle_case("cube64_L5")
    prob, _, _ = gpu_case("cube64_L5", dtype)
    rng = np.random.default_rng(50)
    X = inp["X0"] + 0.05 * rng.standard_normal(inp["X0"].shape) * inp["X0"].max()
    X[:, :, :8] = 0.0          # whole zero rows of the Dirac basis
    Xr = to_dev(prob, X)
    X = host(Xr)               # the values the library sees
    wbar = rng.uniform(0.2, 1.0, (prob.D, cfg.ny, cfg.nx)) if weighted else None
    wd = None if wbar is None else to_dev(prob, wbar)
    if wbar is not None:
        wbar = host(wd)
    Xg = Xr.clone().requires_grad_(True)
    val = AG.l21_psi_adj(prob, Xg, wd, chunk=chunk)
    val.backward()
    Cr = wavelets.psi_adj(X, 4, 8)
    nr = np.sqrt(np.sum(Cr * Cr, axis=1, keepdims=True))
    w = np.ones((prob.D, 1, cfg.ny, cfg.nx)) if wbar is None else wbar[:, None]
    ref_val = float(np.sum(w * nr))
    ref_grad = wavelets.psi(np.where(nr > 0, w * Cr / np.where(nr > 0, nr, 1.0), 0.0), 4)
    assert abs(float(val.detach()) - ref_val) <= TOL[dtype] * ref_val
    assert rel(host(Xg.grad), ref_grad) <= TOL[dtype]


@pytest.mark.slow
def test_checkpointed_l21_full_cube_memory_and_gradient():
    """512x512x60: the checkpointed l2,1 gradient equals the one composed from the whole
    coefficient array, and its extra device memory is one chunk's coefficients plus the
    row sums, not the [D][L][ny][nx] array."""
    import torch
    from paper_1806_04596_amd import autograd as AG
    from paper_1806_04596_amd.workload import build_problem
    cfg = W.CONFIGS["cube512_L60_autograd"]
    inp = W.make_problem_inputs(cfg)
    prob, X0, _ = build_problem(cfg, inp, W.make_measurements, dtype="f32")
    X = (X0 + 0.01 * float(X0.max()) * _rand(torch, prob, X0.shape, 32).abs()).contiguous()
    torch.cuda.synchronize()

    def run(fn):
        Xg = X.clone().requires_grad_(True)
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        fn(Xg).backward()
        torch.cuda.synchronize()
        return Xg.grad, torch.cuda.max_memory_allocated() - base

    g_full, m_full = run(lambda Z: AG.psi_adj(prob, Z).double().pow(2).sum(dim=1).sqrt().sum())
    chunk = 4
    g_ck, m_ck = run(lambda Z: AG.l21_psi_adj(prob, Z, chunk=chunk))
    N = prob.nx * prob.ny
    coef_bytes = prob.D * prob.L * N * 4
    print(f"peak extra memory: whole {m_full / 1e6:.0f} MB, checkpointed (chunk {chunk}) {m_ck / 1e6:.0f} MB; "
          f"whole coefficient array {coef_bytes / 1e6:.0f} MB", flush=True)
    # chunk coefficients (psi_adj output and its rescaled copy) + S + the gradient cube
    bound = 2 * prob.D * chunk * N * 4 + prob.D * N * 8 + 2 * prob.L * N * 4
    assert m_ck <= bound, (m_ck, bound)
    assert m_ck < m_full / 3
    assert rel(host(g_ck), host(g_full)) <= TOL["f32"]
    prob.close()


@pytest.mark.slow
def test_full_cube_finite_differences():
    """512x512x60 (16 M visibilities): central differences with h = 1e-3 on the
    data-fidelity + l21 loss with lam = mu_hat (Sec. 2.3) match the directional
    derivative from autograd along 8 random directions.  The differences are taken in the FP64
    instantiation (an FP32 loss near 1e10 rounds by more than the 2h-scaled
    change it has to resolve); the FP32 gradient is then checked against the
    FP64 one on the same cube."""
    import torch
    from paper_1806_04596_amd import autograd as AG
    from paper_1806_04596_amd.workload import build_problem
    cfg = W.CONFIGS["cube512_L60_autograd"]
    inp = W.make_problem_inputs(cfg)
    grads = {}
    data = None
    for dtype in ("f64", "f32"):
        # the FP32 problem takes the data the FP64 build formed: one problem, two precisions
        prob, X0, hd = build_problem(cfg, inp, W.make_measurements, dtype=dtype, data=data)
        data = {"y_raw": hd["y_raw"], "theta": hd["theta"], "eps": hd["eps"]}
        y = to_dev(prob, np.concatenate([t * yr for t, yr in zip(hd["theta"], hd["y_raw"])]), complex_=True)
        if dtype == "f64":
            # mu_hat = ||X_dirty||_* / ||Psi^dag X_dirty||_{2,1}; X_dirty = Re Phi^dag y over the PSF peak
            delta = torch.zeros_like(X0)
            delta[:, prob.ny // 2, prob.nx // 2] = 1
            peak = prob.phi_adj(prob.phi(delta))[:, prob.ny // 2, prob.nx // 2]
            Xd = prob.phi_adj(y) / peak[:, None, None]
            nuc = torch.linalg.svdvals(Xd.reshape(prob.L, -1).T).sum()
            lam = float(nuc / prob.psi_adj(Xd).pow(2).sum(1).sqrt().sum())
            amp = float(X0.max())
        X = (X0 + 0.01 * amp * _rand(torch, prob, X0.shape, 30).abs()).contiguous()

        def loss(Z):
            r = (AG.phi(prob, Z) - y).to(torch.complex128)
            # the l2,1 term with checkpointed per-channel recomputation (4 channels at a time)
            return 0.5 * (r.abs() ** 2).sum() + lam * AG.l21_psi_adj(prob, Z, chunk=4)

        Xg = X.clone().requires_grad_(True)
        loss(Xg).backward()
        grads[dtype] = Xg.grad.double()
        if dtype == "f64":
            # central differences along 8 seeded random directions
            h = 1e-3
            for k in range(8):
                d = 0.01 * amp * _rand(torch, prob, X0.shape, 31 + k)
                with torch.no_grad():
                    fd = float((loss(X + h * d) - loss(X - h * d)) / (2 * h))
                an = float((grads[dtype] * d).sum())
                assert abs(fd - an) <= 1e-6 * abs(an), (k, fd, an)
        prob.close()
        del prob, X0, y, X, Xg
    err = float((grads["f32"] - grads["f64"]).norm() / grads["f64"].norm())
    assert err <= TOL["f32"], err
