"""Autograd wrappers of Phi, Re Phi^dagger, Psi^dagger and Psi.

Gradients must be the adjoint maps: checked by torch's gradcheck in FP64,
against the oracle's adjoints for a data-fidelity + l21 loss, and by central
finite differences on the full 512x512x60 cube in FP32 (h = 1e-3)."""
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


@pytest.mark.slow
def test_full_cube_finite_differences():
    """512x512x60 (16 M visibilities): central differences with h = 1e-3 on the
    data-fidelity + l21 loss with lam = mu_hat (Sec. 2.3) match the directional
    derivative from autograd.  The differences are taken in the FP64
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
            C = AG.psi_adj(prob, Z).double()
            return 0.5 * (r.abs() ** 2).sum() + lam * C.pow(2).sum(dim=1).sqrt().sum()

        Xg = X.clone().requires_grad_(True)
        loss(Xg).backward()
        grads[dtype] = Xg.grad.double()
        if dtype == "f64":
            d = 0.01 * amp * _rand(torch, prob, X0.shape, 31)
            h = 1e-3
            with torch.no_grad():
                fd = float((loss(X + h * d) - loss(X - h * d)) / (2 * h))
            an = float((grads[dtype] * d).sum())
            assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
        prob.close()
        del prob, X0, y, X, Xg
    err = float((grads["f32"] - grads["f64"]).norm() / grads["f64"].norm())
    assert err <= TOL["f32"], err
