"""CPU-side checks of the C-ABI library: it loads, exports every declared entry
point, and its host logic (density preconditioner, visibility order, filter
generation) agrees with the oracle's definitions bit for bit where integer."""
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import binning, precond, wavelets

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hypersara.h")


def _lib():
    from paper_1806_04596_amd import _lib as L
    return L.load(), L


def test_library_exports_every_declared_symbol():
    lib, L = _lib()
    text = open(HEADER).read()
    declared = sorted(set(re.findall(r"^\s*(?:hs_status|const char\*)\s+(hs_\w+)\s*\(", text, re.M)))
    assert len(declared) >= 28
    for name in declared:
        assert hasattr(lib, name), name
        assert name in L.SIGNATURES, f"binding lacks {name}"


def test_status_strings():
    lib, L = _lib()
    assert lib.hs_status_string(0) == b"ok"
    assert lib.hs_status_string(-7) == b"HIP runtime error"


def test_density_precond_bit_exact():
    from paper_1806_04596_amd import density_precond
    for name in ("cube64_L5", "cube128x64_L4"):
        cfg = W.CONFIGS[name]
        uvs, _ = W.synth.make_uv(cfg)
        for uv in uvs:
            a = density_precond(uv, cfg.nx, cfg.ny)
            b = precond.density_precond(uv, cfg.nx, cfg.ny)
            assert np.array_equal(a, b)


@pytest.mark.parametrize("name,tile,pre", [("cube32_L3", 8, True), ("cube64_L5", 16, True), ("cube64_L5", 32, False),
                                           ("cube128x64_L4", 16, True), ("cube64_L5", 16, "continuous")])
def test_visibility_order_bit_exact(name, tile, pre):
    from paper_1806_04596_amd import visibility_order
    cfg = W.CONFIGS[name]
    uvs, bps = W.synth.make_uv(cfg)
    rng = np.random.default_rng(3)
    for uv, bp in zip(uvs, bps):
        u = precond.density_precond(uv, cfg.nx, cfg.ny) if pre else None
        if pre == "continuous":       # a distinct value for almost every visibility
            u = u * rng.uniform(0.5, 1.0, len(u))
        perm, rp = visibility_order(uv, u, bp, cfg.nx, cfg.ny, tile)
        perm_o, rp_o = binning.order(uv, u, bp, cfg.nx, cfg.ny, tile)
        assert np.array_equal(perm, perm_o)
        assert np.array_equal(rp, rp_o)


def test_visibility_order_edge_cases():
    from paper_1806_04596_amd import visibility_order
    # empty channel, points exactly on grid nodes / tile borders, |u| > 1/2
    uv = np.array([[0.0, 0.0], [0.25, -0.25], [-0.5, 0.5], [0.49999, -0.49999], [1.75, -3.125],
                   [1 / 32, 1 / 32], [-1 / 64, 3 / 64]])
    bp = np.array([0, 3, 7])
    perm, rp = visibility_order(uv, None, bp, 16, 16, 8)
    perm_o, rp_o = binning.order(uv, None, bp, 16, 16, 8)
    assert np.array_equal(perm, perm_o) and np.array_equal(rp, rp_o)
    perm, rp = visibility_order(np.zeros((0, 2)), None, np.array([0, 0]), 16, 16, 8)
    assert perm.size == 0 and rp[-1] == 0


def test_daubechies_filters_match_oracle():
    from paper_1806_04596_amd import daubechies_filter
    for K in range(1, 9):
        assert np.allclose(daubechies_filter(K), wavelets.daubechies(K), rtol=0, atol=1e-14)


def test_create_without_gpu_fails_cleanly():
    import ctypes as C
    lib, L = _lib()
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("GPU present")
    except Exception:
        pass
    desc = L.ProblemDesc(nx=32, ny=32, L=2, oversamp=2, J=8, levels=4, n_db=8, dtype=0, tile=0, device=0, stream=None)
    ctx = C.c_void_p()
    st = lib.hs_create(C.byref(desc), C.byref(ctx))
    assert st == -7 and not ctx.value
    # argument validation happens before the device check
    bad = L.ProblemDesc(nx=30, ny=32, L=2, oversamp=2, J=8, levels=4, n_db=8, dtype=0, tile=0, device=0, stream=None)
    assert lib.hs_create(C.byref(bad), C.byref(ctx)) == -2
    bad.nx, bad.dtype = 32, 7
    assert lib.hs_create(C.byref(bad), C.byref(ctx)) == -3


def test_product_path_refuses_without_gpu():
    import paper_1806_04596_amd as H
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("GPU present")
    except Exception:
        pass
    with pytest.raises(H.HSError):
        H.Problem(32, 32, [dict(uv=np.zeros((1, 2)), y_raw=np.zeros(1), theta=np.ones(1),
                                block_ptr=np.array([0, 1]), eps=np.ones(1))])


def test_single_hip_runtime_in_process():
    # the library must share torch's HIP runtime, never load a second one
    import re
    from paper_1806_04596_amd import _lib as L
    L.load()
    maps = open("/proc/self/maps").read()
    libs = set(re.findall(r"/\S*libamdhip64\S*", maps))
    assert len(libs) == 1, libs


def _bare_problem():
    """A Problem with its shape fields set and no context: the binding's argument checks
    run before any library call, so they can be exercised without a GPU."""
    import torch
    from paper_1806_04596_amd.problem import Problem
    p = Problem.__new__(Problem)
    p.torch = torch
    p.nx, p.ny, p.L, p.D, p.M = 8, 8, 2, 9, 5
    p.tdtype, p.cdtype = torch.float64, torch.complex128
    p.device = torch.device("cpu")
    p.nblocks = [1, 1]
    p._block_ptrs = [np.array([0, 3]), np.array([0, 2])]
    p.ctx = None

    def no_call(*a, **k):
        raise AssertionError("the library was called")
    p._call = no_call
    return p


def test_binding_rejects_bad_state_and_weights_before_calling_the_library():
    import torch
    from paper_1806_04596_amd._lib import HSError
    p = _bare_problem()
    cube = torch.zeros(2, 8, 8, dtype=torch.float64)
    bad = [dict(X=torch.zeros(2, 8, 8, dtype=torch.float32)),            # dtype
           dict(Xt=torch.zeros(2, 8, 7, dtype=torch.float64)),            # shape
           dict(P=torch.zeros(8, 2, 8, dtype=torch.float64).transpose(0, 1)),  # not contiguous
           dict(A=torch.zeros(8, 2, 8, 8, dtype=torch.float64)),          # D
           dict(v=torch.zeros(4, dtype=torch.complex128)),                # M
           dict(v=torch.zeros(5, dtype=torch.complex64)),                 # complex dtype
           dict(wbar=torch.zeros(9, 8, 8, dtype=torch.float64), prior="sara"),   # SARA weights per channel
           dict(eps=np.ones(3)), dict(vartheta=np.zeros(1)), dict(beta=0.5),
           dict(w=np.ones(3))]
    for kw in bad:
        with pytest.raises(HSError):
            p.set_state(X=cube, **kw) if "X" not in kw else p.set_state(**kw)
    with pytest.raises(HSError):
        p.pd_init(mu=0.1, tau=0.3, kappa3=1.0, wbar=torch.zeros(9, 2, 8, 8, dtype=torch.float64))
    with pytest.raises(HSError):
        p.pd_init(mu=0.1, tau=0.3, kappa3=1.0, w=np.ones(3))
    with pytest.raises(HSError):
        p.prox_l21(torch.zeros(9, 2, 8, 8, dtype=torch.float64), 0.1, wbar=torch.zeros(9, 8, 9, dtype=torch.float64))
    with pytest.raises(HSError):
        p.proj_ellipsoid(0, 0, torch.zeros(2, dtype=torch.complex128))     # block 0 of channel 0 has 3
    with pytest.raises(HSError):
        p.proj_ellipsoid(1, 1, torch.zeros(2, dtype=torch.complex128))     # no block 1 in channel 1
    with pytest.raises(HSError):
        p.proj_ellipsoid(0, 0, torch.zeros(3, dtype=torch.complex64))
