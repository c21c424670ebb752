"""The nuclear prox without allocation (hs_prox_nuclear_noalloc, scratch in a fixed
device array) against hs_prox_nuclear of a context, through the C ABI: two calls in a
row, the second on a smaller cube, in FP64 and FP32."""
import ctypes as C

import numpy as np
import pytest

from oracle import prox
from gpu_cases import TOL, check_rel, gpu_case, host, oracle_case, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(prob, X, w):
    from paper_1806_04596_amd import _lib as L
    lib = L.load()
    wa = np.ascontiguousarray(w, dtype=np.float64)
    sig = np.zeros(prob.L)
    prob.torch.cuda.synchronize()
    st = L.check(lib.hs_prox_nuclear_noalloc(C.c_void_p(X.data_ptr()), L.HS_F32 if prob.dtype == "f32" else L.HS_F64,
                                             prob.nx * prob.ny, prob.L, L.as_dptr(wa), L.as_dptr(sig),
                                             C.c_void_p(prob.stream.cuda_stream), prob.device.index or 0),
                 None, "hs_prox_nuclear_noalloc")
    return X, sig


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_nuclear_prox_matches_context_entry_point(dtype):
    for name in ("cube64_L5", "cube32_L3"):          # the second call is on a smaller cube
        cfg, inp, _ = oracle_case(name)
        prob, _, _ = gpu_case(name, dtype)
        rng = np.random.default_rng(60)
        X = inp["X0"] + 0.01 * rng.standard_normal(inp["X0"].shape)
        s_ref = np.linalg.svd(X.reshape(cfg.L, -1).T, compute_uv=False)
        w = np.sort(rng.uniform(0.0, 0.5 * s_ref[0], cfg.L))
        prob.set_state()                              # fresh eigen-solver start for the context call
        Xc, sc = prob.prox_nuclear(to_dev(prob, X), w)
        Xn, sn = _noalloc(prob, to_dev(prob, X), w)
        tol = TOL[dtype]
        check_rel(host(Xn), host(Xc), tol, f"{name}: X against hs_prox_nuclear")
        check_rel(sn, sc, tol, f"{name}: sigma against hs_prox_nuclear")
        ref, s = prox.prox_nuclear_svd(X, w)
        check_rel(host(Xn), ref, tol, f"{name}: X against the oracle")
        check_rel(sn, s, tol, f"{name}: sigma against the oracle")


def test_noalloc_rejects_sizes_beyond_its_scratch():
    from paper_1806_04596_amd import _lib as L
    lib = L.load()
    prob, _, _ = gpu_case("cube32_L3", "f64")
    X = prob.empty_cube()
    assert lib.hs_prox_nuclear_noalloc(C.c_void_p(X.data_ptr()), L.HS_F64, prob.nx * prob.ny, 65, None, None,
                                       C.c_void_p(prob.stream.cuda_stream), 0) == -2
    assert lib.hs_prox_nuclear_noalloc(C.c_void_p(X.data_ptr()), L.HS_F64, 0, 3, None, None,
                                       C.c_void_p(prob.stream.cuda_stream), 0) == -1
