"""Thin Python front end of the C ABI: one ``Problem`` per context.

Argument marshalling only -- every operator runs in the HIP kernels of
libhypersara.so.  Torch provides device memory (the workspace and the
caller's tensors) and the stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


def _require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise L.HSError("a HIP device is required (no CPU fallback)")
    # initialise the HIP runtime and the device context before the library's
    # first runtime call (counting devices does not initialise it)
    torch.cuda.init()
    torch.empty(1, device="cuda").zero_()
    return torch


class Problem:
    """A HyperSARA measurement/prior configuration bound to one GPU.

    channels: list of dicts with keys uv [M][2], y_raw [M] complex, theta [M],
    block_ptr [B+1], eps [B] and optionally precond [M] (None = U = I).
    """

    def __init__(self, nx: int, ny: int, channels, dtype: str = "f32", levels: int = 4, n_db: int = 8,
                 tile: int = 0, device: int = 0, stream=None, gram_mode: str = "f64", autotune: bool = False,
                 tune_cache: str | None = None, tuning: dict | None = None, per_channel: bool = False):
        """autotune: pick the batching decomposition with hs_autotune (timed on this GPU,
        cached in tune_cache, default the package's tuning_cache.jsonl); tuning: an
        explicit decomposition (hs_set_tuning fields) instead."""
        torch = _require_gpu()
        self.torch = torch
        self.lib = L.load()
        self.nx, self.ny, self.L = nx, ny, len(channels)
        self.levels, self.n_db, self.D = levels, n_db, 1 + n_db
        self.dtype = dtype
        self.tdtype = torch.float32 if dtype == "f32" else torch.float64
        self.cdtype = torch.complex64 if dtype == "f32" else torch.complex128
        self.device = torch.device("cuda", device)
        # a dedicated (default-priority) stream so one PD iteration can be captured in a HIP graph
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        desc = L.ProblemDesc(nx=nx, ny=ny, L=self.L, oversamp=2, J=8, levels=levels, n_db=n_db,
                             dtype=L.HS_F32 if dtype == "f32" else L.HS_F64, tile=tile, device=device,
                             stream=C.c_void_p(self.stream.cuda_stream), gram_mode=L.GRAM_MODES[gram_mode],
                             per_channel=1 if per_channel else 0)
        self.gram_mode = gram_mode
        ctx = C.c_void_p()
        L.check(self.lib.hs_create(C.byref(desc), C.byref(ctx)), None, "hs_create")
        self.ctx = ctx
        self.counts = []
        self.nblocks = []
        self._block_ptrs = []
        for l, ch in enumerate(channels):
            uv = np.ascontiguousarray(ch["uv"], dtype=np.float64)
            M = uv.shape[0]
            y = np.ascontiguousarray(np.asarray(ch["y_raw"], dtype=np.complex128)).view(np.float64)
            th = np.ascontiguousarray(ch["theta"], dtype=np.float64)
            bp = np.ascontiguousarray(ch["block_ptr"], dtype=np.int64)
            eps = np.ascontiguousarray(ch["eps"], dtype=np.float64)
            pre = ch.get("precond")
            pre = None if pre is None else np.ascontiguousarray(pre, dtype=np.float64)
            self._chk(self.lib.hs_set_channel(ctx, l, M, len(bp) - 1, L.as_i64p(bp), L.as_dptr(uv), L.as_dptr(y),
                                              L.as_dptr(th), L.as_dptr(pre), L.as_dptr(eps)), "hs_set_channel")
            self.counts.append(M)
            self.nblocks.append(len(bp) - 1)
            self._block_ptrs.append(bp.copy())
        if tuning:
            t = L.Tuning(**{k: int(v) for k, v in tuning.items() if k != "ms"})
            self._chk(self.lib.hs_set_tuning(ctx, C.byref(t)), "hs_set_tuning")
        ws = C.c_size_t()
        self._chk(self.lib.hs_plan(ctx, C.byref(ws)), "hs_plan")
        if autotune:
            tb = C.c_size_t()
            self._chk(self.lib.hs_autotune_bytes(ctx, C.byref(tb)), "hs_autotune_bytes")
            tmp = torch.empty(tb.value + 256, dtype=torch.uint8, device=self.device)
            cache = (tune_cache or L.TUNING_CACHE).encode()
            chosen = L.Tuning()
            torch.cuda.synchronize(self.device)
            self._chk(self.lib.hs_autotune(ctx, C.c_void_p((tmp.data_ptr() + 255) // 256 * 256), tb.value, cache,
                                           C.byref(chosen)), "hs_autotune")
            del tmp
            self._chk(self.lib.hs_plan(ctx, C.byref(ws)), "hs_plan")
        self.ws_bytes = ws.value
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._chk(self.lib.hs_bind_workspace(ctx, C.c_void_p(self._ws_ptr), self.ws_bytes), "hs_bind_workspace")
        self.M = int(sum(self.counts))

    # ------------------------------------------------------------ helpers
    def _chk(self, status, what):
        L.check(status, self.ctx, what)

    def _enter(self):
        # order the library's stream after the caller's work on its current stream
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)
        return cur

    def _leave(self, cur):
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def _call(self, what, fn, *args):
        cur = self._enter()
        try:
            self._chk(fn(self.ctx, *args), what)
        finally:
            self._leave(cur)

    @staticmethod
    def _p(t):
        return C.c_void_p(t.data_ptr()) if t is not None else None

    def set_launch_tuning(self, **fields):
        """Changes the launch-time fields of the decomposition (fft_col_tile,
        grid_xcd_group, degrid_xcd_group); the plan and the bound state are kept."""
        launch = ("fft_col_tile", "grid_xcd_group", "degrid_xcd_group")
        bad = [k for k in fields if k not in launch]
        if bad:
            raise L.HSError(f"set_launch_tuning: {bad} shape the plan; pass them to the constructor")
        cur = self.tuning()
        cur.update({k: int(v) for k, v in fields.items()})
        t = L.Tuning(**{k: v for k, v in cur.items()})
        self._chk(self.lib.hs_set_tuning(self.ctx, C.byref(t)), "hs_set_tuning")

    def tuning(self):
        t = L.Tuning()
        self._chk(self.lib.hs_get_tuning(self.ctx, C.byref(t)), "hs_get_tuning")
        return {k: getattr(t, k) for k, _ in L.Tuning._fields_}

    def info(self):
        i = L.Info()
        self._chk(self.lib.hs_get_info(self.ctx, C.byref(i)), "hs_get_info")
        return {k: getattr(i, k) for k, _ in L.Info._fields_}

    def empty_cube(self):
        return self.torch.empty((self.L, self.ny, self.nx), dtype=self.tdtype, device=self.device)

    def empty_vis(self):
        return self.torch.empty(self.M, dtype=self.cdtype, device=self.device)

    def empty_coef(self):
        return self.torch.empty((self.D, self.L, self.ny, self.nx), dtype=self.tdtype, device=self.device)

    def _check_cube(self, X, shape=None):
        shape = shape or (self.L, self.ny, self.nx)
        if X.dtype != self.tdtype or tuple(X.shape) != tuple(shape) or not X.is_contiguous() or X.device != self.device:
            raise L.HSError(f"expected contiguous {self.tdtype} {shape} on {self.device}")

    def _check_vis(self, Y):
        if Y.dtype != self.cdtype or Y.numel() != self.M or not Y.is_contiguous() or Y.device != self.device:
            raise L.HSError(f"expected contiguous {self.cdtype} [{self.M}] on {self.device}")

    def set_data(self, l, y_raw, theta, eps):
        y = np.ascontiguousarray(np.asarray(y_raw, dtype=np.complex128)).view(np.float64)
        th = np.ascontiguousarray(theta, dtype=np.float64)
        ep = np.ascontiguousarray(eps, dtype=np.float64)
        self._call("hs_set_data", self.lib.hs_set_data, int(l), L.as_dptr(y), L.as_dptr(th), L.as_dptr(ep))

    # ----------------------------------------------------------- operators
    def phi(self, X, Y=None):
        self._check_cube(X)
        Y = self.empty_vis() if Y is None else Y
        self._check_vis(Y)
        self._call("hs_phi", self.lib.hs_phi, self._p(X), self._p(Y))
        return Y

    def phi_adj(self, Y, X=None):
        self._check_vis(Y)
        X = self.empty_cube() if X is None else X
        self._check_cube(X)
        self._call("hs_phi_adj", self.lib.hs_phi_adj, self._p(Y), self._p(X))
        return X

    def _nch(self, X, lead):
        """Channel count of a cube ([n][ny][nx], lead = 0) or coefficient array
        ([D][n][ny][nx], lead = 1) of 1..L channels."""
        n = X.shape[lead] if X.dim() == 3 + lead else -1
        if not 1 <= n <= self.L:
            raise L.HSError(f"expected 1..{self.L} channels, got shape {tuple(X.shape)}")
        return n

    def psi_adj(self, X, Cc=None):
        """Psi^dagger of L channels, or of a chunk of n < L contiguous channels."""
        n = self._nch(X, 0)
        self._check_cube(X, (n, self.ny, self.nx))
        Cc = self.torch.empty((self.D, n, self.ny, self.nx), dtype=self.tdtype, device=self.device) if Cc is None else Cc
        self._check_cube(Cc, (self.D, n, self.ny, self.nx))
        self._call("hs_psi_adj_n", self.lib.hs_psi_adj_n, self._p(X), self._p(Cc), n)
        return Cc

    def psi(self, Cc, X=None):
        """Psi of L channels' coefficients, or of a chunk of n < L channels."""
        n = self._nch(Cc, 1)
        self._check_cube(Cc, (self.D, n, self.ny, self.nx))
        X = self.torch.empty((n, self.ny, self.nx), dtype=self.tdtype, device=self.device) if X is None else X
        self._check_cube(X, (n, self.ny, self.nx))
        self._call("hs_psi_n", self.lib.hs_psi_n, self._p(Cc), self._p(X), n)
        return X

    def _check_rowsq(self, S):
        if S.dtype != self.torch.float64 or tuple(S.shape) != (self.D, self.ny, self.nx) or not S.is_contiguous() \
                or S.device != self.device:
            raise L.HSError(f"expected contiguous float64 {(self.D, self.ny, self.nx)} on {self.device}")

    def l21_rowsq(self, Cc, S, accumulate=False):
        """S (+)= the per-row sums of squares of the chunk's coefficients Cc [D][n][ny][nx]."""
        n = self._nch(Cc, 1)
        self._check_cube(Cc, (self.D, n, self.ny, self.nx))
        self._check_rowsq(S)
        self._call("hs_l21_rowsq", self.lib.hs_l21_rowsq, self._p(Cc), n, self._p(S), int(bool(accumulate)))
        return S

    def l21_rowscale(self, Cc, S, wbar=None, scale=1.0):
        """Cc <- scale * wbar * Cc / ||row|| in place (the l2,1 gradient of the chunk)."""
        n = self._nch(Cc, 1)
        self._check_cube(Cc, (self.D, n, self.ny, self.nx))
        self._check_rowsq(S)
        if wbar is not None:
            self._check_cube(wbar, (self.D, self.ny, self.nx))
        self._call("hs_l21_rowscale", self.lib.hs_l21_rowscale, self._p(Cc), n, self._p(S), self._p(wbar),
                   float(scale))
        return Cc

    def l21_from_rowsq(self, S, wbar=None):
        """sum wbar * sqrt(S) (host float; synchronising)."""
        self._check_rowsq(S)
        if wbar is not None:
            self._check_cube(wbar, (self.D, self.ny, self.nx))
        v = C.c_double()
        self._call("hs_l21_from_rowsq", self.lib.hs_l21_from_rowsq, self._p(S), self._p(wbar), C.byref(v))
        return v.value

    def prox_l21(self, A, t, wbar=None):
        self._check_cube(A, (self.D, self.L, self.ny, self.nx))
        if wbar is not None:
            self._check_cube(wbar, (self.D, self.ny, self.nx))
        self._call("hs_prox_l21", self.lib.hs_prox_l21, self._p(A), self._p(wbar), float(t))
        return A

    def dual_l21(self, A, Xt, mu, wbar=None, want_sum=False):
        self._check_cube(A, (self.D, self.L, self.ny, self.nx))
        self._check_cube(Xt)
        if wbar is not None:
            self._check_cube(wbar, (self.D, self.ny, self.nx))
        S = self.empty_cube() if want_sum else None
        self._call("hs_dual_l21", self.lib.hs_dual_l21, self._p(A), self._p(Xt), self._p(wbar), float(mu), self._p(S))
        return (A, S) if want_sum else A

    def _w(self, w):
        if w is None:
            return None, None
        wa = np.ascontiguousarray(w, dtype=np.float64)
        return wa, L.as_dptr(wa)

    def prox_nuclear(self, X, w=None):
        self._check_cube(X)
        wa, wp = self._w(w)
        sig = np.zeros(self.L)
        self._call("hs_prox_nuclear", self.lib.hs_prox_nuclear, self._p(X), wp, L.as_dptr(sig))
        return X, sig

    def dual_nuclear(self, P, Xt, w=None):
        self._check_cube(P)
        self._check_cube(Xt)
        wa, wp = self._w(w)
        self._call("hs_dual_nuclear", self.lib.hs_dual_nuclear, self._p(P), self._p(Xt), wp)
        return P

    def dual_data(self, v, Xt, want_adj=False):
        self._check_vis(v)
        self._check_cube(Xt)
        adj = self.empty_cube() if want_adj else None
        self._call("hs_dual_data", self.lib.hs_dual_data, self._p(v), self._p(Xt), self._p(adj))
        return (v, adj) if want_adj else v

    def proj_ellipsoid(self, l, b, z):
        if not (0 <= l < self.L and 0 <= b < self.nblocks[l]):
            raise L.HSError(f"no block {b} in channel {l}")
        mb = int(self._block_ptrs[l][b + 1] - self._block_ptrs[l][b])
        if z.dtype != self.cdtype or z.numel() != mb or not z.is_contiguous() or z.device != self.device:
            raise L.HSError(f"expected contiguous {self.cdtype} [{mb}] on {self.device}")
        self._call("hs_proj_ellipsoid", self.lib.hs_proj_ellipsoid, int(l), int(b), self._p(z))
        return z

    def op_norm(self, x0=None, max_it=1000, tol=1e-10, which="phi"):
        out = C.c_double()
        per = np.zeros(self.L)
        it = C.c_int32()
        if which == "psi":
            self._call("hs_op_norm", self.lib.hs_op_norm, L.HS_NORM_PSI, 1, 0.0, None, C.byref(out), None, C.byref(it))
            return out.value, None, 0
        self._check_cube(x0)
        self._call("hs_op_norm", self.lib.hs_op_norm, L.HS_NORM_PHI_PRECOND, int(max_it), float(tol), self._p(x0),
                                      C.byref(out), L.as_dptr(per), C.byref(it))
        return out.value, per, it.value

    def dirty_mu(self, want_cube=True):
        """(mu_hat, X_dirty or None): the dirty cube and mu_hat of Sec. 2.3."""
        Xd = self.empty_cube() if want_cube else None
        mu = C.c_double()
        self._call("hs_dirty_mu", self.lib.hs_dirty_mu, self._p(Xd), C.byref(mu))
        return mu.value, Xd

    # ----------------------------------------------------------------- PD
    def pd_init(self, mu, tau, kappa3, kappa1=1.0, kappa2=0.0, wbar=None, w=None, adaptive_eps=False,
                lam1=5e-4, lam2=0.01, lam3=0.618, vartheta_bar=100, prior="lrjas"):
        if wbar is not None:
            self._check_cube(wbar, self.wbar_shape(prior))
        self._wkeep = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        if self._wkeep is not None and self._wkeep.shape != (self.L,):
            raise L.HSError(f"nuclear weights: expected [{self.L}]")
        prm = L.PDParams(mu=mu, tau=tau, kappa1=kappa1, kappa2=kappa2, kappa3=kappa3,
                         wbar=None if wbar is None else wbar.data_ptr(),
                         w=None if self._wkeep is None else L.as_dptr(self._wkeep),
                         adaptive_eps=1 if adaptive_eps else 0, lam1=lam1, lam2=lam2, lam3=lam3,
                         vartheta_bar=vartheta_bar, prior=L.PRIORS[prior])
        self._call("hs_pd_init", self.lib.hs_pd_init, C.byref(prm))

    def wbar_shape(self, prior="lrjas"):
        """Shape of the sparsity weights: one per coefficient row [D][ny][nx], or per
        channel [D][L][ny][nx] for the SARA prior."""
        if prior == "sara":
            return (self.D, self.L, self.ny, self.nx)
        return (self.D, self.ny, self.nx)

    def _state(self, X=None, Xt=None, P=None, A=None, v=None, eps=None, vartheta=None, scalars=None, wbar=None,
               w=None):
        f = lambda t: None if t is None else t.data_ptr()
        return L.StatePtrs(X=f(X), Xt=f(Xt), P=f(P), A=f(A), v=f(v),
                           eps=None if eps is None else L.as_dptr(eps),
                           vartheta=None if vartheta is None else vartheta.ctypes.data_as(C.POINTER(C.c_int32)),
                           scalars=None if scalars is None else L.as_dptr(scalars), wbar=f(wbar),
                           w=None if w is None else L.as_dptr(w))

    def set_state(self, X=None, Xt=None, P=None, A=None, v=None, eps=None, vartheta=None, beta=None, t=None,
                  wbar=None, w=None, prior="lrjas"):
        """Restores a state of Algorithm 2.  eps, vartheta (per block), beta and t, and the
        weights wbar and w are optional: the bookkeeping not given restarts (the data's
        bounds, vartheta = 0, beta = 1, t = 0) and the weights not given are kept."""
        for tt in (X, Xt, P):
            if tt is not None:
                self._check_cube(tt)
        if A is not None:
            self._check_cube(A, (self.D, self.L, self.ny, self.nx))
        if v is not None:
            self._check_vis(v)
        if wbar is not None:
            self._check_cube(wbar, self.wbar_shape(prior))
        nb = int(sum(self.nblocks))
        ep = None if eps is None else np.ascontiguousarray(eps, dtype=np.float64)
        vt = None if vartheta is None else np.ascontiguousarray(vartheta, dtype=np.int32)
        if (ep is not None and ep.shape != (nb,)) or (vt is not None and vt.shape != (nb,)):
            raise L.HSError(f"eps and vartheta: expected [{nb}]")
        if (beta is None) != (t is None):
            raise L.HSError("give beta and t together")
        sc = None if beta is None else np.array([beta, t], dtype=np.float64)
        wa = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        if wa is not None and wa.shape != (self.L,):
            raise L.HSError(f"nuclear weights: expected [{self.L}]")
        st = self._state(X, Xt, P, A, v, ep, vt, sc, wbar, wa)
        self._call("hs_pd_set_state", self.lib.hs_pd_set_state, C.byref(st))

    def get_state(self, full=False, prior="lrjas"):
        """The state of Algorithm 2; with full=True also eps, vartheta, beta, t and the
        weights wbar and w."""
        X, Xt, P = self.empty_cube(), self.empty_cube(), self.empty_cube()
        A, v = self.empty_coef(), self.empty_vis()
        out = {"X": X, "Xt": Xt, "P": P, "A": A, "v": v}
        if full:
            nb = int(sum(self.nblocks))
            out.update(eps=np.zeros(nb), vartheta=np.zeros(nb, np.int32), scalars=np.zeros(2),
                       wbar=self.torch.empty(self.wbar_shape(prior), dtype=self.tdtype, device=self.device),
                       w=np.zeros(self.L))
            st = self._state(X, Xt, P, A, v, out["eps"], out["vartheta"], out["scalars"], out["wbar"], out["w"])
        else:
            st = self._state(X, Xt, P, A, v)
        self._call("hs_pd_get_state", self.lib.hs_pd_get_state, C.byref(st))
        if full:
            sc = out.pop("scalars")
            out["beta"], out["t"] = float(sc[0]), int(sc[1])
        return out

    def iterate(self, n=1):
        self._call("hs_pd_iterate", self.lib.hs_pd_iterate, int(n))

    def profile_phases(self, n=5):
        t = np.zeros(len(L.PHASES))
        self._call("hs_profile_phases", self.lib.hs_profile_phases, int(n), L.as_dptr(t))
        return dict(zip(L.PHASES, t.tolist()))

    def diag(self):
        out = np.zeros(4)
        self._call("hs_get_diag", self.lib.hs_get_diag, L.as_dptr(out), 4)
        return {"beta": out[0], "device_iterations": out[1], "eig_sweeps": out[2], "host_iterations": out[3]}

    def stats(self):
        nb = int(sum(self.nblocks))
        beta = C.c_double()
        rho = np.zeros(nb)
        eps = np.zeros(nb)
        self._call("hs_pd_stats", self.lib.hs_pd_stats, C.byref(beta), L.as_dptr(rho), L.as_dptr(eps))
        return beta.value, rho, eps

    def solve(self, n_reweights, iters_per_reweight, gamma_factor=0.8, beta_tol=0.0, check_every=0, gamma0=1.0,
              gamma_bar0=1.0, reweight_first=False):
        X = self.empty_cube()
        prm = L.SolveParams(n_reweights=n_reweights, iters_per_reweight=iters_per_reweight,
                            gamma_factor=gamma_factor, beta_tol=beta_tol, check_every=check_every, gamma0=gamma0,
                            gamma_bar0=gamma_bar0, reweight_first=1 if reweight_first else 0)
        rep = L.Report()
        self._call("hs_solve", self.lib.hs_solve, C.byref(prm), self._p(X), C.byref(rep))
        return X, {"iterations": rep.iterations, "reweights": rep.reweights, "final_beta": rep.final_beta,
                   "gamma": rep.gamma, "gamma_bar": rep.gamma_bar}

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.hs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------- host utilities
def density_precond(uv: np.ndarray, nx: int, ny: int) -> np.ndarray:
    lib = L.load()
    uv = np.ascontiguousarray(uv, dtype=np.float64)
    out = np.empty(uv.shape[0])
    L.check(lib.hs_density_precond(uv.shape[0], L.as_dptr(uv), nx, ny, L.as_dptr(out)), None, "hs_density_precond")
    return out


def visibility_order(uv, precond, block_ptr, nx, ny, tile):
    lib = L.load()
    uv = np.ascontiguousarray(uv, dtype=np.float64)
    M = uv.shape[0]
    pre = None if precond is None else np.ascontiguousarray(precond, dtype=np.float64)
    bp = np.ascontiguousarray(block_ptr, dtype=np.int64)
    perm = np.empty(M, dtype=np.int64)
    ntr = (nx // tile + 1) * (2 * ny // tile) * 9
    rp = np.empty(ntr + 1, dtype=np.int64)
    L.check(lib.hs_visibility_order(M, L.as_dptr(uv), L.as_dptr(pre), len(bp) - 1, L.as_i64p(bp), nx, ny, tile,
                                    L.as_i64p(perm), L.as_i64p(rp)), None, "hs_visibility_order")
    return perm, rp


def daubechies_filter(K: int) -> np.ndarray:
    lib = L.load()
    h = np.empty(2 * K)
    L.check(lib.hs_daubechies_filter(K, L.as_dptr(h)), None, "hs_daubechies_filter")
    return h
