// C ABI entry points: lifecycle, workspace, operators, proxes and the PD solver.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <fstream>
#include <sstream>

#include "hs_internal.h"

namespace hs {

static std::string g_create_err;

hs_status fail(hs_ctx* c, hs_status s, const std::string& msg) {
    if (c) c->err = msg;
    else g_create_err = msg;
    return s;
}

hs_status hip_check(hs_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return HS_OK;
    return fail(c, HS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

hs_status build_plan(hs_ctx* c);

// ------------------------------------------------------------ workspace layout
struct Carver {
    size_t off = 0;
    template <typename P>
    void take(P*& p, size_t bytes, char* base) {
        off = (off + 255) & ~(size_t)255;
        p = base ? reinterpret_cast<P*>(base + off) : nullptr;
        off += std::max<size_t>(bytes, 1);
    }
};

static size_t carve(hs_ctx* c, char* base) {
    Carver k;
    Dev& d = c->d;
    const size_t r = c->rsz, cx = 2 * c->rsz;
    const size_t M = (size_t)c->Mtot, LN = (size_t)c->L * c->N;
    k.take(d.vis_cell, M * 4, base);
    k.take(d.vis_frac, M * cx, base);
    k.take(d.vis_y, M * cx, base);
    k.take(d.vis_theta, M * r, base);
    k.take(d.vis_u, M * r, base);
    k.take(d.vis_bin, M * 4, base);
    k.take(d.vis_perm, M * 4, base);
    k.take(d.vis_pos, M * 4, base);
    k.take(d.v, M * cx, base);
    k.take(d.vwork, M * cx, base);
    k.take(d.dunits, c->dunits.size() * sizeof(DegridUnit), base);
    k.take(d.gunits, c->gunits.size() * sizeof(GridUnit), base);
    k.take(d.splits, c->splits.size() * sizeof(SplitTile), base);
    k.take(d.glist, c->h_glist.size() * 4, base);
    k.take(d.gpartial, (size_t)c->npartial * GB * GB * cx, base);
    k.take(d.bin_u, (size_t)c->nbins * 8, base);
    k.take(d.blk_bin_ptr, (size_t)(c->nblk + 1) * 4, base);
    k.take(d.blk_eps, (size_t)c->nblk * 8, base);
    k.take(d.blk_lambda, (size_t)c->nblk * 8, base);
    k.take(d.blk_rho2, (size_t)c->nblk * 8, base);
    k.take(d.blk_vartheta, (size_t)c->nblk * 4, base);
    k.take(d.run_sum, (size_t)c->nruns * 16, base);
    k.take(d.bin_run_ptr, (size_t)(c->nbins + 1) * 4, base);
    k.take(d.run_slot, (size_t)c->nruns * 4, base);
    k.take(d.chunk_run, c->h_chunk_run.size() * 4, base);
    k.take(d.bin_S, (size_t)c->nbins * 16, base);
    k.take(d.bin_f, (size_t)c->nbins * 8, base);
    k.take(d.grid, (size_t)c->L * c->Ky * c->Wg * cx, base);
    k.take(d.H, (size_t)c->L * c->ny * c->Hs * cx, base);
    k.take(d.tw_x, (size_t)c->Kx * cx, base);
    k.take(d.tw_y, (size_t)c->Ky * cx, base);
    k.take(d.sx, (size_t)c->nx * r, base);
    k.take(d.sy, (size_t)c->ny * r, base);
    k.take(d.X, LN * r, base);
    k.take(d.Xt, LN * r, base);
    k.take(d.P, LN * r, base);
    k.take(d.img0, LN * r, base);
    k.take(d.img1, LN * r, base);
    k.take(d.A, (size_t)c->D * LN * r, base);
    k.take(d.coef, (size_t)std::max(c->n_db, 1) * LN * r, base);
    k.take(d.wtmp, (size_t)std::max(c->n_db, 1) * LN * r, base);
    k.take(d.wbar, (size_t)c->D * LN * r, base);   // per channel for the SARA prior
    k.take(d.filt, (size_t)MAX_DB * 32 * r, base);
    k.take(d.gram_part, (size_t)NGRAM * MAX_L * MAX_L * 8, base);
    k.take(d.gram, (size_t)MAX_L * MAX_L * 8, base);
    k.take(d.eigV, (size_t)MAX_L * MAX_L * 8, base);
    k.take(d.eig_sig, (size_t)MAX_L * 8, base);
    k.take(d.w_nuc, (size_t)MAX_L * 8, base);
    k.take(d.Wmat, (size_t)MAX_L * MAX_L * r, base);
    k.take(d.red_part, (size_t)std::max<int64_t>(NRED * 4, 64 * MAX_L) * 8, base);
    k.take(d.scal, 64 * 8, base);
    k.take(d.chan_nrm, (size_t)MAX_L * 8, base);
    if (c->dtype == HS_F32) {   // FP64 copies for the power iteration
        Dev64& e = c->d64;
        k.take(e.vis_frac, M * 16, base);
        k.take(e.vis_theta, M * 8, base);
        k.take(e.vis_u, M * 8, base);
        k.take(e.vwork, M * 16, base);
        k.take(e.gpartial, (size_t)c->npartial * GB * GB * 16, base);
        k.take(e.grid, (size_t)c->L * c->Ky * c->Wg * 16, base);
        k.take(e.H, (size_t)c->L * c->ny * c->Hs * 16, base);
        k.take(e.tw_x, (size_t)c->Kx * 16, base);
        k.take(e.tw_y, (size_t)c->Ky * 16, base);
        k.take(e.sx, (size_t)c->nx * 8, base);
        k.take(e.sy, (size_t)c->ny * 8, base);
        k.take(e.x, LN * 8, base);
    }
    return (k.off + 255) & ~(size_t)255;
}

template <typename T>
static void upload_real(hs_ctx* c, void* dst, const std::vector<double>& src) {
    std::vector<T> tmp(src.begin(), src.end());
    if (!tmp.empty()) (void)hipMemcpy(dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice);
}

template <typename V>
static void upload(void* dst, const std::vector<V>& src) {
    if (!src.empty()) (void)hipMemcpy(dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice);
}

// Algorithm 2's initial values: t = 0, beta = 1 (the adaptive-bound test cannot fire before a
// real iteration), the l2 bounds given by hs_set_data and their last-update
// iterations vartheta = 0.
static void restart_counters(hs_ctx* c, bool scalars = true, bool vartheta = true, bool eps = true) {
    if (scalars) {
        launch_fill<double>(c->stream, c->d.scal, 1.0, 1);
        launch_fill<double>(c->stream, c->d.scal + 1, 0.0, 1);
    }
    if (vartheta) launch_fill<int32_t>(c->stream, c->d.blk_vartheta, 0, c->nblk);
    if (eps && c->nblk)
        hipMemcpyAsync(c->d.blk_eps, c->h_blk_eps.data(), (size_t)c->nblk * 8, hipMemcpyHostToDevice, c->stream);
}

// Elements of the sparsity weights for the current prior: one per coefficient row,
// or per channel and coefficient (SARA).
static int64_t wbar_elems(const hs_ctx* c) {
    return (int64_t)c->D * c->N * (c->prior == HS_PRIOR_SARA ? c->L : 1);
}

template <typename T>
static hs_status bind_impl(hs_ctx* c) {
    Dev& d = c->d;
    upload(d.vis_cell, c->h_cell);
    upload_real<T>(c, d.vis_frac, c->h_frac);
    upload_real<T>(c, d.vis_y, c->h_y);
    upload_real<T>(c, d.vis_theta, c->h_theta);
    upload_real<T>(c, d.vis_u, c->h_u);
    upload(d.vis_bin, c->h_bin);
    upload(d.vis_perm, c->h_perm);
    {
        std::vector<int32_t> pos(c->h_pos_of.begin(), c->h_pos_of.end());
        upload(d.vis_pos, pos);
    }
    upload(d.dunits, c->dunits);
    upload(d.gunits, c->gunits);
    upload(d.splits, c->splits);
    upload(d.glist, c->h_glist);
    upload(d.bin_u, c->h_bin_u);
    upload(d.blk_bin_ptr, c->h_blk_bin_ptr);
    upload(d.blk_eps, c->h_blk_eps);
    upload(d.bin_run_ptr, c->h_bin_run_ptr);
    upload(d.run_slot, c->h_run_slot);
    upload(d.chunk_run, c->h_chunk_run);
    // FFT twiddles exp(-2 pi i k / K) and deapodisation 1/phihat(p/K)
    const long double pi = 3.141592653589793238462643383279502884L;
    const bool shadow = c->dtype == HS_F32;
    for (int dim = 0; dim < 2; ++dim) {
        const int K = dim == 0 ? c->Kx : c->Ky;
        std::vector<double> tw(2 * (size_t)K);
        for (int k = 0; k < K; ++k) {
            const long double a = 2.0L * pi * (long double)k / (long double)K;
            tw[2 * k] = (double)std::cos(a);
            tw[2 * k + 1] = (double)(-std::sin(a));
        }
        upload_real<T>(c, dim == 0 ? d.tw_x : d.tw_y, tw);
        if (shadow) upload_real<double>(c, dim == 0 ? c->d64.tw_x : c->d64.tw_y, tw);
        const int n = dim == 0 ? c->nx : c->ny;
        std::vector<double> s(n);
        for (int i = 0; i < n; ++i) s[i] = 1.0 / kb_ft((double)(i - n / 2) / (double)K);
        upload_real<T>(c, dim == 0 ? d.sx : d.sy, s);
        if (shadow) upload_real<double>(c, dim == 0 ? c->d64.sx : c->d64.sy, s);
    }
    if (shadow) {
        upload_real<double>(c, c->d64.vis_frac, c->h_frac);
        upload_real<double>(c, c->d64.vis_theta, c->h_theta);
        upload_real<double>(c, c->d64.vis_u, c->h_u);
    }
    {
        std::vector<double> f((size_t)MAX_DB * 32, 0.0);
        for (int b = 0; b < c->n_db; ++b) {
            const int K = b + 1;
            double h[2 * MAX_DB];
            daubechies_host(K, h);
            for (int j = 0; j < 2 * K; ++j) {
                f[b * 32 + j] = h[j];
                f[b * 32 + 16 + j] = ((j & 1) ? -1.0 : 1.0) * h[2 * K - 1 - j];
            }
        }
        upload_real<T>(c, d.filt, f);
    }
    {
        std::vector<double> I((size_t)MAX_L * MAX_L, 0.0);
        for (int i = 0; i < MAX_L; ++i) I[i * MAX_L + i] = 1.0;
        upload(d.eigV, I);
        std::vector<double> ones(MAX_L, 1.0);
        upload(d.w_nuc, ones);
    }
    const int64_t LN = (int64_t)c->L * c->N;
    launch_fill<T>(c->stream, (T*)d.X, T(0), LN);
    launch_fill<T>(c->stream, (T*)d.Xt, T(0), LN);
    launch_fill<T>(c->stream, (T*)d.P, T(0), LN);
    launch_fill<T>(c->stream, (T*)d.A, T(0), (int64_t)c->D * LN);
    launch_fill<T>(c->stream, (T*)d.v, T(0), 2 * c->Mtot);
    launch_fill<T>(c->stream, (T*)d.wbar, T(1), (int64_t)c->D * LN);
    launch_fill<double>(c->stream, d.scal, 0.0, 64);
    restart_counters(c);
    launch_fill<double>(c->stream, d.blk_lambda, 0.0, c->nblk);
    launch_fill<double>(c->stream, d.blk_rho2, 0.0, c->nblk);
    return hip_check(c, hipStreamSynchronize(c->stream), "hs_bind_workspace");
}

// ------------------------------------------------------------- operator bodies
// F Z of X into the grid: all channels in one launch per pass, or (plain execution,
// lc >= 0) channel lc only.
template <typename T>
static void fft_fwd(hs_ctx* c, const T* X, int lc = -1) {
    const int L = lc < 0 ? c->L : 1, l0 = lc < 0 ? 0 : lc;
    launch_fft_rows_fwd<T>(c, X, L, l0);
    launch_fft_cols_fwd<T>(c, L, l0);
}

template <typename T>
static void phi_impl(hs_ctx* c, const T* X, cplx<T>* Y) {
    if (!c->per_channel) {
        fft_fwd<T>(c, X);
        launch_degrid_plain<T>(c, Y);
        return;
    }
    for (int l = 0; l < c->L; ++l) {
        fft_fwd<T>(c, X, l);
        launch_degrid_plain<T>(c, Y, l);
    }
}

// grid-order visibility values (already weighted) -> Re Z^T F^H G^T vals
template <typename T>
static void adj_from_grid_order(hs_ctx* c, const cplx<T>* vals, const T* weight, T* X, int lc = -1) {
    const int L = lc < 0 ? c->L : 1, l0 = lc < 0 ? 0 : lc;
    if (lc < 0 && c->per_channel) {
        for (int l = 0; l < c->L; ++l) adj_from_grid_order<T>(c, vals, weight, X, l);
        return;
    }
    launch_grid_pull<T>(c, vals, weight, lc);
    launch_fft_cols_adj<T>(c, L, l0);
    launch_fft_rows_adj<T>(c, X, L, l0);
}

template <typename T>
static void phi_adj_impl(hs_ctx* c, const cplx<T>* Y, T* X) {
    launch_gather_user<T>(c, Y, (cplx<T>*)c->d.vwork, true);
    adj_from_grid_order<T>(c, (const cplx<T>*)c->d.vwork, nullptr, X);
}

// Event hook between the phases of one iteration (diagnostics only).
struct PhaseMarks {
    hipEvent_t* ev = nullptr;
    void mark(hs_ctx* c, int k) const {
        if (ev) (void)hipEventRecord(ev[k], c->stream);
    }
};

// Data-fidelity dual of Algorithm 2 on v (grid order, in place); its adjoint G^T Theta^T
// and F^H Z^T into adj if given.
template <typename T>
static void dual_data_impl(hs_ctx* c, cplx<T>* v, const T* Xt, T* adj, const PhaseMarks& pm = PhaseMarks(),
                           bool do_fft_fwd = true, hipEvent_t after_degrid = nullptr) {
    if (c->per_channel) {
        // plain execution: the whole chain channel by channel, one launch per kernel and channel
        for (int l = 0; l < c->L; ++l) {
            fft_fwd<T>(c, Xt, l);
            launch_degrid_dual_v<T>(c, v, l);
            launch_bins_and_roots<T>(c, l);
            launch_dual_apply_v<T>(c, v, l);
            if (adj) adj_from_grid_order<T>(c, v, (const T*)c->d.vis_theta, adj, l);
        }
        for (int k = HS_PH_FFT_FWD; k <= HS_PH_FFT_ADJ; ++k) pm.mark(c, k + 1);
        if (after_degrid) (void)hipEventRecord(after_degrid, c->stream);
        return;
    }
    if (do_fft_fwd) fft_fwd<T>(c, Xt);
    pm.mark(c, HS_PH_FFT_FWD + 1);
    launch_degrid_dual_v<T>(c, v);
    pm.mark(c, HS_PH_DEGRID + 1);
    if (after_degrid) (void)hipEventRecord(after_degrid, c->stream);
    launch_bins_and_roots<T>(c);
    pm.mark(c, HS_PH_ROOTS + 1);
    launch_dual_apply_v<T>(c, v);
    pm.mark(c, HS_PH_DUAL_APPLY + 1);
    if (adj) {
        launch_grid_pull<T>(c, v, (const T*)c->d.vis_theta);
        pm.mark(c, HS_PH_GRID + 1);
        launch_fft_cols_adj<T>(c, c->L);
        launch_fft_rows_adj<T>(c, adj, c->L);
        pm.mark(c, HS_PH_FFT_ADJ + 1);
    }
}

// Eigen-decomposition of the Gram matrix of Z = P + Xt (Xt may be null), refined by a
// Rayleigh-Ritz step where the context asks for it (the refinement counts as eig time).
template <typename T>
static void nuclear_eig(hs_ctx* c, const T* P, const T* Xt, int mode, bool force64,
                        const PhaseMarks& pm = PhaseMarks()) {
    launch_gram<T>(c, P, Xt, force64);
    pm.mark(c, HS_PH_GRAM + 1);
    launch_eig(c, mode);
    if (eig_refined(c, force64)) launch_eig_refine<T>(c, P, Xt, mode);
    pm.mark(c, HS_PH_EIG + 1);
}

template <typename T>
static void dual_nuclear_impl(hs_ctx* c, T* P, const T* Xt, const PhaseMarks& pm = PhaseMarks()) {
    nuclear_eig<T>(c, P, Xt, 0, false, pm);
    launch_backproject<T>(c, P, P, Xt);
    pm.mark(c, HS_PH_BACKPROJ + 1);
}

// Prior terms the iteration carries.
static bool use_nuclear(const hs_ctx* c) { return c->prior == HS_PRIOR_LRJAS || c->prior == HS_PRIOR_LR; }
static bool use_sparsity(const hs_ctx* c) { return c->prior != HS_PRIOR_LR; }

template <typename T>
static void dual_l21_impl(hs_ctx* c, T* A, const T* Xt, const T* wbar, double mu, T* At_sum,
                          const PhaseMarks& pm = PhaseMarks()) {
    launch_psi_adj<T>(c, Xt, nullptr);
    pm.mark(c, HS_PH_PSI_ADJ + 1);
    launch_l21_dual<T>(c, A, Xt, (const T*)c->d.coef, wbar, mu * (double)c->D, c->prior == HS_PRIOR_SARA ? 2 : 0);
    pm.mark(c, HS_PH_L21 + 1);
    if (At_sum) launch_psi_sum<T>(c, A + (size_t)c->L * c->N, A, At_sum);
    pm.mark(c, HS_PH_PSI + 1);
}

// One iteration of Algorithm 2 as three independent branches (data fidelity,
// low rankness, joint sparsity) joined before the primal update; used for the
// captured graph so the branches overlap on the device.
// Where the side branches start: 0 at the iteration start, 1 after the forward
// FFT, 2 after the degridding pass.
constexpr int L21_START = 1, NUC_START = 1;
template <typename T>
static void pd_iter_forked(hs_ctx* c) {
    Dev& d = c->d;
    T* Xt = (T*)d.Xt;
    hipStream_t main = c->stream;
    const bool nuc = use_nuclear(c), sp = use_sparsity(c);
    auto branch_nuc = [&]() {
        c->stream = c->side[0];
        dual_nuclear_impl<T>(c, (T*)d.P, Xt);
        (void)hipEventRecord(c->ev_join[0], c->side[0]);
        c->stream = main;
    };
    auto branch_l21 = [&]() {
        c->stream = c->side[1];
        dual_l21_impl<T>(c, (T*)d.A, Xt, (const T*)d.wbar, c->mu, (T*)d.img1);
        (void)hipEventRecord(c->ev_join[1], c->side[1]);
        c->stream = main;
    };
    (void)hipEventRecord(c->ev_fork, main);
    if (nuc && NUC_START == 0) { (void)hipStreamWaitEvent(c->side[0], c->ev_fork, 0); branch_nuc(); }
    if (sp && L21_START == 0) { (void)hipStreamWaitEvent(c->side[1], c->ev_fork, 0); branch_l21(); }
    fft_fwd<T>(c, Xt);
    if ((nuc && NUC_START == 1) || (sp && L21_START == 1)) {
        (void)hipEventRecord(c->ev_mid, main);
        if (nuc && NUC_START == 1) { (void)hipStreamWaitEvent(c->side[0], c->ev_mid, 0); branch_nuc(); }
        if (sp && L21_START == 1) { (void)hipStreamWaitEvent(c->side[1], c->ev_mid, 0); branch_l21(); }
    }
    const bool late = (nuc && NUC_START == 2) || (sp && L21_START == 2);
    if (late) {
        // record after the degridding; the branches are forked below, after the
        // data branch's remaining launches are enqueued in capture order
        dual_data_impl<T>(c, (cplx<T>*)d.v, Xt, (T*)d.img0, PhaseMarks(), false, c->ev_mid);
        if (nuc && NUC_START == 2) { (void)hipStreamWaitEvent(c->side[0], c->ev_mid, 0); branch_nuc(); }
        if (sp && L21_START == 2) { (void)hipStreamWaitEvent(c->side[1], c->ev_mid, 0); branch_l21(); }
    } else {
        dual_data_impl<T>(c, (cplx<T>*)d.v, Xt, (T*)d.img0, PhaseMarks(), false);
    }
    if (nuc) (void)hipStreamWaitEvent(main, c->ev_join[0], 0);
    if (sp) (void)hipStreamWaitEvent(main, c->ev_join[1], 0);
    launch_primal<T>(c, sp ? (const T*)d.img1 : nullptr, (const T*)d.img0, nuc);
}

// One iteration of Algorithm 2 on the context state.
template <typename T>
static void pd_iter_impl(hs_ctx* c, const PhaseMarks& pm = PhaseMarks()) {
    Dev& d = c->d;
    T* Xt = (T*)d.Xt;
    pm.mark(c, 0);
    // data fidelity -> img0 = Re Phi^dag v
    dual_data_impl<T>(c, (cplx<T>*)d.v, Xt, (T*)d.img0, pm);
    // low rankness; a prior that is off still records its phase marks
    const bool nuc = use_nuclear(c), sp = use_sparsity(c);
    if (nuc) dual_nuclear_impl<T>(c, (T*)d.P, Xt, pm);
    else for (int k = HS_PH_GRAM; k <= HS_PH_BACKPROJ; ++k) pm.mark(c, k + 1);
    // joint average sparsity -> img1 = sum_d Psi_d A_d
    if (sp) dual_l21_impl<T>(c, (T*)d.A, Xt, (const T*)d.wbar, c->mu, (T*)d.img1, pm);
    else for (int k = HS_PH_PSI_ADJ; k <= HS_PH_PSI; ++k) pm.mark(c, k + 1);
    // primal update
    launch_primal<T>(c, sp ? (const T*)d.img1 : nullptr, (const T*)d.img0, nuc);
    pm.mark(c, HS_PH_PRIMAL + 1);
}

template <typename T>
static hs_status op_norm_impl(hs_ctx* c, int max_it, double tol, const T* x0, double* out, double* per, int* iters) {
    Dev& d = c->d;
    const int64_t LN = (int64_t)c->L * c->N;
    T* x = (T*)d.img1;
    if ((const void*)x != (const void*)x0) hipMemcpyAsync(x, x0, LN * sizeof(T), hipMemcpyDeviceToDevice, c->stream);
    launch_chan_norms<T>(c, x, d.chan_nrm);
    launch_chan_scale<T>(c, x, d.chan_nrm);
    std::vector<double> lam(c->L, 0.0), prev(c->L, 0.0);
    int it = 0;
    for (it = 1; it <= max_it; ++it) {
        if (c->per_channel) {
            for (int l = 0; l < c->L; ++l) {
                fft_fwd<T>(c, x, l);
                launch_degrid_grid_order<T>(c, (cplx<T>*)d.vwork, (const T*)d.vis_u, l);
                adj_from_grid_order<T>(c, (const cplx<T>*)d.vwork, (const T*)d.vis_theta, x, l);
            }
        } else {
            fft_fwd<T>(c, x);
            launch_degrid_grid_order<T>(c, (cplx<T>*)d.vwork, (const T*)d.vis_u);
            adj_from_grid_order<T>(c, (const cplx<T>*)d.vwork, (const T*)d.vis_theta, x);
        }
        launch_chan_norms<T>(c, x, d.chan_nrm);
        hs_status s = hip_check(c, hipMemcpyAsync(lam.data(), d.chan_nrm, c->L * 8, hipMemcpyDeviceToHost, c->stream),
                                "hs_op_norm");
        if (s) return s;
        s = hip_check(c, hipStreamSynchronize(c->stream), "hs_op_norm");
        if (s) return s;
        launch_chan_scale<T>(c, x, d.chan_nrm);
        bool done = true;
        for (int l = 0; l < c->L; ++l)
            if (!(lam[l] == 0.0 || std::fabs(lam[l] - prev[l]) <= tol * lam[l])) done = false;
        prev = lam;
        if (done) break;
    }
    if (it > max_it) it = max_it;
    double mx = 0.0;
    for (int l = 0; l < c->L; ++l) mx = std::max(mx, lam[l]);
    *out = mx;
    if (per) std::copy(lam.begin(), lam.end(), per);
    if (iters) *iters = it;
    return HS_OK;
}

// Dirty cube and trade-off estimate (Sec. 2.3, normalisation of Sec. 4.3):
// PSF_l = Re Phi_l^dag Phi_l delta (delta at the phase centre), X_l = Re Phi_l^dag y_l / max PSF_l,
// mu = ||X||_* / ||Psi^dag X||_{2,1}.
template <typename T>
static hs_status dirty_mu_impl(hs_ctx* c, T* Xd, double* mu) {
    Dev& d = c->d;
    const int64_t LN = (int64_t)c->L * c->N;
    T* delta = (T*)d.img1;
    T* psf = (T*)d.img0;
    T* X = Xd ? Xd : (T*)d.img0;
    launch_fill<T>(c->stream, delta, T(0), LN);
    launch_set_center<T>(c, delta);
    if (c->per_channel) {
        for (int l = 0; l < c->L; ++l) {
            fft_fwd<T>(c, delta, l);
            launch_degrid_grid_order<T>(c, (cplx<T>*)d.vwork, (const T*)nullptr, l);
        }
    } else {
        fft_fwd<T>(c, delta);
        launch_degrid_grid_order<T>(c, (cplx<T>*)d.vwork, (const T*)nullptr);
    }
    adj_from_grid_order<T>(c, (const cplx<T>*)d.vwork, (const T*)d.vis_theta, psf);
    launch_chan_max<T>(c, psf, d.chan_nrm);
    adj_from_grid_order<T>(c, (const cplx<T>*)d.vis_y, (const T*)d.vis_theta, X);
    launch_chan_scale<T>(c, X, d.chan_nrm);
    if (!mu) return HS_OK;
    // nuclear norm from the FP64 eigen-decomposition of the L x L Gram matrix
    nuclear_eig<T>(c, X, (const T*)nullptr, 0, true);
    std::vector<double> sg(MAX_L);
    hipMemcpyAsync(sg.data(), d.eig_sig, MAX_L * 8, hipMemcpyDeviceToHost, c->stream);
    launch_psi_adj<T>(c, X, nullptr);
    const int np = launch_l21_norm<T>(c, X, (const T*)d.coef);
    std::vector<double> part(np);
    hipMemcpyAsync(part.data(), d.red_part, np * 8, hipMemcpyDeviceToHost, c->stream);
    launch_eig_reset(c);   // the eigen-solver warm start belongs to the PD iteration
    hs_status s = hip_check(c, hipStreamSynchronize(c->stream), "hs_dirty_mu");
    if (s) return s;
    double nuc = 0.0, l21 = 0.0;
    for (int l = 0; l < c->L; ++l) nuc += sg[l];
    for (int k = 0; k < np; ++k) l21 += part[k];
    *mu = l21 > 0.0 ? nuc / l21 : 0.0;
    return HS_OK;
}

}  // namespace hs

using namespace hs;

#define HS_TRY_BEGIN try {
#define HS_TRY_END(c)                                                           \
    }                                                                           \
    catch (const std::exception& ex) {                                          \
        return fail(c, HS_ERR_INVALID_ARG, std::string("exception: ") + ex.what()); \
    }                                                                           \
    catch (...) {                                                               \
        return fail(c, HS_ERR_INVALID_ARG, "unknown exception");                \
    }

#define HS_DISPATCH(c, CALL)                          \
    do {                                              \
        if ((c)->dtype == HS_F32) { typedef float T; CALL; } \
        else { typedef double T; CALL; }              \
    } while (0)

static hs_status ready(hs_ctx* c) {
    if (!c) return HS_ERR_INVALID_ARG;
    if (!c->planned) return fail(c, HS_ERR_NOT_PLANNED, "call hs_plan first");
    if (!c->bound) return fail(c, HS_ERR_NO_WORKSPACE, "call hs_bind_workspace first");
    hipSetDevice(c->device);
    return HS_OK;
}

static hs_status launched(hs_ctx* c, const char* what) {
    return hip_check(c, hipGetLastError(), what);
}

extern "C" {

const char* hs_status_string(hs_status s) {
    switch (s) {
        case HS_OK: return "ok";
        case HS_ERR_INVALID_ARG: return "invalid argument";
        case HS_ERR_SHAPE: return "unsupported shape";
        case HS_ERR_DTYPE: return "unsupported dtype";
        case HS_ERR_NOT_PLANNED: return "not planned";
        case HS_ERR_NO_WORKSPACE: return "no workspace bound";
        case HS_ERR_NONFINITE: return "non-finite input";
        case HS_ERR_HIP: return "HIP runtime error";
        case HS_ERR_NOT_CONVERGED: return "not converged";
        default: return "unknown status";
    }
}

const char* hs_last_error(const hs_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

hs_status hs_create(const hs_problem_desc* desc, hs_ctx** out) {
    HS_TRY_BEGIN
    if (!desc || !out) return fail(nullptr, HS_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    const hs_problem_desc& d = *desc;
    if (d.dtype != HS_F32 && d.dtype != HS_F64) return fail(nullptr, HS_ERR_DTYPE, "dtype must be HS_F32 or HS_F64");
    if (d.gram_mode < HS_GRAM_F64 || d.gram_mode > HS_GRAM_BF16_SPLIT)
        return fail(nullptr, HS_ERR_INVALID_ARG, "gram_mode must be HS_GRAM_F64, HS_GRAM_F32 or HS_GRAM_BF16_SPLIT");
    if (d.dtype == HS_F64 && d.gram_mode != HS_GRAM_F64)
        return fail(nullptr, HS_ERR_DTYPE, "an FP64 context forms its Gram matrix in FP64 (HS_GRAM_F64)");
    if (d.oversamp != 2) return fail(nullptr, HS_ERR_INVALID_ARG, "oversamp must be 2");
    if (d.J != KB_J) return fail(nullptr, HS_ERR_INVALID_ARG, "J must be 8");
    if (d.L < 1 || d.L > MAX_L) return fail(nullptr, HS_ERR_SHAPE, "L must be in 1..64");
    if (d.levels < 1 || d.levels > 6 || d.n_db < 0 || d.n_db > MAX_DB)
        return fail(nullptr, HS_ERR_INVALID_ARG, "levels in 1..6 and n_db in 0..8");
    const int q = 1 << d.levels;
    // one FFT line of the 2x oversampled grid (<= 4096 points) lives in one workgroup's LDS
    if (d.nx < 16 || d.ny < 16 || d.nx % q || d.ny % q || d.nx > 2048 || d.ny > 2048 || (d.nx & (d.nx - 1)) ||
        (d.ny & (d.ny - 1)))
        return fail(nullptr, HS_ERR_SHAPE, "nx, ny must be powers of two in 16..2048 and multiples of 2^levels");
    int dev_count = 0;
    const hipError_t derr = hipGetDeviceCount(&dev_count);
    if (derr != hipSuccess || d.device < 0 || d.device >= dev_count)
        return fail(nullptr, HS_ERR_HIP, std::string("no such HIP device (hipGetDeviceCount: ") +
                                             hipGetErrorString(derr) + ", count " + std::to_string(dev_count) +
                                             ", device " + std::to_string(d.device) + ")");
    hs_ctx* c = new hs_ctx();
    c->desc = d;
    c->nx = d.nx;
    c->ny = d.ny;
    c->L = d.L;
    c->Kx = 2 * d.nx;
    c->Ky = 2 * d.ny;
    c->Kh = d.nx;
    c->N = (int64_t)d.nx * d.ny;
    c->n_db = d.n_db;
    c->D = 1 + d.n_db;
    c->levels = d.levels;
    c->dtype = d.dtype;
    c->gram_mode = d.gram_mode;
    c->per_channel = d.per_channel != 0;
    c->rsz = d.dtype == HS_F32 ? 4 : 8;
    c->stream = (hipStream_t)d.stream;
    c->device = d.device;
    c->ch.resize(d.L);
    c->w_host.assign(MAX_L, 1.0);
    c->k2 = 1.0 / c->D;
    *out = c;
    return HS_OK;
    HS_TRY_END(nullptr)
}

hs_status hs_destroy(hs_ctx* c) {
    if (!c) return HS_ERR_INVALID_ARG;
    // the context's work (graph replays, side streams) must be done before its graph,
    // streams and events go away
    if (c->gexec || c->side[0] || c->side[1]) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        for (int k = 0; k < 2; ++k)
            if (c->side[k]) (void)hipStreamSynchronize(c->side[k]);
    }
    if (c->gexec) hipGraphExecDestroy(c->gexec);
    if (c->graph) hipGraphDestroy(c->graph);
    for (int k = 0; k < 2; ++k) {
        if (c->side[k]) hipStreamDestroy(c->side[k]);
        if (c->ev_join[k]) hipEventDestroy(c->ev_join[k]);
    }
    if (c->ev_fork) hipEventDestroy(c->ev_fork);
    if (c->ev_mid) hipEventDestroy(c->ev_mid);
    delete c;
    return HS_OK;
}

hs_status hs_set_channel(hs_ctx* c, int32_t l, int64_t M, int32_t nblocks, const int64_t* bp, const double* uv,
                         const double* y_raw, const double* theta, const double* precond, const double* eps) {
    HS_TRY_BEGIN
    if (!c) return HS_ERR_INVALID_ARG;
    if (c->planned) return fail(c, HS_ERR_INVALID_ARG, "hs_set_channel after hs_plan (use hs_set_data)");
    if (l < 0 || l >= c->L) return fail(c, HS_ERR_INVALID_ARG, "channel index out of range");
    if (M < 0 || nblocks < 0 || (M > 0 && nblocks < 1) || !bp) return fail(c, HS_ERR_INVALID_ARG, "bad M / blocks");
    if (M > 0 && (!uv || !y_raw || !theta)) return fail(c, HS_ERR_INVALID_ARG, "null data pointer");
    if (nblocks > 0 && !eps) return fail(c, HS_ERR_INVALID_ARG, "null eps");
    if (nblocks > 0 && (bp[0] != 0 || bp[nblocks] != M)) return fail(c, HS_ERR_INVALID_ARG, "block_ptr must span 0..M");
    for (int b = 0; b < nblocks; ++b)
        if (bp[b + 1] < bp[b]) return fail(c, HS_ERR_INVALID_ARG, "block_ptr not monotone");
    for (int64_t m = 0; m < 2 * M; ++m)
        if (!std::isfinite(uv[m]) || !std::isfinite(y_raw[m])) return fail(c, HS_ERR_NONFINITE, "non-finite uv or y");
    for (int64_t m = 0; m < M; ++m) {
        if (!std::isfinite(theta[m]) || !(theta[m] > 0)) return fail(c, HS_ERR_NONFINITE, "theta must be finite and > 0");
        if (precond && (!std::isfinite(precond[m]) || !(precond[m] > 0)))
            return fail(c, HS_ERR_NONFINITE, "preconditioner must be finite and > 0");
        const double tx = std::fabs(uv[2 * m]) * c->Kx, ty = std::fabs(uv[2 * m + 1]) * c->Ky;
        if (tx > 1e9 || ty > 1e9) return fail(c, HS_ERR_INVALID_ARG, "|u| too large");
    }
    for (int b = 0; b < nblocks; ++b)
        if (!std::isfinite(eps[b]) || eps[b] < 0) return fail(c, HS_ERR_NONFINITE, "eps must be finite and >= 0");
    Channel& ch = c->ch[l];
    ch.M = M;
    ch.nb = nblocks;
    ch.bp.assign(bp, bp + nblocks + 1);
    ch.uv.assign(uv, uv + 2 * M);
    ch.y.assign(y_raw, y_raw + 2 * M);
    ch.theta.assign(theta, theta + M);
    ch.has_u = precond != nullptr;
    if (precond) ch.u.assign(precond, precond + M);
    else ch.u.clear();
    ch.eps.assign(eps, eps + nblocks);
    ch.set = true;
    return HS_OK;
    HS_TRY_END(c)
}

hs_status hs_set_data(hs_ctx* c, int32_t l, const double* y_raw, const double* theta, const double* eps) {
    HS_TRY_BEGIN
    hs_status s = ready(c);
    if (s) return s;
    if (l < 0 || l >= c->L) return fail(c, HS_ERR_INVALID_ARG, "channel index out of range");
    Channel& ch = c->ch[l];
    for (int64_t m = 0; m < ch.M; ++m) {
        if (!std::isfinite(y_raw[2 * m]) || !std::isfinite(y_raw[2 * m + 1])) return fail(c, HS_ERR_NONFINITE, "y");
        if (!std::isfinite(theta[m]) || !(theta[m] > 0)) return fail(c, HS_ERR_NONFINITE, "theta");
    }
    for (int b = 0; b < ch.nb; ++b)
        if (!std::isfinite(eps[b]) || eps[b] < 0) return fail(c, HS_ERR_NONFINITE, "eps");
    ch.y.assign(y_raw, y_raw + 2 * ch.M);
    ch.theta.assign(theta, theta + ch.M);
    ch.eps.assign(eps, eps + ch.nb);
    const int64_t base = c->chan_off[l];
    for (int64_t k = 0; k < ch.M; ++k) {
        const int64_t g = base + k;
        const int64_t m = c->h_perm[g] - base;
        c->h_theta[g] = ch.theta[m];
        c->h_y[2 * g] = ch.theta[m] * ch.y[2 * m];
        c->h_y[2 * g + 1] = ch.theta[m] * ch.y[2 * m + 1];
    }
    for (int b = 0; b < ch.nb; ++b) c->h_blk_eps[c->blk_off[l] + b] = ch.eps[b];
    hipStreamSynchronize(c->stream);
    const size_t n = (size_t)ch.M;
    if (c->dtype == HS_F32) {
        std::vector<float> th(c->h_theta.begin() + base, c->h_theta.begin() + base + n);
        std::vector<float> yy(c->h_y.begin() + 2 * base, c->h_y.begin() + 2 * (base + n));
        hipMemcpy((float*)c->d.vis_theta + base, th.data(), n * 4, hipMemcpyHostToDevice);
        hipMemcpy((float*)c->d.vis_y + 2 * base, yy.data(), 2 * n * 4, hipMemcpyHostToDevice);
        hipMemcpy((double*)c->d64.vis_theta + base, c->h_theta.data() + base, n * 8, hipMemcpyHostToDevice);
    } else {
        hipMemcpy((double*)c->d.vis_theta + base, c->h_theta.data() + base, n * 8, hipMemcpyHostToDevice);
        hipMemcpy((double*)c->d.vis_y + 2 * base, c->h_y.data() + 2 * base, 2 * n * 8, hipMemcpyHostToDevice);
    }
    hipMemcpy(c->d.blk_eps + c->blk_off[l], ch.eps.data(), ch.nb * 8, hipMemcpyHostToDevice);
    return launched(c, "hs_set_data");
    HS_TRY_END(c)
}

hs_status hs_plan(hs_ctx* c, size_t* ws) {
    HS_TRY_BEGIN
    if (!c || !ws) return HS_ERR_INVALID_ARG;
    if (c->planned) {
        *ws = c->ws_bytes;
        return HS_OK;
    }
    hs_status s = build_plan(c);
    if (s) return s;
    c->ws_bytes = carve(c, nullptr);
    c->planned = true;
    *ws = c->ws_bytes;
    return HS_OK;
    HS_TRY_END(c)
}

hs_status hs_bind_workspace(hs_ctx* c, void* dev, size_t bytes) {
    HS_TRY_BEGIN
    if (!c || !dev) return HS_ERR_INVALID_ARG;
    if (!c->planned) return fail(c, HS_ERR_NOT_PLANNED, "call hs_plan first");
    if (bytes < c->ws_bytes) return fail(c, HS_ERR_NO_WORKSPACE, "workspace too small");
    if (((uintptr_t)dev) & 255) return fail(c, HS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    hs_status s = hip_check(c, hipSetDevice(c->device), "hipSetDevice");
    if (s) return s;
    fft_init_attrs();
    c->ws = dev;
    carve(c, (char*)dev);
    if (c->dtype == HS_F32) s = bind_impl<float>(c);
    else s = bind_impl<double>(c);
    if (s) return s;
    c->bound = true;
    c->graph_valid = false;
    return HS_OK;
    HS_TRY_END(c)
}

hs_status hs_get_info(const hs_ctx* c, hs_info* info) {
    if (!c || !info) return HS_ERR_INVALID_ARG;
    info->n_vis = c->Mtot;
    info->n_blocks = c->nblk;
    info->n_bins = c->nbins;
    info->n_runs = c->nruns;
    info->n_degrid_units = (int64_t)c->dunits.size();
    info->n_grid_units = (int64_t)c->gunits.size();
    info->tile = c->T;
    info->kb_terms = c->kb_terms;
    info->workspace_bytes = c->ws_bytes;
    return HS_OK;
}

hs_status hs_phi(hs_ctx* c, const void* X, void* Y) {
    hs_status s = ready(c);
    if (s) return s;
    if (!X || !Y) return fail(c, HS_ERR_INVALID_ARG, "null pointer");
    HS_DISPATCH(c, phi_impl<T>(c, (const T*)X, (cplx<T>*)Y));
    return launched(c, "hs_phi");
}

hs_status hs_phi_adj(hs_ctx* c, const void* Y, void* X) {
    hs_status s = ready(c);
    if (s) return s;
    if (!X || !Y) return fail(c, HS_ERR_INVALID_ARG, "null pointer");
    HS_DISPATCH(c, phi_adj_impl<T>(c, (const cplx<T>*)Y, (T*)X));
    return launched(c, "hs_phi_adj");
}

hs_status hs_psi_adj_n(hs_ctx* c, const void* X, void* C, int32_t nl) {
    hs_status s = ready(c);
    if (s) return s;
    if (!X || !C) return fail(c, HS_ERR_INVALID_ARG, "null pointer");
    if (nl < 1 || nl > c->L) return fail(c, HS_ERR_INVALID_ARG, "channel count must be in 1..L");
    const size_t LN = (size_t)nl * c->N;
    hipMemcpyAsync(C, X, LN * c->rsz, hipMemcpyDeviceToDevice, c->stream);
    HS_DISPATCH(c, launch_psi_adj<T>(c, (const T*)X, (T*)C + LN, nl));
    return launched(c, "hs_psi_adj");
}

hs_status hs_psi_adj(hs_ctx* c, const void* X, void* C) { return hs_psi_adj_n(c, X, C, c ? c->L : 0); }

hs_status hs_psi_n(hs_ctx* c, const void* C, void* X, int32_t nl) {
    hs_status s = ready(c);
    if (s) return s;
    if (!X || !C) return fail(c, HS_ERR_INVALID_ARG, "null pointer");
    if (nl < 1 || nl > c->L) return fail(c, HS_ERR_INVALID_ARG, "channel count must be in 1..L");
    const size_t LN = (size_t)nl * c->N;
    HS_DISPATCH(c, launch_psi_sum<T>(c, (const T*)C + LN, (const T*)C, (T*)X, nl));
    return launched(c, "hs_psi");
}

hs_status hs_psi(hs_ctx* c, const void* C, void* X) { return hs_psi_n(c, C, X, c ? c->L : 0); }

hs_status hs_l21_rowsq(hs_ctx* c, const void* C, int32_t nl, double* S, int32_t accumulate) {
    hs_status s = ready(c);
    if (s) return s;
    if (!C || !S) return fail(c, HS_ERR_INVALID_ARG, "null pointer");
    if (nl < 1 || nl > c->L) return fail(c, HS_ERR_INVALID_ARG, "channel count must be in 1..L");
    const size_t LN = (size_t)nl * c->N;
    HS_DISPATCH(c, launch_l21_rowsq<T>(c, (const T*)C, (const T*)C + LN, nl, S, accumulate != 0));
    return launched(c, "hs_l21_rowsq");
}

hs_status hs_l21_rowscale(hs_ctx* c, void* C, int32_t nl, const double* S, const void* wbar, double scale) {
    hs_status s = ready(c);
    if (s) return s;
    if (!C || !S || !std::isfinite(scale)) return fail(c, HS_ERR_INVALID_ARG, "bad argument");
    if (nl < 1 || nl > c->L) return fail(c, HS_ERR_INVALID_ARG, "channel count must be in 1..L");
    const size_t LN = (size_t)nl * c->N;
    HS_DISPATCH(c, launch_l21_rowscale<T>(c, (T*)C, (T*)C + LN, nl, S, (const T*)wbar, scale));
    return launched(c, "hs_l21_rowscale");
}

hs_status hs_l21_from_rowsq(hs_ctx* c, const double* S, const void* wbar, double* value) {
    hs_status s = ready(c);
    if (s) return s;
    if (!S || !value) return fail(c, HS_ERR_INVALID_ARG, "null pointer");
    int np = 0;
    HS_DISPATCH(c, np = launch_l21_from_rowsq<T>(c, S, (const T*)wbar));
    std::vector<double> part(np);
    hipMemcpyAsync(part.data(), c->d.red_part, (size_t)np * 8, hipMemcpyDeviceToHost, c->stream);
    s = hip_check(c, hipStreamSynchronize(c->stream), "hs_l21_from_rowsq");
    if (s) return s;
    double v = 0.0;
    for (int k = 0; k < np; ++k) v += part[k];
    *value = v;
    return HS_OK;
}

hs_status hs_prox_l21(hs_ctx* c, void* A, const void* wbar, double t) {
    hs_status s = ready(c);
    if (s) return s;
    if (!A || !(t >= 0)) return fail(c, HS_ERR_INVALID_ARG, "bad argument");
    HS_DISPATCH(c, launch_l21_dual<T>(c, (T*)A, nullptr, nullptr, (const T*)wbar, t, 1));
    return launched(c, "hs_prox_l21");
}

hs_status hs_dual_l21(hs_ctx* c, void* A, const void* Xt, const void* wbar, double mu, void* At_sum) {
    hs_status s = ready(c);
    if (s) return s;
    if (!A || !Xt || !(mu >= 0)) return fail(c, HS_ERR_INVALID_ARG, "bad argument");
    HS_DISPATCH(c, dual_l21_impl<T>(c, (T*)A, (const T*)Xt, (const T*)wbar, mu, (T*)At_sum));
    return launched(c, "hs_dual_l21");
}

static hs_status upload_w(hs_ctx* c, const double* w) {
    std::vector<double> wv(MAX_L, 1.0);
    if (w)
        for (int l = 0; l < c->L; ++l) {
            if (!std::isfinite(w[l]) || w[l] < 0) return fail(c, HS_ERR_NONFINITE, "nuclear weights must be >= 0");
            wv[l] = w[l];
        }
    c->w_host = wv;
    hs_status s = hip_check(c, hipStreamSynchronize(c->stream), "upload w");
    if (s) return s;
    return hip_check(c, hipMemcpy(c->d.w_nuc, c->w_host.data(), MAX_L * 8, hipMemcpyHostToDevice), "upload w");
}

hs_status hs_prox_nuclear(hs_ctx* c, void* X, const double* w, double* sigma_out) {
    hs_status s = ready(c);
    if (s) return s;
    if (!X) return fail(c, HS_ERR_INVALID_ARG, "null pointer");
    std::vector<double> saved = c->w_host;
    s = upload_w(c, w);
    if (s) return s;
    HS_DISPATCH(c, { nuclear_eig<T>(c, (const T*)X, (const T*)nullptr, 1, false);
                     launch_backproject<T>(c, (T*)X, (const T*)X, nullptr); });
    s = launched(c, "hs_prox_nuclear");
    if (s) return s;
    std::vector<double> sg(MAX_L);
    s = hip_check(c, hipMemcpyAsync(sg.data(), c->d.eig_sig, MAX_L * 8, hipMemcpyDeviceToHost, c->stream), "sigma");
    if (s) return s;
    s = hip_check(c, hipStreamSynchronize(c->stream), "hs_prox_nuclear");
    if (s) return s;
    if (sigma_out) std::copy(sg.begin(), sg.begin() + c->L, sigma_out);
    return upload_w(c, saved.data());
}

hs_status hs_dual_nuclear(hs_ctx* c, void* P, const void* Xt, const double* w) {
    hs_status s = ready(c);
    if (s) return s;
    if (!P || !Xt) return fail(c, HS_ERR_INVALID_ARG, "null pointer");
    std::vector<double> saved = c->w_host;
    s = upload_w(c, w);
    if (s) return s;
    HS_DISPATCH(c, dual_nuclear_impl<T>(c, (T*)P, (const T*)Xt));
    s = launched(c, "hs_dual_nuclear");
    if (s) return s;
    return upload_w(c, saved.data());
}

hs_status hs_dual_data(hs_ctx* c, void* v, const void* Xt, void* adj_out) {
    hs_status s = ready(c);
    if (s) return s;
    if (!v || !Xt) return fail(c, HS_ERR_INVALID_ARG, "null pointer");
    HS_DISPATCH(c, {
        cplx<T>* vw = (cplx<T>*)c->d.vwork;
        launch_gather_user<T>(c, (const cplx<T>*)v, vw, false);
        dual_data_impl<T>(c, vw, (const T*)Xt, (T*)adj_out);
        launch_scatter_user<T>(c, vw, (cplx<T>*)v);
    });
    return launched(c, "hs_dual_data");
}

hs_status hs_proj_ellipsoid(hs_ctx* c, int32_t l, int32_t b, void* z) {
    hs_status s = ready(c);
    if (s) return s;
    if (!z || l < 0 || l >= c->L || b < 0 || b >= c->ch[l].nb) return fail(c, HS_ERR_INVALID_ARG, "bad block");
    const int64_t pos0 = c->chan_off[l] + c->ch[l].bp[b];
    const int64_t Mb = c->ch[l].bp[b + 1] - c->ch[l].bp[b];
    if (Mb == 0) return HS_OK;
    HS_DISPATCH(c, launch_proj_block<T>(c, pos0, Mb, c->blk_off[l] + b, (cplx<T>*)z));
    s = launched(c, "hs_proj_ellipsoid");
    if (s) return s;
    return hip_check(c, hipStreamSynchronize(c->stream), "hs_proj_ellipsoid");
}

hs_status hs_op_norm(hs_ctx* c, int32_t which, int32_t max_it, double tol, const void* x0, double* out,
                     double* per_channel, int32_t* iters) {
    hs_status s = ready(c);
    if (s) return s;
    if (!out) return fail(c, HS_ERR_INVALID_ARG, "null out");
    if (which == HS_NORM_PSI) {
        *out = (double)c->D;
        if (iters) *iters = 0;
        return HS_OK;
    }
    if (which != HS_NORM_PHI_PRECOND || !x0 || max_it < 1 || !(tol >= 0))
        return fail(c, HS_ERR_INVALID_ARG, "bad op_norm arguments");
    c->graph_valid = false;  // scratch buffers are reused
    if (c->dtype == HS_F32) {
        // the FP64 operators on the FP64 copies of the plan's arrays (Sec. 3.4: the
        // step-size norm stays in FP64); the caller's FP32 start is widened exactly
        const Dev saved = c->d;
        const std::vector<double> kb_saved = c->kb_c;
        Dev& d = c->d;
        const Dev64& e = c->d64;
        d.vis_frac = e.vis_frac; d.vis_theta = e.vis_theta; d.vis_u = e.vis_u; d.vwork = e.vwork;
        d.gpartial = e.gpartial; d.grid = e.grid; d.H = e.H; d.tw_x = e.tw_x; d.tw_y = e.tw_y;
        d.sx = e.sx; d.sy = e.sy; d.img1 = e.x;
        c->kb_c = c->kb_c64;
        launch_convert<float, double>(c->stream, (double*)e.x, (const float*)x0, (int64_t)c->L * c->N);
        s = op_norm_impl<double>(c, max_it, tol, (const double*)e.x, out, per_channel, iters);
        c->d = saved;
        c->kb_c = kb_saved;
    } else {
        s = op_norm_impl<double>(c, max_it, tol, (const double*)x0, out, per_channel, iters);
    }
    if (s) return s;
    return launched(c, "hs_op_norm");
}

hs_status hs_dirty_mu(hs_ctx* c, void* Xd, double* mu) {
    hs_status s = ready(c);
    if (s) return s;
    if (!Xd && !mu) return fail(c, HS_ERR_INVALID_ARG, "nothing requested");
    HS_DISPATCH(c, s = dirty_mu_impl<T>(c, (T*)Xd, mu));
    if (s) return s;
    return launched(c, "hs_dirty_mu");
}

hs_status hs_pd_init(hs_ctx* c, const hs_pd_params* p) {
    hs_status s = ready(c);
    if (s) return s;
    if (!p) return fail(c, HS_ERR_INVALID_ARG, "null params");
    if (!(p->mu >= 0) || !(p->tau > 0) || !(p->kappa3 > 0))
        return fail(c, HS_ERR_INVALID_ARG, "need mu >= 0, tau > 0, kappa3 > 0");
    c->mu = p->mu;
    c->tau = p->tau;
    c->k1 = p->kappa1 > 0 ? p->kappa1 : 1.0;
    c->k2 = p->kappa2 > 0 ? p->kappa2 : 1.0 / c->D;
    c->k3 = p->kappa3;
    c->adaptive = p->adaptive_eps != 0;
    c->lam1 = p->lam1 > 0 ? p->lam1 : 5e-4;
    c->lam2 = p->lam2 > 0 ? p->lam2 : 0.01;
    c->lam3 = p->lam3 > 0 ? p->lam3 : 0.618;
    c->vartheta_bar = p->vartheta_bar > 0 ? p->vartheta_bar : 100;
    if (p->prior < HS_PRIOR_LRJAS || p->prior > HS_PRIOR_SARA) return fail(c, HS_ERR_INVALID_ARG, "unknown prior");
    c->prior = p->prior;
    s = upload_w(c, p->w);
    if (s) return s;
    if (p->wbar) hipMemcpyAsync(c->d.wbar, p->wbar, (size_t)wbar_elems(c) * c->rsz, hipMemcpyDeviceToDevice, c->stream);
    else HS_DISPATCH(c, launch_fill<T>(c->stream, (T*)c->d.wbar, T(1), (int64_t)c->D * c->L * c->N));
    c->pd_ready = true;
    c->graph_valid = false;
    return launched(c, "hs_pd_init");
}

hs_status hs_pd_set_state(hs_ctx* c, const hs_state_ptrs* st) {
    hs_status s = ready(c);
    if (s) return s;
    if (!st) return fail(c, HS_ERR_INVALID_ARG, "null state");
    if ((st->wbar || st->w) && !c->pd_ready) return fail(c, HS_ERR_INVALID_ARG, "weights need hs_pd_init first");
    if (st->eps)
        for (int64_t b = 0; b < c->nblk; ++b)
            if (!std::isfinite(st->eps[b]) || st->eps[b] < 0) return fail(c, HS_ERR_NONFINITE, "eps must be >= 0");
    if (st->scalars && !(std::isfinite(st->scalars[0]) && st->scalars[1] >= 0))
        return fail(c, HS_ERR_INVALID_ARG, "scalars: beta finite and t >= 0");
    const size_t LN = (size_t)c->L * c->N * c->rsz;
    if (st->X) hipMemcpyAsync(c->d.X, st->X, LN, hipMemcpyDeviceToDevice, c->stream);
    if (st->Xt) hipMemcpyAsync(c->d.Xt, st->Xt, LN, hipMemcpyDeviceToDevice, c->stream);
    if (st->P) hipMemcpyAsync(c->d.P, st->P, LN, hipMemcpyDeviceToDevice, c->stream);
    if (st->A) hipMemcpyAsync(c->d.A, st->A, LN * c->D, hipMemcpyDeviceToDevice, c->stream);
    if (st->v) HS_DISPATCH(c, launch_gather_user<T>(c, (const cplx<T>*)st->v, (cplx<T>*)c->d.v, false));
    if (st->wbar) hipMemcpyAsync(c->d.wbar, st->wbar, (size_t)wbar_elems(c) * c->rsz, hipMemcpyDeviceToDevice, c->stream);
    launch_eig_reset(c);   // a new state starts the eigen-solver history afresh (reproducible runs)
    restart_counters(c, !st->scalars, !st->vartheta, !st->eps);
    s = hip_check(c, hipStreamSynchronize(c->stream), "hs_pd_set_state");
    if (s) return s;
    if (st->eps && c->nblk)
        s = hip_check(c, hipMemcpy(c->d.blk_eps, st->eps, (size_t)c->nblk * 8, hipMemcpyHostToDevice), "eps");
    if (!s && st->vartheta && c->nblk)
        s = hip_check(c, hipMemcpy(c->d.blk_vartheta, st->vartheta, (size_t)c->nblk * 4, hipMemcpyHostToDevice),
                      "vartheta");
    if (!s && st->scalars) {
        s = hip_check(c, hipMemcpy(c->d.scal, st->scalars, 2 * 8, hipMemcpyHostToDevice), "scalars");
        c->t_iter = (int64_t)st->scalars[1];
    }
    if (s) return s;
    if (st->w) {
        s = upload_w(c, st->w);
        if (s) return s;
    }
    return launched(c, "hs_pd_set_state");
}

hs_status hs_pd_get_state(hs_ctx* c, const hs_state_ptrs* st) {
    hs_status s = ready(c);
    if (s) return s;
    if (!st) return fail(c, HS_ERR_INVALID_ARG, "null state");
    const size_t LN = (size_t)c->L * c->N * c->rsz;
    if (st->X) hipMemcpyAsync(st->X, c->d.X, LN, hipMemcpyDeviceToDevice, c->stream);
    if (st->Xt) hipMemcpyAsync(st->Xt, c->d.Xt, LN, hipMemcpyDeviceToDevice, c->stream);
    if (st->P) hipMemcpyAsync(st->P, c->d.P, LN, hipMemcpyDeviceToDevice, c->stream);
    if (st->A) hipMemcpyAsync(st->A, c->d.A, LN * c->D, hipMemcpyDeviceToDevice, c->stream);
    if (st->v) HS_DISPATCH(c, launch_scatter_user<T>(c, (const cplx<T>*)c->d.v, (cplx<T>*)st->v));
    if (st->wbar) hipMemcpyAsync(st->wbar, c->d.wbar, (size_t)wbar_elems(c) * c->rsz, hipMemcpyDeviceToDevice, c->stream);
    if (st->eps || st->vartheta || st->scalars) {
        s = hip_check(c, hipStreamSynchronize(c->stream), "hs_pd_get_state");
        if (!s && st->eps && c->nblk)
            s = hip_check(c, hipMemcpy(st->eps, c->d.blk_eps, (size_t)c->nblk * 8, hipMemcpyDeviceToHost), "eps");
        if (!s && st->vartheta && c->nblk)
            s = hip_check(c, hipMemcpy(st->vartheta, c->d.blk_vartheta, (size_t)c->nblk * 4, hipMemcpyDeviceToHost),
                          "vartheta");
        if (!s && st->scalars) s = hip_check(c, hipMemcpy(st->scalars, c->d.scal, 2 * 8, hipMemcpyDeviceToHost), "scalars");
        if (s) return s;
    }
    if (st->w) std::copy(c->w_host.begin(), c->w_host.begin() + c->L, st->w);
    return launched(c, "hs_pd_get_state");
}

static hs_status pd_capture(hs_ctx* c) {
    if (c->gexec) {
        // replays of the old graph may still be in flight on the stream
        hs_status s0 = hip_check(c, hipStreamSynchronize(c->stream), "before re-capture");
        if (s0) return s0;
        hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    if (c->graph) { hipGraphDestroy(c->graph); c->graph = nullptr; }
    hs_status s = HS_OK;
    for (int k = 0; k < 2 && !s; ++k) {
        if (!c->side[k]) s = hip_check(c, hipStreamCreateWithFlags(&c->side[k], hipStreamNonBlocking), "side stream");
        if (!s && !c->ev_join[k])
            s = hip_check(c, hipEventCreateWithFlags(&c->ev_join[k], hipEventDisableTiming), "join event");
    }
    if (!s && !c->ev_fork) s = hip_check(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming), "fork event");
    if (!s && !c->ev_mid) s = hip_check(c, hipEventCreateWithFlags(&c->ev_mid, hipEventDisableTiming), "mid event");
    if (s) return s;
    s = hip_check(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed), "begin capture");
    if (s) return s;
    HS_DISPATCH(c, pd_iter_forked<T>(c));
    hipError_t le = hipGetLastError();
    s = hip_check(c, hipStreamEndCapture(c->stream, &c->graph), "end capture");
    if (s) return s;
    if (le != hipSuccess) return hip_check(c, le, "launch during capture");
    s = hip_check(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0), "graph instantiate");
    if (s) return s;
    c->graph_valid = true;
    return HS_OK;
}

hs_status hs_pd_iterate(hs_ctx* c, int32_t n) {
    hs_status s = ready(c);
    if (s) return s;
    if (!c->pd_ready) return fail(c, HS_ERR_INVALID_ARG, "call hs_pd_init first");
    if (n < 0) return fail(c, HS_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return HS_OK;
    if (c->stream == nullptr || c->per_channel) {
        // the legacy default stream cannot be captured, and the plain execution is eager
        for (int i = 0; i < n; ++i) HS_DISPATCH(c, pd_iter_impl<T>(c));
        c->t_iter += n;
        return launched(c, "hs_pd_iterate");
    }
    if (!c->graph_valid) {
        s = pd_capture(c);
        if (s) return s;
    }
    for (int i = 0; i < n; ++i) {
        s = hip_check(c, hipGraphLaunch(c->gexec, c->stream), "hipGraphLaunch");
        if (s) return s;
    }
    c->t_iter += n;
    return HS_OK;
}

hs_status hs_profile_phases(hs_ctx* c, int32_t n, double* times_ms) {
    hs_status s = ready(c);
    if (s) return s;
    if (!c->pd_ready) return fail(c, HS_ERR_INVALID_ARG, "call hs_pd_init first");
    if (n < 1 || !times_ms) return fail(c, HS_ERR_INVALID_ARG, "bad profile arguments");
    hipEvent_t ev[HS_NPHASES + 1];
    for (int k = 0; k <= HS_NPHASES; ++k)
        if ((s = hip_check(c, hipEventCreate(&ev[k]), "hipEventCreate"))) return s;
    std::vector<double> acc(HS_NPHASES, 0.0);
    PhaseMarks pm;
    pm.ev = ev;
    for (int it = 0; it < n && !s; ++it) {
        HS_DISPATCH(c, pd_iter_impl<T>(c, pm));
        s = hip_check(c, hipStreamSynchronize(c->stream), "hs_profile_phases");
        for (int k = 0; k < HS_NPHASES && !s; ++k) {
            float ms = 0.f;
            s = hip_check(c, hipEventElapsedTime(&ms, ev[k], ev[k + 1]), "hipEventElapsedTime");
            acc[k] += ms;
        }
    }
    for (int k = 0; k <= HS_NPHASES; ++k) (void)hipEventDestroy(ev[k]);
    if (s) return s;
    c->t_iter += n;
    for (int k = 0; k < HS_NPHASES; ++k) times_ms[k] = acc[k] / n;
    return HS_OK;
}

hs_status hs_pd_stats(hs_ctx* c, double* beta, double* rho, double* eps) {
    hs_status s = ready(c);
    if (s) return s;
    double sc[4];
    s = hip_check(c, hipMemcpyAsync(sc, c->d.scal, sizeof(sc), hipMemcpyDeviceToHost, c->stream), "stats");
    if (s) return s;
    std::vector<double> r2(c->nblk), ep(c->nblk);
    if (c->nblk) {
        hipMemcpyAsync(r2.data(), c->d.blk_rho2, c->nblk * 8, hipMemcpyDeviceToHost, c->stream);
        hipMemcpyAsync(ep.data(), c->d.blk_eps, c->nblk * 8, hipMemcpyDeviceToHost, c->stream);
    }
    s = hip_check(c, hipStreamSynchronize(c->stream), "hs_pd_stats");
    if (s) return s;
    if (beta) *beta = sc[0];
    if (rho)
        for (int64_t b = 0; b < c->nblk; ++b) rho[b] = std::sqrt(r2[b]);
    if (eps) std::copy(ep.begin(), ep.end(), eps);
    return HS_OK;
}

hs_status hs_get_diag(hs_ctx* c, double* out, int32_t n) {
    hs_status s = ready(c);
    if (s) return s;
    if (!out || n < 1) return fail(c, HS_ERR_INVALID_ARG, "bad diag arguments");
    double sc[16];
    s = hip_check(c, hipMemcpyAsync(sc, c->d.scal, sizeof(sc), hipMemcpyDeviceToHost, c->stream), "diag");
    if (s) return s;
    s = hip_check(c, hipStreamSynchronize(c->stream), "hs_get_diag");
    if (s) return s;
    const double vals[4] = {sc[0], sc[1], sc[8], (double)c->t_iter};
    for (int k = 0; k < n && k < 4; ++k) out[k] = vals[k];
    return HS_OK;
}

// Algorithm 1's weight update from the current estimate: eq:weights-l21 and eq:weights-n
// (SARA: the per-channel reweighted l1).
static hs_status solve_reweight(hs_ctx* c, double gamma, double gamma_bar) {
    const bool sara = c->prior == HS_PRIOR_SARA;
    HS_DISPATCH(c, {
        launch_psi_adj<T>(c, (const T*)c->d.X, nullptr);
        if (sara) {
            launch_reweight_l1<T>(c, (const T*)c->d.X, (const T*)c->d.coef, (T*)c->d.wbar, gamma_bar);
        } else {
            launch_reweight_l21<T>(c, (const T*)c->d.X, (const T*)c->d.coef, (T*)c->d.wbar, gamma_bar);
            nuclear_eig<T>(c, (const T*)c->d.X, (const T*)nullptr, 0, true);
        }
    });
    hs_status s = launched(c, "hs_solve reweight");
    if (s || sara) return s;
    std::vector<double> sg(MAX_L);
    hipMemcpyAsync(sg.data(), c->d.eig_sig, MAX_L * 8, hipMemcpyDeviceToHost, c->stream);
    s = hip_check(c, hipStreamSynchronize(c->stream), "hs_solve");
    if (s) return s;
    std::vector<double> w(c->L);
    for (int l = 0; l < c->L; ++l) w[l] = gamma / (gamma + sg[l]);
    return upload_w(c, w.data());
}

hs_status hs_solve(hs_ctx* c, const hs_solve_params* p, void* X_out, hs_report* rep) {
    hs_status s = ready(c);
    if (s) return s;
    if (!p || p->iters_per_reweight < 1 || p->n_reweights < 0 || !(p->gamma_factor > 0))
        return fail(c, HS_ERR_INVALID_ARG, "bad solve parameters");
    if (!c->pd_ready) return fail(c, HS_ERR_INVALID_ARG, "call hs_pd_init first");
    double gamma = p->gamma0 > 0 ? p->gamma0 : 1.0, gamma_bar = p->gamma_bar0 > 0 ? p->gamma_bar0 : 1.0, beta = 0.0;
    int64_t total = 0;
    int nrw = 0;
    const int check = p->check_every > 0 ? p->check_every : p->iters_per_reweight;
    if (p->reweight_first) {
        s = solve_reweight(c, gamma, gamma_bar);
        if (s) return s;
        gamma *= p->gamma_factor;
        gamma_bar *= p->gamma_factor;
        ++nrw;
    }
    for (int k = 0; k <= p->n_reweights; ++k) {
        int done = 0;
        while (done < p->iters_per_reweight) {
            const int n = std::min(check, p->iters_per_reweight - done);
            s = hs_pd_iterate(c, n);
            if (s) return s;
            done += n;
            total += n;
            s = hs_pd_stats(c, &beta, nullptr, nullptr);
            if (s) return s;
            if (p->beta_tol > 0 && beta < p->beta_tol) break;
        }
        if (k == p->n_reweights) break;
        s = solve_reweight(c, gamma, gamma_bar);
        if (s) return s;
        gamma *= p->gamma_factor;
        gamma_bar *= p->gamma_factor;
        ++nrw;
    }
    if (X_out) hipMemcpyAsync(X_out, c->d.X, (size_t)c->L * c->N * c->rsz, hipMemcpyDeviceToDevice, c->stream);
    s = hip_check(c, hipStreamSynchronize(c->stream), "hs_solve");
    if (s) return s;
    if (rep) {
        rep->iterations = total;
        rep->reweights = nrw;
        rep->final_beta = beta;
        rep->gamma = gamma;
        rep->gamma_bar = gamma_bar;
    }
    return HS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ tuning
namespace hs {

// A candidate replaces the best one only when it is faster by more than the
// run-to-run spread of the timing.
constexpr double TUNE_MARGIN = 0.98;

static hs_tuning tuning_of(const hs_ctx* c) {
    hs_tuning t{};
    t.tile = c->T;
    t.grid_split = c->grid_split;
    t.degrid_batches = c->deg_batches;
    t.fft_col_tile = fft_col_tile(c);
    t.grid_xcd_group = c->grid_group;
    t.degrid_xcd_group = c->deg_group;
    t.ms = c->tune_ms;
    return t;
}

static bool tile_ok(const hs_ctx* c, int T) {
    return T >= 8 && T <= 32 && (T & (T - 1)) == 0 && c->Kx % T == 0 && c->Ky % T == 0 && c->Kx / T >= 3 &&
           c->Ky / T >= 3;
}

static hs_status apply_tuning(hs_ctx* c, const hs_tuning& t) {
    if (t.tile && !tile_ok(c, t.tile)) return fail(c, HS_ERR_INVALID_ARG, "tuning: tile must be 8, 16 or 32 (>= 3 tiles per dimension)");
    if (t.grid_split && (t.grid_split < 64 || t.grid_split > (1 << 20)))
        return fail(c, HS_ERR_INVALID_ARG, "tuning: grid_split in 64..2^20");
    if (t.degrid_batches && (t.degrid_batches < 1 || t.degrid_batches > 64))
        return fail(c, HS_ERR_INVALID_ARG, "tuning: degrid_batches in 1..64");
    if (t.fft_col_tile && !fft_col_tile_ok(c, t.fft_col_tile))
        return fail(c, HS_ERR_INVALID_ARG, "tuning: fft_col_tile must be a power of two that fits the column passes");
    if (t.grid_xcd_group < 0 || t.grid_xcd_group > 4096 || t.degrid_xcd_group < 0 || t.degrid_xcd_group > 4096)
        return fail(c, HS_ERR_INVALID_ARG, "tuning: XCD groups in 1..4096");
    c->tune_tile = t.tile;
    c->grid_split = t.grid_split ? t.grid_split : GRID_SPLIT;
    c->deg_batches = t.degrid_batches ? t.degrid_batches : DEG_BATCHES;
    c->fft_ct = t.fft_col_tile;
    c->grid_group = t.grid_xcd_group ? t.grid_xcd_group : GRID_XCD_GROUP;
    c->deg_group = t.degrid_xcd_group ? t.degrid_xcd_group : DEG_XCD_GROUP;
    c->tune_ms = t.ms;
    return HS_OK;
}

// Plans with the context's tunables; the workspace size is recomputed and the
// context left unbound.
static hs_status replan(hs_ctx* c) {
    hs_status s = build_plan(c);
    if (s) return s;
    c->ws_bytes = carve(c, nullptr);
    c->planned = true;
    c->bound = false;
    c->pd_ready = false;
    c->graph_valid = false;
    return HS_OK;
}

static std::string tune_key(const hs_ctx* c) {
    std::ostringstream k;
    k << c->nx << "x" << c->ny << "x" << c->L << "_M" << c->Mtot << "_" << (c->dtype == HS_F32 ? "f32" : "f64");
    return k.str();
}

static bool cache_lookup(const char* path, const std::string& key, hs_tuning& t) {
    std::ifstream in(path);
    std::string line;
    bool found = false;
    const std::string pat = "\"key\": \"" + key + "\"";
    while (std::getline(in, line)) {
        if (line.find(pat) == std::string::npos) continue;
        hs_tuning u{};
        auto num = [&](const char* name, double& v) {
            const std::string f = std::string("\"") + name + "\": ";
            const size_t p = line.find(f);
            if (p == std::string::npos) return false;
            v = std::atof(line.c_str() + p + f.size());
            return true;
        };
        double a, b, d, e, ms = 0;
        if (num("tile", a) && num("grid_split", b) && num("degrid_batches", d) && num("fft_col_tile", e)) {
            num("ms", ms);
            u.tile = (int)a;
            u.grid_split = (int)b;
            u.degrid_batches = (int)d;
            u.fft_col_tile = (int)e;
            double gg = 0, dg = 0;   // absent in older entries: the defaults
            if (num("grid_xcd_group", gg)) u.grid_xcd_group = (int)gg;
            if (num("degrid_xcd_group", dg)) u.degrid_xcd_group = (int)dg;
            u.ms = ms;
            t = u;
            found = true;   // the last entry of the key wins
        }
    }
    return found;
}

static void cache_append(const char* path, const std::string& key, const hs_tuning& t) {
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f,
                 "{\"key\": \"%s\", \"tile\": %d, \"grid_split\": %d, \"degrid_batches\": %d, \"fft_col_tile\": %d, "
                 "\"grid_xcd_group\": %d, \"degrid_xcd_group\": %d, \"ms\": %.5f}\n",
                 key.c_str(), t.tile, t.grid_split, t.degrid_batches, t.fft_col_tile, t.grid_xcd_group,
                 t.degrid_xcd_group, t.ms);
    std::fclose(f);
}

// Fastest of 8 runs (after one warm-up) of the data-fidelity branch of one PD
// iteration on the bound workspace (F Z, the degridding and dual step, the
// projection roots and update, the gridding, F^H Z^T): the operators the
// decomposition shapes.  It starts from the zero state the workspace was bound with.
template <typename T>
static hs_status time_ops(hs_ctx* c, double& ms) {
    hipEvent_t e0, e1;
    hs_status s = hip_check(c, hipEventCreate(&e0), "hipEventCreate");
    if (s) return s;
    s = hip_check(c, hipEventCreate(&e1), "hipEventCreate");
    if (s) { (void)hipEventDestroy(e0); return s; }
    std::vector<double> t;
    for (int r = 0; r < 9 && !s; ++r) {
        (void)hipEventRecord(e0, c->stream);
        dual_data_impl<T>(c, (cplx<T>*)c->d.v, (const T*)c->d.Xt, (T*)c->d.img0);
        (void)hipEventRecord(e1, c->stream);
        s = hip_check(c, hipEventSynchronize(e1), "autotune timing");
        float m = 0.f;
        if (!s) s = hip_check(c, hipEventElapsedTime(&m, e0, e1), "hipEventElapsedTime");
        if (r > 0) t.push_back(m);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s) return s;
    ms = *std::min_element(t.begin(), t.end());
    return launched(c, "autotune timing");
}

}  // namespace hs

extern "C" {

hs_status hs_get_tuning(const hs_ctx* c, hs_tuning* out) {
    if (!c || !out) return HS_ERR_INVALID_ARG;
    if (!c->planned) return HS_ERR_NOT_PLANNED;
    *out = tuning_of(c);
    return HS_OK;
}

hs_status hs_set_tuning(hs_ctx* c, const hs_tuning* t) {
    HS_TRY_BEGIN
    if (!c || !t) return HS_ERR_INVALID_ARG;
    const int T0 = c->tune_tile, g0 = c->grid_split, b0 = c->deg_batches;
    hs_status s = apply_tuning(c, *t);
    if (s) return s;
    c->graph_valid = false;   // launch parameters are captured in the graph
    // the FFT column tile and the XCD groups are launch parameters: no new plan
    if (c->planned && (c->tune_tile != T0 || c->grid_split != g0 || c->deg_batches != b0)) return replan(c);
    return HS_OK;
    HS_TRY_END(c)
}

hs_status hs_autotune_bytes(hs_ctx* c, size_t* bytes) {
    HS_TRY_BEGIN
    if (!c || !bytes) return HS_ERR_INVALID_ARG;
    if (!c->planned) return fail(c, HS_ERR_NOT_PLANNED, "call hs_plan first");
    const hs_tuning keep = tuning_of(c);
    const int keep_tile = c->tune_tile, keep_ct = c->fft_ct;
    size_t mx = c->ws_bytes;
    hs_status s = HS_OK;
    // the largest plan: each tile edge with the smallest units
    for (int T : {8, 16, 32}) {
        if (!tile_ok(c, T)) continue;
        hs_tuning t{T, 512, 2, 0, 0, 0, 0.0};
        s = apply_tuning(c, t);
        if (!s) s = build_plan(c);
        if (s) break;
        mx = std::max(mx, carve(c, nullptr));
    }
    hs_tuning back = keep;
    back.tile = keep_tile;
    back.fft_col_tile = keep_ct;
    hs_status s2 = apply_tuning(c, back);
    if (!s2) s2 = build_plan(c);
    if (s) return s;
    if (s2) return s2;
    *bytes = mx;
    return HS_OK;
    HS_TRY_END(c)
}

hs_status hs_autotune(hs_ctx* c, void* dev, size_t bytes, const char* cache_path, hs_tuning* chosen) {
    HS_TRY_BEGIN
    if (!c) return HS_ERR_INVALID_ARG;
    if (!c->planned) return fail(c, HS_ERR_NOT_PLANNED, "call hs_plan first");
    const std::string key = tune_key(c);
    hs_tuning best{};
    hs_status s = HS_OK;
    if (cache_path && cache_lookup(cache_path, key, best)) {
        s = apply_tuning(c, best);
        if (!s) s = replan(c);
        if (!s && chosen) *chosen = tuning_of(c);
        return s;
    }
    if (!dev || ((uintptr_t)dev & 255)) return fail(c, HS_ERR_INVALID_ARG, "autotune workspace: 256-byte aligned device memory");
    s = hip_check(c, hipSetDevice(c->device), "hipSetDevice");
    if (s) return s;
    fft_init_attrs();
    // evaluate one decomposition: plan, lay out in the temporary workspace, upload, time
    auto eval = [&](const hs_tuning& t, double& ms) -> hs_status {
        hs_status r = apply_tuning(c, t);
        if (!r) r = build_plan(c);
        if (r) return r;
        const size_t need = carve(c, nullptr);
        if (need > bytes) return fail(c, HS_ERR_NO_WORKSPACE, "autotune workspace too small (see hs_autotune_bytes)");
        carve(c, (char*)dev);
        c->planned = true;
        r = c->dtype == HS_F32 ? bind_impl<float>(c) : bind_impl<double>(c);
        if (r) return r;
        c->bound = true;
        r = c->dtype == HS_F32 ? time_ops<float>(c, ms) : time_ops<double>(c, ms);
        c->bound = false;
        return r;
    };
    best = hs_tuning{0, GRID_SPLIT, DEG_BATCHES, 0, GRID_XCD_GROUP, DEG_XCD_GROUP, 0.0};
    double best_ms = 1e30;
    // coordinate descent: tile edge, gridding split, degridding unit, FFT column tile
    for (int T : {32, 16, 8}) {
        if (!tile_ok(c, T)) continue;
        hs_tuning t = best;
        t.tile = T;
        double ms;
        if ((s = eval(t, ms))) return s;
        if (ms < TUNE_MARGIN * best_ms) { best_ms = ms; best = t; }
    }
    for (int g : {512, 2048}) {
        hs_tuning t = best;
        t.grid_split = g;
        double ms;
        if ((s = eval(t, ms))) return s;
        if (ms < TUNE_MARGIN * best_ms) { best_ms = ms; best = t; }
    }
    for (int b : {2, 8}) {
        hs_tuning t = best;
        t.degrid_batches = b;
        double ms;
        if ((s = eval(t, ms))) return s;
        if (ms < TUNE_MARGIN * best_ms) { best_ms = ms; best = t; }
    }
    {
        // the column tile needs no new plan: time it on the best plan
        hs_tuning base = best;
        double ms;
        if ((s = eval(base, ms))) return s;
        best_ms = std::min(best_ms, ms);
        base.fft_col_tile = fft_col_tile(c);
        best = base;
        for (int ct : {2, 4, 8, 16}) {
            if (ct == base.fft_col_tile || !fft_col_tile_ok(c, ct)) continue;
            c->fft_ct = ct;
            if ((s = (c->dtype == HS_F32 ? [&] { carve(c, (char*)dev); c->bound = true; return time_ops<float>(c, ms); }()
                                         : [&] { carve(c, (char*)dev); c->bound = true; return time_ops<double>(c, ms); }())))
                return s;
            c->bound = false;
            if (ms < TUNE_MARGIN * best_ms) { best_ms = ms; best = base; best.fft_col_tile = ct; }
        }
    }
    {
        // XCD groups of the gridding and degridding units: launch parameters too
        c->fft_ct = best.fft_col_tile;
        for (int which = 0; which < 2; ++which)
            for (int g : {1, 4, 16, 64}) {
                hs_tuning t = best;
                int& field = which ? t.degrid_xcd_group : t.grid_xcd_group;
                if (field == g) continue;
                field = g;
                c->grid_group = t.grid_xcd_group;
                c->deg_group = t.degrid_xcd_group;
                double ms;
                carve(c, (char*)dev);
                c->bound = true;
                s = c->dtype == HS_F32 ? time_ops<float>(c, ms) : time_ops<double>(c, ms);
                c->bound = false;
                if (s) return s;
                if (ms < TUNE_MARGIN * best_ms) { best_ms = ms; best = t; }
            }
    }
    best.ms = best_ms;
    s = apply_tuning(c, best);
    if (!s) s = replan(c);
    if (s) return s;
    if (cache_path) cache_append(cache_path, key, tuning_of(c));
    if (chosen) *chosen = tuning_of(c);
    return HS_OK;
    HS_TRY_END(c)
}

}  // extern "C"
