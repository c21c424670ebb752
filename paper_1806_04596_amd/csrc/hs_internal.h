// Internal declarations of the HyperSARA gfx950 library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "hypersara.h"

namespace hs {

constexpr int KB_J = 8;             // kernel support per dimension (taps)
constexpr int KB_MAX_TERMS = 40;    // power-series terms of the kernel (upper bound)
constexpr int MAX_L = 64;           // channels (Gram matrix edge)
constexpr int DEG_THREADS = 256;    // degridding workgroup = one batch of visibilities
constexpr int DEG_BATCHES = 4;      // default batches per degridding work unit (tunable)
constexpr int GRID_SPLIT = 1024;    // default entries per gridding work unit (tunable)
constexpr int GRID_XCD_GROUP = 64;  // default gridding units per XCD turn (tunable)
constexpr int DEG_XCD_GROUP = 4;    // default degridding units per XCD turn (tunable)
constexpr int MAX_DB = 8;
constexpr int MAX_TAPS = 16;        // 2 * MAX_DB

// One degridding work unit: `count` (<= DEG_THREADS*DEG_BATCHES) visibilities of
// one tile of channel l starting at global position `start`.  Runs of equal bin
// are cut at every DEG_CHUNK visibilities of the unit (one wave's share);
// chunk_run[chunk0 + j] is the number of the first run of chunk j; the sums of
// run r are stored at slot run_slot[r], so that each bin's runs are contiguous.
constexpr int DEG_CHUNK = 64;
struct DegridUnit {
    int32_t l, tile, start, count;
    int32_t run_base, chunk0, pad1, pad2;
};

// One gridding work unit: entries [g0, g0 + gn) of the sorted entry list of
// `tile` of channel l (its own visibilities and its neighbours' border ones, by
// first-tap cell), part `split` of `nsplit`.  nsplit > 1 writes a partial tile
// to slot partial + split; nsplit == 1 writes the grid directly.
// Gridding works on GB x GB output blocks of the half-plane grid; the grid rows
// carry GR_MARGIN cells beyond kx = 0 and kx = Kx/2 (column = kx + GR_MARGIN).
constexpr int GB = 16;
constexpr int GR_MARGIN = 32;
// One gridding work unit: entries [g0, g0 + gn) of the entry list of output
// block `tile` of channel l (every visibility whose footprint meets the block),
// part `split` of `nsplit`.  nsplit > 1 writes a partial block to slot
// partial + split; nsplit == 1 writes the grid directly.
struct GridUnit {
    int32_t l, tile, split, nsplit;
    int32_t partial, g0, gn, pad;
};

// A tile whose gridding was split: the partials are summed in order.
struct SplitTile {
    int32_t l, tile, partial, nsplit;
};

// The kernel values of a visibility, phi(f + 3 - j) for taps j = 0..7 and the
// fractional offset f in [0, 1), as one polynomial per tap in t = f - 1/2 (the
// Chebyshev interpolant of phi on that tap's unit interval, in monomial form).
// phi is even, so tap 7 - j is tap j at -t: only taps 0..3 are stored, each
// split into its even and odd parts, p_j(+-t) = E_j(t^2) +- t O_j(t^2).
// Degree per precision (maximum error 1e-7 in FP32 Horner arithmetic, 6e-15 in FP64,
// relative to phi(0); FP32 rounding dominates from degree 7 on).
template <typename T> struct KBDeg;
template <> struct KBDeg<float> { static constexpr int n = 7; };
template <> struct KBDeg<double> { static constexpr int n = 13; };

template <typename T>
struct KBPoly {
    static constexpr int NE = KBDeg<T>::n / 2 + 1;        // even coefficients t^0, t^2, ...
    static constexpr int NO = (KBDeg<T>::n + 1) / 2;      // odd coefficients t^1, t^3, ...
    T e[4][NE];
    T o[4][NO];
};

template <typename T>
struct alignas(2 * sizeof(T)) cplx {   // aligned to its size: one 64/128-bit access
    T re, im;
};

// Device pointers carved from the caller's workspace.
struct Dev {
    // per visibility, tile-major order
    int32_t* vis_cell = nullptr;   // (cy << 16) | (reflected << 15) | cx, half-plane cell
    void* vis_frac = nullptr;      // [M][2] real, t - floor(t)
    void* vis_y = nullptr;         // [M] complex, theta * y_raw
    void* vis_theta = nullptr;     // [M] real
    void* vis_u = nullptr;         // [M] real, preconditioner
    int32_t* vis_bin = nullptr;    // [M] global bin
    int32_t* vis_perm = nullptr;   // [M] caller's global index
    int32_t* vis_pos = nullptr;    // [M] caller's global index -> position
    void* v = nullptr;             // [M] complex, PD dual
    void* vwork = nullptr;         // [M] complex scratch
    // work lists
    DegridUnit* dunits = nullptr;
    GridUnit* gunits = nullptr;
    SplitTile* splits = nullptr;
    int32_t* glist = nullptr;      // gridding entries: plan positions, per tile sorted by first-tap cell
    void* gpartial = nullptr;      // [npartial][T*T] complex
    // bins / blocks
    double* bin_u = nullptr;       // [nbins]
    int32_t* blk_bin_ptr = nullptr;// [nblk+1]
    double* blk_eps = nullptr;     // [nblk]
    double* blk_lambda = nullptr;  // [nblk]
    double* blk_rho2 = nullptr;    // [nblk] ||y - Phi Xt||^2 (residual norms, Sec. 3.6)
    int32_t* blk_vartheta = nullptr; // [nblk]
    double* run_sum = nullptr;     // [nruns][2] (|d|^2, |y - Phi Xt|^2)
    int32_t* bin_run_ptr = nullptr;// [nbins+1]
    int32_t* run_slot = nullptr;   // [nruns] slot of each run's sums in run_sum (grouped by bin)
    int32_t* chunk_run = nullptr;  // [chunks] first run of each DEG_CHUNK-visibility chunk
    double* bin_S = nullptr;       // [nbins][2]
    double* bin_f = nullptr;       // [nbins] lam/(u + lam) of each bin's visibilities (v = f d)
    // FFT
    void* grid = nullptr;          // [L][Ky][Kx] complex
    void* H = nullptr;             // [L][ny][Kx] complex
    void* tw_x = nullptr;          // [Kx] complex exp(-2 pi i k/Kx)
    void* tw_y = nullptr;          // [Ky]
    void* sx = nullptr;            // [nx] real
    void* sy = nullptr;            // [ny] real
    // images
    void* X = nullptr;
    void* Xt = nullptr;
    void* P = nullptr;
    void* img0 = nullptr;
    void* img1 = nullptr;
    void* A = nullptr;             // [D][L][N]
    void* coef = nullptr;          // [n_db][L][N]
    void* wtmp = nullptr;          // [n_db][L][N]
    void* wbar = nullptr;          // [D][N] ([D][L][N] for the SARA prior)
    void* filt = nullptr;          // [n_db][2][16] real (h, g)
    // nuclear norm
    double* gram_part = nullptr;   // [ngram][64][64]
    double* gram = nullptr;        // [64][64]
    double* eigV = nullptr;        // [64][64]
    double* eig_sig = nullptr;     // [64]
    double* w_nuc = nullptr;       // [64]
    void* Wmat = nullptr;          // [64][64] real
    // reductions
    double* red_part = nullptr;    // [nred][4]
    double* scal = nullptr;        // [64]: beta, iteration, ||dX||^2, ||X||^2
    double* chan_nrm = nullptr;    // [64] per-channel norms
};

// FP64 copies of what the measurement operator reads, for the FP64 power iteration
// of an FP32 context (the step-size norm stays in FP64, Sec. 3.4).
struct Dev64 {
    void* vis_frac = nullptr;      // [M][2] double
    void* vis_theta = nullptr;     // [M] double
    void* vis_u = nullptr;         // [M] double
    void* vwork = nullptr;         // [M] complex double
    void* gpartial = nullptr;      // [npartial][GB*GB] complex double
    void* grid = nullptr;          // [L][Ky][Wg] complex double
    void* H = nullptr;             // [L][ny][Hs] complex double
    void* tw_x = nullptr;
    void* tw_y = nullptr;
    void* sx = nullptr;
    void* sy = nullptr;
    void* x = nullptr;             // [L][N] double, the iterate
};

struct Channel {
    bool set = false;
    int64_t M = 0;
    int32_t nb = 0;
    std::vector<int64_t> bp;
    std::vector<double> uv, y, theta, u, eps;
    bool has_u = false;
};

enum { NRED = 512, NGRAM = 512 };

}  // namespace hs

struct hs_ctx {
    hs_problem_desc desc{};
    int nx = 0, ny = 0, L = 0, Kx = 0, Ky = 0, D = 0, n_db = 0, levels = 0;
    int64_t N = 0;
    int dtype = HS_F32;
    int gram_mode = HS_GRAM_F64;
    size_t rsz = 4;  // sizeof(real)
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    std::vector<hs::Channel> ch;
    // plan
    bool planned = false, bound = false;
    // Hermitian half plane: visibilities live at kx in [0, Kx/2] (those at
    // negative kx are reflected); visibility tiles cover [0, Kx/2 + T), gridding
    // blocks [-GB, Kx/2 + GB) of the Wg columns of a grid row (column = kx + GR_MARGIN).
    int T = 32, tiles_x = 0, tiles_y = 0, ntiles = 0;   // visibility tiles
    // tunables (hs_set_tuning / hs_autotune): tile edge (0 = rule), entries per gridding
    // unit, batches per degridding unit, columns per FFT column tile (0 = rule)
    int tune_tile = 0, grid_split = hs::GRID_SPLIT, deg_batches = hs::DEG_BATCHES, fft_ct = 0;
    int grid_group = hs::GRID_XCD_GROUP, deg_group = hs::DEG_XCD_GROUP;   // XCD grouping of the work units
    double tune_ms = 0.0;
    int gtiles_x = 0, ngtiles = 0;                      // gridding blocks (GB x GB) in x, in all
    int Kh = 0, Wh = 0, Wg = 0, Hs = 0;                 // Kx/2, Kx/2 + 1, Kx/2 + 2 GR_MARGIN, Kx/2 + 16
    int64_t Mtot = 0;
    std::vector<int64_t> chan_off;     // [L+1]
    std::vector<int32_t> blk_off;      // [L+1]
    int64_t nblk = 0, nbins = 0, nruns = 0, npartial = 0;
    std::vector<hs::DegridUnit> dunits;
    std::vector<hs::GridUnit> gunits;
    std::vector<hs::SplitTile> splits;
    // per-channel ranges [off[l], off[l + 1]) of the work lists and bins (one launch
    // per channel in the plain, unbatched execution)
    std::vector<int64_t> dunit_off, gunit_off, split_off, bin_off;
    bool per_channel = false;          // plain execution: one launch per channel, eager iteration
    int kb_terms = 0;
    std::vector<double> kb_c;          // power-series coefficients
    std::vector<double> kb_c64;        // FP64 coefficients (the FP64 power iteration of an FP32 context)
    // host staging of the plan (uploaded at bind)
    std::vector<int32_t> h_cell, h_bin, h_perm, h_glist, h_blk_bin_ptr, h_bin_run_ptr, h_run_slot;
    std::vector<int32_t> h_chunk_run;
    std::vector<double> h_frac, h_y, h_theta, h_u, h_bin_u, h_blk_eps;
    std::vector<int64_t> h_pos_of;     // caller global index -> grid position
    size_t ws_bytes = 0;
    void* ws = nullptr;
    hs::Dev d;
    hs::Dev64 d64;                     // FP32 contexts only
    // PD
    bool pd_ready = false;
    double mu = 0, tau = 0.33, k1 = 1, k2 = 0, k3 = 0;
    bool adaptive = false;
    double lam1 = 5e-4, lam2 = 0.01, lam3 = 0.618;
    int vartheta_bar = 100;
    int prior = HS_PRIOR_LRJAS;        // which prior terms the iteration carries
    int64_t t_iter = 0;
    std::vector<double> w_host;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t side[2] = {nullptr, nullptr};   // fork/join branches of the captured iteration
    hipEvent_t ev_fork = nullptr, ev_mid = nullptr, ev_join[2] = {nullptr, nullptr};
    bool graph_valid = false;
};

namespace hs {

// ------------------------------------------------------------ host helpers
hs_status fail(hs_ctx* c, hs_status s, const std::string& msg);
hs_status hip_check(hs_ctx* c, hipError_t e, const char* what);
// Monomial coefficients in t = f - 1/2 of taps 0..3, [4][deg + 1].
void kb_taps(int deg, std::vector<double>& coef);
double kb_ft(double xi);
void daubechies_host(int K, double* h);

// ------------------------------------------------------------ kernel launchers
template <typename T> void launch_fill(hipStream_t s, T* p, T v, int64_t n);
template <typename S, typename D> void launch_convert(hipStream_t s, D* dst, const S* src, int64_t n);
template <typename T> void launch_axpby(hipStream_t s, T* y, const T* x, T a, T b, int64_t n);   // y = a*x + b*y

// NUFFT (k_nufft.hip)
void fft_init_attrs();
int fft_col_tile(const hs_ctx* c);              // columns per column-pass tile in use
bool fft_col_tile_ok(const hs_ctx* c, int ct);  // ct fits the column passes of c
// Channel ranges: the FFT launchers transform channels l0 .. l0 + L - 1; lc < 0 means
// every channel, lc >= 0 channel lc only (the plain, one-launch-per-channel execution).
template <typename T> void launch_fft_rows_fwd(hs_ctx* c, const T* X, int L, int l0 = 0);
template <typename T> void launch_fft_cols_fwd(hs_ctx* c, int L, int l0 = 0);
template <typename T> void launch_fft_cols_adj(hs_ctx* c, int L, int l0 = 0);
template <typename T> void launch_fft_rows_adj(hs_ctx* c, T* Xout, int L, int l0 = 0);
template <typename T> void launch_degrid_plain(hs_ctx* c, cplx<T>* out_user, int lc = -1);
template <typename T> void launch_degrid_grid_order(hs_ctx* c, cplx<T>* out, const T* mult, int lc = -1);
template <typename T> void launch_degrid_dual_v(hs_ctx* c, cplx<T>* v, int lc = -1);
template <typename T> void launch_bins_and_roots(hs_ctx* c, int lc = -1);
template <typename T> void launch_dual_apply_v(hs_ctx* c, cplx<T>* v, int lc = -1);
template <typename T> void launch_grid_pull(hs_ctx* c, const cplx<T>* vals, const T* weight, int lc = -1);
template <typename T> void launch_gather_user(hs_ctx* c, const cplx<T>* in_user, cplx<T>* out_grid, bool times_theta);
template <typename T> void launch_scatter_user(hs_ctx* c, const cplx<T>* in_grid, cplx<T>* out_user);
template <typename T> void launch_proj_block(hs_ctx* c, int64_t pos0_user, int64_t Mb, int blk, cplx<T>* z);

// wavelets (k_wavelet.hip)
// nl: channels of the arrays (default: all L)
template <typename T> void launch_psi_adj(hs_ctx* c, const T* X, T* Cout /*[n_db][L][N]; null -> coef*/, int nl = -1);
template <typename T> void launch_psi_sum(hs_ctx* c, const T* Cdb /*[n_db][L][N]*/, const T* C0, T* Xout, int nl = -1);
template <typename T> void launch_l21_dual(hs_ctx* c, T* A, const T* Xt, const T* coef, const T* wbar, double thr, int mode);

// nuclear (k_nuclear.hip)
// Gram of P + Xt (Xt may be null) in the context's Gram precision, or in FP64 when force64.
template <typename T> void launch_gram(hs_ctx* c, const T* P, const T* Xt, bool force64 = false);
void launch_eig(hs_ctx* c, int mode);
// Rayleigh-Ritz refinement of the eigen-decomposition (FP64 contexts, and the BF16-split
// Gram of FP32 contexts); eig_refined says whether a context applies it.
template <typename T> void launch_eig_refine(hs_ctx* c, const T* P, const T* Xt, int mode);
bool eig_refined(const hs_ctx* c, bool force64 = false);
void launch_eig_reset(hs_ctx* c);
template <typename T> void launch_backproject(hs_ctx* c, T* out, const T* in1, const T* in2);

// primal and helpers (k_misc.hip)
template <typename T> void launch_primal(hs_ctx* c, const T* Atsum, const T* Dimg, bool use_p);
template <typename T> void launch_chan_norms(hs_ctx* c, const T* X, double* out);
template <typename T> void launch_chan_max(hs_ctx* c, const T* X, double* out);
template <typename T> void launch_set_center(hs_ctx* c, T* X);
template <typename T> int launch_l21_norm(hs_ctx* c, const T* X, const T* coef);
template <typename T> void launch_l21_rowsq(hs_ctx* c, const T* X, const T* coef, int nl, double* S, bool acc);
template <typename T> void launch_l21_rowscale(hs_ctx* c, T* X, T* coef, int nl, const double* S, const T* wbar, double scale);
template <typename T> int launch_l21_from_rowsq(hs_ctx* c, const double* S, const T* wbar);
template <typename T> void launch_chan_scale(hs_ctx* c, T* X, const double* nrm);
template <typename T> void launch_reweight_l21(hs_ctx* c, const T* X, const T* coef, T* wbar, double gb);
template <typename T> void launch_reweight_l1(hs_ctx* c, const T* X, const T* coef, T* wbar, double gb);

}  // namespace hs
