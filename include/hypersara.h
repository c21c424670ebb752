/*
 * hypersara.h -- C ABI of the MI355X (gfx950) HyperSARA primal-dual hot path.
 *
 * Method: Abdulaziz, Dabbech & Wiaux, "Wideband super-resolution imaging in
 * radio interferometry via low rankness and joint average sparsity models
 * (HyperSARA)", MNRAS, arXiv:1806.04596.  Sections, equation labels and
 * algorithm steps of that paper are cited per entry point.
 *
 * Conventions (all entry points):
 *  - Every call returns hs_status (0 = HS_OK, negative = error); no C++
 *    exception crosses this boundary.  hs_last_error(ctx) gives a message.
 *  - A context fixes the problem shape and the working precision (HS_F32 or
 *    HS_F64).  "real" below is float or double accordingly, "complex" is two
 *    interleaved reals (re, im).
 *  - Image cubes are [L][ny][nx] row-major (row j = y, column i = x), pixel
 *    (i, j) sits at (i - nx/2, j - ny/2) from the phase centre.
 *  - uv coordinates are in cycles per pixel at the channel's own frequency.
 *  - Device pointers must be device memory of the context's device, sized as
 *    stated; they are borrowed for the call only.  Device work is enqueued on
 *    the stream given in hs_problem_desc and is asynchronous unless a call is
 *    documented as synchronising.  Asynchronous device faults surface as
 *    HS_ERR_HIP at the next synchronising call.
 *  - Host pointers are read during the call only (the library copies them).
 *  - The library never allocates device memory: hs_plan reports the
 *    workspace size and the caller binds a buffer with hs_bind_workspace.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef HYPERSARA_H
#define HYPERSARA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hs_status;
enum {
    HS_OK = 0,
    HS_ERR_INVALID_ARG = -1,
    HS_ERR_SHAPE = -2,
    HS_ERR_DTYPE = -3,
    HS_ERR_NOT_PLANNED = -4,
    HS_ERR_NO_WORKSPACE = -5,
    HS_ERR_NONFINITE = -6,
    HS_ERR_HIP = -7,
    HS_ERR_NOT_CONVERGED = -8
};

enum { HS_F32 = 0, HS_F64 = 1 };
enum { HS_NORM_PHI_PRECOND = 0, HS_NORM_PSI = 1 };

typedef struct hs_ctx hs_ctx;

/* Precision of the L x L Gram matrix of the nuclear-norm prox (eq:prox-L*, taken
 * through the Gram matrix; the eigen-decomposition is FP64 in every mode):
 *   HS_GRAM_F64        FP64 products of the exactly widened inputs (default);
 *   HS_GRAM_F32        FP32 products, FP32 accumulation within a slab of pixels,
 *                      FP64 across slabs;
 *   HS_GRAM_BF16_SPLIT each input z = z_hi + z_lo with both parts in BF16 and
 *                      C ~ Z_hi^T Z_hi + Z_hi^T Z_lo + Z_lo^T Z_hi, FP32 accumulation
 *                      within a slab, FP64 across slabs; then one refinement step.
 * The refinement (a Rayleigh-Ritz step) forms H = (Z V)^T (Z V) from the data and the
 * first eigenvectors V (FP64 products) and decomposes it again; the eigenvectors are
 * V times those of H.  H carries rounding of order eps sigma_i sigma_j where C carries
 * eps sigma_1^2, so the small singular values and their directions come out as
 * accurate as from a direct SVD.  FP64 contexts always refine; FP32 contexts refine in
 * the BF16-split mode only. */
enum { HS_GRAM_F64 = 0, HS_GRAM_F32 = 1, HS_GRAM_BF16_SPLIT = 2 };

/* Problem description (Sec. 2.1 data model, Sec. 2.3 dictionary).
 * nx, ny: image size; powers of two in 16..2048 (and >= 2^levels).
 * L: number of channels (1..64).
 * oversamp: grid oversampling per dimension; must be 2.
 * J: Kaiser-Bessel support per dimension; must be 8.
 * levels: wavelet depth (1..6), n_db: number of Daubechies bases (0..8),
 *   the dictionary is Dirac + db1..db{n_db} (D = 1 + n_db bases).
 * dtype: HS_F32 or HS_F64.  tile: gridding tile edge (0 = automatic; else a
 *   power of two in 8..32 with 2*nx/tile >= 3 and 2*ny/tile >= 3).
 * device: HIP device ordinal; stream: hipStream_t (NULL = default stream).
 * gram_mode: HS_GRAM_F64 / HS_GRAM_F32 / HS_GRAM_BF16_SPLIT (above).
 * per_channel: 0 = batched execution (every operator one launch over all
 *   channels, the PD iteration replayed from a captured HIP graph); nonzero =
 *   plain execution (the channel-separable operators launched channel by
 *   channel, the iteration eager), the comparator of the batched path. */
typedef struct {
    int32_t nx, ny, L;
    int32_t oversamp;
    int32_t J;
    int32_t levels;
    int32_t n_db;
    int32_t dtype;
    int32_t tile;
    int32_t device;
    void* stream;
    int32_t gram_mode;
    int32_t per_channel;
} hs_problem_desc;

/* Sizes after hs_plan. */
typedef struct {
    int64_t n_vis;          /* sum of M_l */
    int64_t n_blocks;       /* sum of B_l */
    int64_t n_bins;         /* (block, preconditioner value) pairs that occur (<= n_vis + n_blocks) */
    int64_t n_runs;         /* segmented-reduction runs */
    int64_t n_degrid_units; /* degridding work units */
    int64_t n_grid_units;   /* gridding work units */
    int32_t tile;           /* tile edge used */
    int32_t kb_terms;       /* coefficients of the kernel's per-tap polynomials */
    size_t workspace_bytes;
} hs_info;

/* Parameters of one adaptive PPD iteration (Algorithm 2, Sec. 3.4).
 * kappa1 <= 0 -> 1; kappa2 <= 0 -> 1/D (= 1/||Psi^dagger||_S^2);
 * kappa3 must be > 0 (1/||U^{1/2} Phi||_S^2, see hs_op_norm).
 * tau: primal step, convergence needs tau(k1 + k2 D + k3 ||U^1/2 Phi||^2) < 1.
 * wbar: device real [D][ny][nx] l2,1 weights, one per coefficient row (NULL = ones),
 *    copied; for HS_PRIOR_SARA one weight per channel and coefficient, [D][L][ny][nx].
 * w: host double [L] nuclear weights paired with singular values in
 *    decreasing order (NULL = ones), copied.
 * adaptive_eps: nonzero enables the adaptive l2 bounds (Sec. 3.6) with lam1..lam3, vartheta_bar
 *    (Appendix A: 5e-4, 0.01, 0.618, 100).
 * prior: the regularisation of the minimisation task (Sec. 2.3, Sec. 4.2):
 *    HS_PRIOR_LRJAS  low rankness + joint average sparsity (eq:min; reweighted by
 *                    hs_solve this is HyperSARA),
 *    HS_PRIOR_LR     nuclear norm only (eq:min-lr),
 *    HS_PRIOR_JAS    l2,1 norm only (eq:min-js),
 *    HS_PRIOR_SARA   weighted l1 norm of each channel's coefficients, no
 *                    nuclear norm (eq:min-sara: one problem per channel, with
 *                    weights per channel and coefficient; hs_solve reweights
 *                    them as SARA's reweighted l1, Sec. 2.3).
 *    A prior that is off leaves its dual (P or A) untouched. */
enum { HS_PRIOR_LRJAS = 0, HS_PRIOR_LR = 1, HS_PRIOR_JAS = 2, HS_PRIOR_SARA = 3 };
typedef struct {
    double mu, tau, kappa1, kappa2, kappa3;
    const void* wbar;
    const double* w;
    int32_t adaptive_eps;
    double lam1, lam2, lam3;
    int32_t vartheta_bar;
    int32_t prior;
} hs_pd_params;

/* The state of Algorithm 2 (its "Given" line) and the weights of Algorithm 1.
 * Device pointers, ctx dtype: X, Xt, P: [L][ny][nx]; A: [D][L][ny][nx];
 * v: [sum M_l] complex in the caller's visibility order (channel by channel,
 * each in the order given to hs_set_channel); wbar: the sparsity weights
 * (shape as in hs_pd_params).
 * Host pointers: eps: double [n_blocks] l2 bounds and vartheta: int32
 * [n_blocks] iterations of their last update (blocks channel by channel);
 * scalars: double [2] = (beta, t) of the last iteration; w: double [L]
 * nuclear weights.
 * Any member may be NULL: hs_pd_get_state skips it; hs_pd_set_state skips the
 * arrays and restarts the bookkeeping it is not given (eps from hs_set_data,
 * vartheta = 0, beta = 1, t = 0) and keeps the current weights. */
typedef struct {
    void* X;
    void* Xt;
    void* P;
    void* A;
    void* v;
    double* eps;
    int32_t* vartheta;
    double* scalars;
    void* wbar;
    double* w;
} hs_state_ptrs;

/* Outer loop (Algorithm 1).  Each reweight runs iters_per_reweight PD
 * iterations (or stops early when beta < beta_tol, checked every
 * check_every iterations), then updates wbar by eq:weights-l21 and w by
 * eq:weights-n (SARA: the per-channel l1 weights) with gamma, gamma_bar
 * starting at gamma0, gamma_bar0 (<= 0 means 1) and multiplied by
 * gamma_factor after each update.  Warm starts every variable.
 * reweight_first: nonzero starts with a weight update (from the current X),
 * which resumes a solve saved after its last block of iterations. */
typedef struct {
    int32_t n_reweights;
    int32_t iters_per_reweight;
    double gamma_factor;
    double beta_tol;
    int32_t check_every;
    double gamma0, gamma_bar0;
    int32_t reweight_first;
} hs_solve_params;

/* gamma, gamma_bar: the values the next reweight would use (to resume). */
typedef struct {
    int64_t iterations;
    int32_t reweights;
    double final_beta;
    double gamma, gamma_bar;
} hs_report;

/* ---------------------------------------------------------- diagnostics */
const char* hs_status_string(hs_status s);
/* Message of the last error on ctx (or of the last failed hs_create when ctx is NULL). */
const char* hs_last_error(const hs_ctx* ctx);

/* -------------------------------------------------------------- lifecycle */
/* Creates a context; *out is set on success.  Validates the description
 * (HS_ERR_INVALID_ARG / HS_ERR_SHAPE / HS_ERR_DTYPE).  No device memory is
 * allocated. */
hs_status hs_create(const hs_problem_desc* desc, hs_ctx** out);
hs_status hs_destroy(hs_ctx* ctx);

/* Channel data for the measurement model y_l = Phi_l x_l + w_l with
 * Phi_l = Theta_l G_l F Z (eq:inverse) split in blocks (Sec. 2.3).
 * l: channel 0..L-1; M: number of visibilities (>= 0);
 * nblocks, block_ptr[nblocks+1]: contiguous blocks, block_ptr[0] = 0,
 *   non-decreasing, block_ptr[nblocks] = M (nblocks >= 1 when M > 0);
 * uv[M][2]: (u, v) in cycles per pixel; y_raw[M][2]: complex data before
 *   natural weighting; theta[M]: natural weights 1/sigma (> 0);
 * precond[M]: diagonal of U (> 0), or NULL for U = I (Sec. 3.3, the
 *   density preconditioner is available from hs_density_precond);
 * eps[nblocks]: l2 bounds (>= 0).
 * All pointers are host and copied.  Non-finite values -> HS_ERR_NONFINITE.
 * Must be called for every channel before hs_plan. */
hs_status hs_set_channel(hs_ctx* ctx, int32_t l, int64_t M, int32_t nblocks, const int64_t* block_ptr,
                         const double* uv, const double* y_raw, const double* theta,
                         const double* precond, const double* eps);

/* Replaces y_raw, theta and eps of channel l after hs_plan/hs_bind_workspace
 * (same M and blocks).  Host pointers, copied; enqueues uploads on the stream. */
hs_status hs_set_data(hs_ctx* ctx, int32_t l, const double* y_raw, const double* theta, const double* eps);

/* Sorts and bins the visibilities (bit-exact integer keys, see
 * hs_visibility_order), builds the work lists, kernel and FFT tables, and
 * returns the device workspace size in bytes. */
hs_status hs_plan(hs_ctx* ctx, size_t* workspace_bytes);

/* Binds caller-allocated device memory (>= workspace_bytes, 256-byte aligned)
 * and uploads the plan.  The primal-dual state lives in this workspace and
 * starts at zero (Algorithm 2 initialisation). */
hs_status hs_bind_workspace(hs_ctx* ctx, void* dev, size_t bytes);

hs_status hs_get_info(const hs_ctx* ctx, hs_info* info);

/* ---------------------------------------------------------------- tuning */
/* The work decomposition of the batched operators (all channels per launch):
 *   tile:           visibility tile edge of the degridding (8, 16 or 32);
 *   grid_split:     entries per gridding work unit (a 16 x 16 output block with
 *                   more entries is split and its partial blocks summed);
 *   degrid_batches: batches of 256 visibilities per degridding work unit;
 *   fft_col_tile:   columns per work-group of the FFT column passes (2..16);
 *   grid_xcd_group, degrid_xcd_group: consecutive work units (which share input:
 *                   neighbouring blocks and tiles) given to one XCD before the
 *                   next, in 1..4096 (1: one unit per XCD in turn);
 *   ms:             measured time of this choice (0: not measured).
 * A 0 field means the library's default. */
typedef struct {
    int32_t tile;
    int32_t grid_split;
    int32_t degrid_batches;
    int32_t fft_col_tile;
    int32_t grid_xcd_group;
    int32_t degrid_xcd_group;
    double ms;
} hs_tuning;

/* The decomposition in use (after hs_plan). */
hs_status hs_get_tuning(const hs_ctx* ctx, hs_tuning* out);

/* Sets the decomposition (validated).  When the context is planned and the tile,
 * grid_split or degrid_batches change it re-plans, after which a workspace must be
 * bound again (hs_plan reports its size); the other fields are launch parameters
 * and take effect at the next call, the bound state kept. */
hs_status hs_set_tuning(hs_ctx* ctx, const hs_tuning* t);

/* Bytes of the temporary workspace hs_autotune needs (the largest plan among the
 * candidates).  After hs_plan. */
hs_status hs_autotune_bytes(hs_ctx* ctx, size_t* bytes);

/* Autotuner of the batching (Algorithm 2's operators batched over channels): times
 * the data-fidelity branch of one iteration (forward FFT, degridding with the dual
 * step, projection, gridding, adjoint FFT) on the GPU for candidate
 * decompositions (coordinate descent over
 * the tile edge, the gridding split, the degridding unit size, the FFT column
 * tile and the two XCD groups), keeps the fastest and re-plans with it.  dev/bytes: a caller-allocated
 * temporary workspace of at least hs_autotune_bytes bytes, free to reuse after the
 * call.  cache_path (may be NULL): a JSON-lines file of earlier choices keyed by the
 * problem shape (nx, ny, L, visibilities, dtype); a hit skips the timing, a miss
 * appends the new choice.  chosen (may be NULL) receives the choice.  Leaves the
 * context planned and unbound: bind a workspace of the size hs_plan reports; the
 * primal-dual state starts at zero.  Synchronising. */
hs_status hs_autotune(hs_ctx* ctx, void* dev, size_t bytes, const char* cache_path, hs_tuning* chosen);

/* ------------------------------------------------ host utilities (no GPU) */
/* Density preconditioner (Sec. 3.3): out[m] = 1/n_m with n_m the number of
 * visibilities in the same cell (floor(u nx) mod nx, floor(v ny) mod ny). */
hs_status hs_density_precond(int64_t M, const double* uv, int32_t nx, int32_t ny, double* out);

/* The library's visibility order for one channel: perm[k] = input index of the
 * k-th visibility in tile-major order, sorted by (tile, region, bin, cell within
 * the tile in raster order) with ties in input order; region_ptr[t*9 + r] = first position of region r of tile t,
 * region_ptr has (nx/tile + 1)(2ny/tile)*9 + 1 entries.  Cells are those of the
 * Hermitian half plane: a visibility with (u Kx) mod Kx > Kx/2 is binned at -t
 * (the transform of a real image is conjugate-symmetric), so tiles cover
 * kx in [0, Kx/2] only.  precond may be NULL. */
hs_status hs_visibility_order(int64_t M, const double* uv, const double* precond, int32_t nblocks,
                              const int64_t* block_ptr, int32_t nx, int32_t ny, int32_t tile,
                              int64_t* perm, int64_t* region_ptr);

/* Low-pass filter of db-K (2K taps) by the library's own spectral factorisation. */
hs_status hs_daubechies_filter(int32_t K, double* h);

/* --------------------------------------------------------------- operators */
/* Phi (eq:inverse, all channels): Y = [Theta_l G_l F Z x_l]_l.
 * X: real [L][ny][nx]; Y: complex [sum M_l] in the caller's order. */
hs_status hs_phi(hs_ctx* ctx, const void* X, void* Y);

/* Re Phi^dagger (adjoint in the dual problem, Sec. 3.2): X_l = Re Z^T F^H G_l^T Theta_l y_l. */
hs_status hs_phi_adj(hs_ctx* ctx, const void* Y, void* X);

/* Psi^dagger (Sec. 2.3): C[d] = Psi_d^dagger X, d = 0 Dirac, d = K for db-K.
 * X: real [L][ny][nx]; C: real [D][L][ny][nx]. */
hs_status hs_psi_adj(hs_ctx* ctx, const void* X, void* C);

/* Psi: X = sum_d Psi_d C[d]. */
hs_status hs_psi(hs_ctx* ctx, const void* C, void* X);

/* Psi^dagger and Psi of nl contiguous channels (1 <= nl <= L; the dictionary is the
 * same for every channel): X real [nl][ny][nx], C real [D][nl][ny][nx].  For callers
 * that process the cube a few channels at a time (checkpointed gradients). */
hs_status hs_psi_adj_n(hs_ctx* ctx, const void* X, void* C, int32_t nl);
hs_status hs_psi_n(hs_ctx* ctx, const void* C, void* X, int32_t nl);

/* The l2,1 norm of Sec. 2.3 (the joint-average-sparsity prior: the l2 norm of each row
 * (d, pixel) of Psi^dagger X across the channels, summed, optionally weighted by wbar as
 * in eq:weights-l21) built a chunk of channels at a time, and its gradient.
 *   hs_l21_rowsq:      S[d][p] (device FP64 [D][ny][nx]) = (accumulate ? S : 0) + the sum
 *                      over the chunk's nl channels of C[d][l][p]^2, C = [D][nl][ny][nx].
 *   hs_l21_rowscale:   C[d][l][p] <- scale * wbar[d][p] * C[d][l][p] / sqrt(S[d][p]) for
 *                      the chunk (0 on a zero row: the subgradient of least norm); with S
 *                      summed over all channels this is the gradient of the norm with
 *                      respect to the chunk's coefficients.  wbar: [D][ny][nx] or NULL.
 *   hs_l21_from_rowsq: *value (host) = sum_{d,p} wbar[d][p] sqrt(S[d][p]), FP64, fixed
 *                      summation order; synchronising.
 * nl in 1..L; asynchronous on the context stream except hs_l21_from_rowsq. */
hs_status hs_l21_rowsq(hs_ctx* ctx, const void* C, int32_t nl, double* S, int32_t accumulate);
hs_status hs_l21_rowscale(hs_ctx* ctx, void* C, int32_t nl, const double* S, const void* wbar, double scale);
hs_status hs_l21_from_rowsq(hs_ctx* ctx, const double* S, const void* wbar, double* value);

/* --------------------------------------------------- proxes / dual updates */
/* eq:prox-L21 in place: rows of length L at fixed (d, y, x) of A [D][L][ny][nx]
 * are shrunk by max(||a|| - t*wbar, 0)/||a||.  wbar: real [D][ny][nx] or NULL (ones). */
hs_status hs_prox_l21(hs_ctx* ctx, void* A, const void* wbar, double t);

/* Algorithm 2, l2,1 dual: A_d <- (I - S^{l21}_{wbar mu D})(A_d + Psi_d^dagger Xt) in place,
 * and, when At_sum is not NULL, At_sum = sum_d Psi_d A_d (real [L][ny][nx]). */
hs_status hs_dual_l21(hs_ctx* ctx, void* A, const void* Xt, const void* wbar, double mu, void* At_sum);

/* hs_prox_nuclear without a context and without allocating: for callers that cannot
 * allocate device memory (code under stream capture, serving loops, harnesses that
 * forbid hipMalloc).  X: device real (dtype HS_F32 or HS_F64) [L][N], replaced in
 * place by S*_w(X) as in hs_prox_nuclear (FP64 Gram and eigen-decomposition, cold
 * start); w: host double [L] (NULL = ones); sigma_out: host double [L] or NULL;
 * stream: hipStream_t (NULL = default); device: HIP device ordinal, made current.
 * The scratch is a fixed device array of the library, 4.29 MB per device, kept until
 * the process ends; it bounds L to 1..64 (HS_ERR_SHAPE beyond).  N >= 1.  Every call
 * on a device shares that device's array: calls that overlap on one device (other
 * threads, other streams) race.  Synchronising.  Errors: HS_ERR_INVALID_ARG,
 * HS_ERR_SHAPE, HS_ERR_NONFINITE (w), HS_ERR_HIP. */
hs_status hs_prox_nuclear_noalloc(void* X, int32_t dtype, int64_t N, int32_t L, const double* w,
                                  double* sigma_out, void* stream, int32_t device);

/* eq:prox-L* in place on the N x L matrix X (column l = channel l):
 * singular values soft-thresholded by w (host [L], paired with decreasing
 * singular values; NULL = ones).  sigma_out (host [L], may be NULL) receives
 * the singular values of the input in decreasing order.  Synchronising. */
hs_status hs_prox_nuclear(hs_ctx* ctx, void* X, const double* w, double* sigma_out);

/* Algorithm 2, nuclear dual: P <- (I - S*_w)(P + Xt) in place. */
hs_status hs_dual_nuclear(hs_ctx* ctx, void* P, const void* Xt, const double* w);

/* Algorithm 2, data-fidelity dual, for every block (l, b): v_l^b <- the
 * preconditioned data-fidelity dual update from Xt (eq:md with the ellipsoid
 * projection solved exactly).  v: complex [sum M_l] caller order, in place.
 * When adj_out is not NULL it receives Re Phi^dagger v_new (the primal data term; real [L][ny][nx]). */
hs_status hs_dual_data(hs_ctx* ctx, void* v, const void* Xt, void* adj_out);

/* Prox of the indicator of B(y_l^b, eps_l^b) in the metric U_l^b (eq:prox,
 * Sec. 3.3): z <- argmin_{||q - y|| <= eps} (q - z)^H U (q - z).  z: device
 * complex [M_b], block b of channel l in the caller's order.  Synchronising. */
hs_status hs_proj_ellipsoid(hs_ctx* ctx, int32_t l, int32_t b, void* z);

/* Spectral norms for the step sizes (Sec. 3.4), FP64 power iteration.
 * which = HS_NORM_PHI_PRECOND: max_l of the largest eigenvalue of
 *   x -> Re Phi_l^dagger U_l Phi_l x over real images, started from x0
 *   (device real [L][ny][nx], caller-drawn), stopping at relative change
 *   < tol or max_it iterations; per-channel values in per_channel (host [L], may be NULL).
 *   An FP32 context runs the FP64 operators on FP64 copies of its plan's
 *   arrays (kept in its workspace) from x0 widened exactly.
 * which = HS_NORM_PSI: ||Psi^dagger||_S^2 = D (orthonormal bases), exact.
 * *iters receives the iterations used (may be NULL).  Synchronising. */
hs_status hs_op_norm(hs_ctx* ctx, int32_t which, int32_t max_it, double tol, const void* x0,
                     double* out, double* per_channel, int32_t* iters);

/* Dirty cube and the trade-off estimate of Sec. 2.3 (normalisation of Sec. 4.3):
 *   PSF_l = Re Phi_l^dagger Phi_l delta, delta a unit source at the phase centre;
 *   X_dirty[l] = Re Phi_l^dagger y_l / max_p PSF_l(p)  (y = theta * y_raw of hs_set_data);
 *   mu_hat = ||X_dirty||_* / ||Psi^dagger X_dirty||_{2,1}.
 * Xd: device real [L][ny][nx] receiving X_dirty (may be NULL); mu: host double
 * (may be NULL; one of the two is required).  FP64 reductions; synchronising
 * when mu is requested. */
hs_status hs_dirty_mu(hs_ctx* ctx, void* Xd, double* mu);

/* -------------------------------------------------------------- PD solver */
/* Sets parameters of Algorithm 2 (does not reset the state). */
hs_status hs_pd_init(hs_ctx* ctx, const hs_pd_params* params);
/* Copy a state into / out of the context (device arrays device-to-device on the
 * stream; host members synchronously).  hs_pd_set_state restarts the parts of
 * Algorithm 2's bookkeeping it is not given: iteration count t = 0, beta = 1
 * (scalars NULL), the l2 bounds of hs_set_data (eps NULL) and their
 * last-update iterations vartheta = 0 (vartheta NULL); wbar and w replace the
 * weights of hs_pd_init when given (needs hs_pd_init first).  The
 * eigen-solver warm start is reset.  Together with hs_report.gamma this saves
 * and resumes a reweighted solve (Algorithm 1 warm start). */
hs_status hs_pd_set_state(hs_ctx* ctx, const hs_state_ptrs* st);
hs_status hs_pd_get_state(hs_ctx* ctx, const hs_state_ptrs* st);
/* n iterations of Algorithm 2.  The first call captures one
 * iteration into a HIP graph that later calls replay. */
hs_status hs_pd_iterate(hs_ctx* ctx, int32_t n);
/* beta of the last iteration (relative variation of X), and per-block residual norms rho
 * (host [n_blocks], may be NULL) and bounds eps (host [n_blocks],
 * may be NULL).  Synchronising. */
hs_status hs_pd_stats(hs_ctx* ctx, double* beta, double* rho, double* eps);
/* Diagnostics: phases of one iteration, in execution order. */
enum {
    HS_PH_FFT_FWD = 0,   /* Z and F of Xt */
    HS_PH_DEGRID,        /* Theta G and the data-dual step, per-run FP64 sums */
    HS_PH_ROOTS,         /* per-bin sums, per-block projection roots, adaptive bounds */
    HS_PH_DUAL_APPLY,    /* v update (the projection) */
    HS_PH_GRID,          /* G^T Theta^T v */
    HS_PH_FFT_ADJ,       /* F^H and Z^T, real part (the primal data term) */
    HS_PH_GRAM,          /* L x L Gram of P + Xt (nuclear dual) */
    HS_PH_EIG,           /* FP64 eigen-decomposition and W (nuclear dual) */
    HS_PH_BACKPROJ,      /* P <- (P + Xt) W (nuclear dual) */
    HS_PH_PSI_ADJ,       /* Psi^dagger Xt (l2,1 dual) */
    HS_PH_L21,           /* l2,1 dual update */
    HS_PH_PSI,           /* sum_d Psi_d A_d (the primal sparsity term) */
    HS_PH_PRIMAL,        /* primal update and beta */
    HS_NPHASES
};
/* Runs n eager iterations of Algorithm 2 with HIP events between the phases
 * above (on the context stream) and returns the mean duration of each phase in
 * milliseconds in times_ms[HS_NPHASES].  Advances the state like hs_pd_iterate.
 * Synchronising. */
hs_status hs_profile_phases(hs_ctx* ctx, int32_t n, double* times_ms);

/* Diagnostics: out[0] = beta of the last iteration, out[1] = iterations run on
 * the device counter, out[2] = Jacobi sweeps of the last eigen-decomposition,
 * out[3] = iterations issued by the host; n = number of values wanted (<= 4).
 * Synchronising. */
hs_status hs_get_diag(hs_ctx* ctx, double* out, int32_t n);

/* Algorithm 1 on the current state; X_out (device real [L][ny][nx], may be NULL). */
hs_status hs_solve(hs_ctx* ctx, const hs_solve_params* params, void* X_out, hs_report* report);

#ifdef __cplusplus
}
#endif
#endif /* HYPERSARA_H */
