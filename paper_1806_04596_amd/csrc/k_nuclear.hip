// Nuclear-norm proximity operator through the L x L Gram matrix (eq:prox-L*,
// Algorithm 2, nuclear-norm dual).
//
//  * Gram C = Z^T Z of the N x L matrix Z (= P + Xt, column l = channel l): FP64
//    MFMA (v_mfma_f64_16x16x4f64) on 64-pixel slabs staged in LDS; inputs in the
//    working precision are widened exactly, so C is the FP64 Gram of Z.  Split-K
//    partials are summed in fixed order (deterministic).
//  * Eigen-decomposition of C: cyclic parallel Jacobi in FP64 inside one
//    workgroup (round-robin pairing, L/2 disjoint rotations per round), warm
//    started from the previous eigenvectors when the Gram changes little.
//  * W = V diag(f(sigma)) V^T with sigma_j = sqrt(lambda_j) sorted in decreasing
//    order and f = min(1, w_j/sigma_j) (dual form I - S*_w) or 1 - that (prox).
//  * Back-projection out = Z W (every pixel's length-L row times W).
#include <algorithm>
#include <cmath>
#include <mutex>

#include "hs_internal.h"

namespace hs {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int GR_SLAB = 64;   // pixels per LDS slab

template <typename T, bool HAS2>
__global__ __launch_bounds__(256) void k_gram(const T* __restrict__ P, const T* __restrict__ Xt,
                                              double* __restrict__ part, int L, int64_t N, int64_t chunk) {
    __shared__ double S[MAX_L][GR_SLAB + 2];
    constexpr int PER = MAX_L * GR_SLAB / 256;   // staged values per thread and slab
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t p_begin = (int64_t)blockIdx.x * chunk;
    const int64_t p_end = min(N, p_begin + chunk);
    double4_t acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = double4_t{0.0, 0.0, 0.0, 0.0};
    // slab values for this thread: channel e / GR_SLAB, pixel e mod GR_SLAB, e = tid + 256 k;
    // the next slab is loaded into registers while the current one is multiplied.
    // Loads are unconditional (clamped indices, padding zeroed after the load) so
    // that they are all in flight together.
    T nv[PER], nv2[PER];
    bool nin[PER];
    auto load = [&](int64_t p0) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + 256 * k;
            const int ch = e / GR_SLAB, pp = e - ch * GR_SLAB;
            const int64_t pix = p0 + pp;
            nin[k] = ch < L && pix < p_end;
            const size_t idx = (size_t)min(ch, L - 1) * N + (size_t)min(pix, p_end - 1);
            nv[k] = P[idx];
            if (HAS2) nv2[k] = Xt[idx];
        }
    };
    load(p_begin);
    for (int64_t p0 = p_begin; p0 < p_end; p0 += GR_SLAB) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + 256 * k;
            const int ch = e / GR_SLAB, pp = e - ch * GR_SLAB;
            T z = nv[k];
            if (HAS2) z += nv2[k];
            S[ch][pp] = nin[k] ? (double)z : 0.0;
        }
        __syncthreads();
        if (p0 + GR_SLAB < p_end) load(p0 + GR_SLAB);
        const int i = lane & 15, kq = lane >> 4;
#pragma unroll 4
        for (int kk = 0; kk < GR_SLAB; kk += 4) {
            const double a = S[wave * 16 + i][kk + kq];
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                const double b = S[jb * 16 + i][kk + kq];
                acc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[jb], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // D layout of the 16x16x4 f64 MFMA (checked on gfx950): lane holds column
    // (lane & 15) and rows (lane >> 4) + 4 r.
    double* out = part + (size_t)blockIdx.x * MAX_L * MAX_L;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = wave * 16 + (lane >> 4) + 4 * r;
            const int col = jb * 16 + (lane & 15);
            out[row * MAX_L + col] = acc[jb][r];
        }
    }
}

// Refinement Gram H = (Z V)^T (Z V) = V^T Z^T Z V for the eigenvectors V of a first
// eigen-decomposition (a Rayleigh-Ritz step): each 64-pixel slab S of Z (channels x
// pixels, widened exactly to FP64) is first turned into T = V^T S on the FP64 matrix
// cores, then T T^T is accumulated as in k_gram.  Entry (i, j) of H carries rounding
// of the order of eps sigma_i sigma_j instead of eps sigma_1^2, so the eigenvectors of
// H (nearly diagonal) refine those of the Gram matrix to the accuracy of a direct SVD.
// V: [MAX_L][MAX_L] row a = channel, column j = mode; rows and columns >= L are those
// of the identity, so the padded modes stay zero.
template <typename T, bool HAS2>
__global__ __launch_bounds__(256) void k_gram_rr(const T* __restrict__ P, const T* __restrict__ Xt,
                                                 const double* __restrict__ V, double* __restrict__ part, int L,
                                                 int64_t N, int64_t chunk) {
    __shared__ double S[MAX_L][GR_SLAB + 2];
    __shared__ double Tt[MAX_L][GR_SLAB + 2];
    constexpr int PER = MAX_L * GR_SLAB / 256;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int i = lane & 15, kq = lane >> 4;
    const int64_t p_begin = (int64_t)blockIdx.x * chunk;
    const int64_t p_end = min(N, p_begin + chunk);
    // A operand of T = V^T S for this wave's 16 modes: A[i][k] = V[4 st + k][16 wave + i]
    double va[MAX_L / 4];
#pragma unroll
    for (int st = 0; st < MAX_L / 4; ++st) va[st] = V[(4 * st + kq) * MAX_L + 16 * wave + i];
    double4_t acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = double4_t{0.0, 0.0, 0.0, 0.0};
    T nv[PER], nv2[PER];
    bool nin[PER];
    auto load = [&](int64_t p0) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + 256 * k;
            const int ch = e / GR_SLAB, pp = e - ch * GR_SLAB;
            const int64_t pix = p0 + pp;
            nin[k] = ch < L && pix < p_end;
            const size_t idx = (size_t)min(ch, L - 1) * N + (size_t)min(pix, p_end - 1);
            nv[k] = P[idx];
            if (HAS2) nv2[k] = Xt[idx];
        }
    };
    load(p_begin);
    for (int64_t p0 = p_begin; p0 < p_end; p0 += GR_SLAB) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + 256 * k;
            const int ch = e / GR_SLAB, pp = e - ch * GR_SLAB;
            T z = nv[k];
            if (HAS2) z += nv2[k];
            S[ch][pp] = nin[k] ? (double)z : 0.0;
        }
        __syncthreads();
        if (p0 + GR_SLAB < p_end) load(p0 + GR_SLAB);
        // T rows 16 wave .. + 15 (modes), all 64 pixel columns
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
            double4_t t = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int st = 0; st < MAX_L / 4; ++st)
                t = __builtin_amdgcn_mfma_f64_16x16x4f64(va[st], S[4 * st + kq][16 * jb + i], t, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) Tt[16 * wave + kq + 4 * r][16 * jb + i] = t[r];
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < GR_SLAB; kk += 4) {
            const double a = Tt[wave * 16 + i][kk + kq];
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                const double b = Tt[jb * 16 + i][kk + kq];
                acc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[jb], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    double* out = part + (size_t)blockIdx.x * MAX_L * MAX_L;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = wave * 16 + (lane >> 4) + 4 * r;
            const int col = jb * 16 + (lane & 15);
            out[row * MAX_L + col] = acc[jb][r];
        }
    }
}

// Gram partials in FP32 products (MODE 1) or BF16 split products (MODE 2) of an FP32
// Z = P + Xt, accumulated in FP32 over the work-group's pixels; the partials are
// summed in FP64 by k_gram_reduce.
//  MODE 1: v_mfma_f32_16x16x4f32, lane (i, kq) supplies Z[pixel kk + kq][channel i].
//  MODE 2: z = hi + lo with hi = bf16(z), lo = bf16(z - hi) (round to nearest even);
//          C ~ hi^T hi + hi^T lo + lo^T hi (lo^T lo, of relative size 2^-16, dropped)
//          on v_mfma_f32_16x16x16bf16_1k, lane (i, kq) supplying pixels kk + 4 kq .. + 3
//          of channel i for both operands (a Gram needs only that A and B index the
//          pixels alike).
// D layout of both (FP32 accumulators): lane holds column (lane & 15), rows 4 (lane >> 4) + r.
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne(float x) {
    const unsigned int b = __float_as_uint(x);
    return (unsigned short)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

__device__ __forceinline__ void bf16_split4(const float* z, bf16x4_t& hi, bf16x4_t& lo) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const unsigned short h = bf16_rne(z[j]);
        hi[j] = (short)h;
        lo[j] = (short)bf16_rne(z[j] - bf16_to_f32(h));
    }
}

template <int MODE, bool HAS2>
__global__ __launch_bounds__(256) void k_gram_lp(const float* __restrict__ P, const float* __restrict__ Xt,
                                                 double* __restrict__ part, int L, int64_t N, int64_t chunk) {
    __shared__ float S[MAX_L][GR_SLAB + 4];
    constexpr int PER = MAX_L * GR_SLAB / 256;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t p_begin = (int64_t)blockIdx.x * chunk;
    const int64_t p_end = min(N, p_begin + chunk);
    f32x4_t acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    float nv[PER], nv2[PER];
    bool nin[PER];
    auto load = [&](int64_t p0) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + 256 * k;
            const int ch = e / GR_SLAB, pp = e - ch * GR_SLAB;
            const int64_t pix = p0 + pp;
            nin[k] = ch < L && pix < p_end;
            const size_t idx = (size_t)min(ch, L - 1) * N + (size_t)min(pix, p_end - 1);
            nv[k] = P[idx];
            if (HAS2) nv2[k] = Xt[idx];
        }
    };
    load(p_begin);
    const int i = lane & 15, kq = lane >> 4;
    for (int64_t p0 = p_begin; p0 < p_end; p0 += GR_SLAB) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + 256 * k;
            const int ch = e / GR_SLAB, pp = e - ch * GR_SLAB;
            float z = nv[k];
            if (HAS2) z += nv2[k];
            S[ch][pp] = nin[k] ? z : 0.f;
        }
        __syncthreads();
        if (p0 + GR_SLAB < p_end) load(p0 + GR_SLAB);
        if constexpr (MODE == 1) {
#pragma unroll 4
            for (int kk = 0; kk < GR_SLAB; kk += 4) {
                const float a = S[wave * 16 + i][kk + kq];
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
                    acc[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, S[jb * 16 + i][kk + kq], acc[jb], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < GR_SLAB; kk += 16) {
                bf16x4_t ahi, alo;
                bf16_split4(&S[wave * 16 + i][kk + 4 * kq], ahi, alo);
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) {
                    bf16x4_t bhi, blo;
                    bf16_split4(&S[jb * 16 + i][kk + 4 * kq], bhi, blo);
                    acc[jb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi, acc[jb], 0, 0, 0);
                    acc[jb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, blo, acc[jb], 0, 0, 0);
                    acc[jb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bhi, acc[jb], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    double* out = part + (size_t)blockIdx.x * MAX_L * MAX_L;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = wave * 16 + 4 * (lane >> 4) + r;
            const int col = jb * 16 + (lane & 15);
            out[row * MAX_L + col] = (double)acc[jb][r];
        }
    }
}

// C[e] = sum of the partial Grams in a fixed order: 8 interleaved groups of
// partials (group g takes partials g, g + 8, ...), then a fixed combine.
constexpr int GRR_E = 32;   // Gram entries per reduction work-group
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ part, double* __restrict__ C,
                                                     int nparts) {
    __shared__ double sg[8][GRR_E];
    const int el = threadIdx.x % GRR_E, g = threadIdx.x / GRR_E;
    const int e = blockIdx.x * GRR_E + el;
    double a = 0.0;
    if (e < MAX_L * MAX_L) {
#pragma unroll 8
        for (int k = g; k < nparts; k += 8) a += part[(size_t)k * MAX_L * MAX_L + e];
    }
    sg[g][el] = a;
    __syncthreads();
    if (g == 0 && e < MAX_L * MAX_L)
        C[e] = ((sg[0][el] + sg[1][el]) + (sg[2][el] + sg[3][el])) + ((sg[4][el] + sg[5][el]) + (sg[6][el] + sg[7][el]));
}

// ------------------------------------------------------------------ Jacobi
// One workgroup of EIG_THREADS threads.  A (n x n, n = L rounded up to even) and V in LDS.
// mode 0: f = min(1, w/s) (I - S*_w); mode 1: f = 1 - min(1, w/s) (S*_w / X).
// warm: start from V = previous eigenvectors (A <- V^T C V).
// Vbase (may be null): Cg is Vbase^T C Vbase (a refinement Gram); the eigenvectors
// returned, stored and used for W are Vbase V.  Vbase may be Vg (it is read into LDS
// before Vg is written), so neither is restrict-qualified.
constexpr int EIG_THREADS = 1024;
template <typename TW>
__global__ __launch_bounds__(EIG_THREADS) void k_eig(const double* __restrict__ Cg, double* Vg,
                                             double* __restrict__ sig_out, const double* __restrict__ w,
                                             TW* __restrict__ Wout, int L, int mode, int warm,
                                             double* __restrict__ diag, const double* Vbase) {
    __shared__ double A[MAX_L][MAX_L + 1];
    __shared__ double V[MAX_L][MAX_L + 1];
    __shared__ double Tm[MAX_L][MAX_L + 1];
    __shared__ double cs[MAX_L / 2], sn[MAX_L / 2];
    __shared__ int pp[MAX_L / 2], qq[MAX_L / 2];
    __shared__ int rotated;
    __shared__ double lam[MAX_L], fac[MAX_L];
    __shared__ int ord[MAX_L];
    const int tid = threadIdx.x;
    const int n = L + (L & 1);
    // load
    for (int e = tid; e < n * n; e += EIG_THREADS) {
        const int i = e / n, j = e - i * n;
        A[i][j] = (i < L && j < L) ? Cg[i * MAX_L + j] : 0.0;
        V[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (warm) {
        // V <- previous eigenvectors, A <- V^T C V
        for (int e = tid; e < n * n; e += EIG_THREADS) {
            const int i = e / n, j = e - i * n;
            V[i][j] = Vg[i * MAX_L + j];
        }
        __syncthreads();
        for (int e = tid; e < n * n; e += EIG_THREADS) {   // Tm = C V
            const int i = e / n, j = e - i * n;
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += A[i][k] * V[k][j];
            Tm[i][j] = s;
        }
        __syncthreads();
        for (int e = tid; e < n * n; e += EIG_THREADS) {   // A = V^T Tm
            const int i = e / n, j = e - i * n;
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += V[k][i] * Tm[k][j];
            A[i][j] = s;
        }
        __syncthreads();
        for (int e = tid; e < n * n; e += EIG_THREADS) {   // symmetrise through Tm
            const int i = e / n, j = e - i * n;
            Tm[i][j] = 0.5 * (A[i][j] + A[j][i]);
        }
        __syncthreads();
        for (int e = tid; e < n * n; e += EIG_THREADS) {
            const int i = e / n, j = e - i * n;
            A[i][j] = Tm[i][j];
        }
        __syncthreads();
    }
    __shared__ double tr_sh;
    __shared__ int sweeps_done;
    if (tid == 0) {
        double tr = 0.0;
        for (int i = 0; i < n; ++i) tr += fabs(A[i][i]);
        tr_sh = tr;
    }
    __syncthreads();
    // rotations below this size are rounding noise (rank-deficient Grams have
    // near-zero diagonals where a purely relative test never stops)
    const double floor_abs = 1e-18 * tr_sh;
    const int half = n / 2;
    __shared__ double maxrel_sh[MAX_L / 2];
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (tid == 0) rotated = 0;
        double sweep_max = 0.0;   // largest |a_pq| / sqrt(a_pp a_qq) rotated in this sweep (thread < half)
        __syncthreads();
        for (int round = 0; round < n - 1; ++round) {
            if (tid < half) {
                // round-robin pairing: player 0 fixed, players 1..n-1 rotate
                int p, q;
                if (tid == 0) {
                    p = 0;
                    q = 1 + (round % (n - 1));
                } else {
                    p = 1 + ((tid + round) % (n - 1));
                    q = 1 + ((n - 1 - tid + round) % (n - 1));
                }
                if (p > q) { const int t = p; p = q; q = t; }
                const double apq = A[p][q], app = A[p][p], aqq = A[q][q];
                const double den = sqrt(fabs(app * aqq));
                double c = 1.0, s = 0.0;
                if (fabs(apq) > floor_abs && fabs(apq) > 1e-15 * den) {
                    const double th = (aqq - app) / (2.0 * apq);
                    const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                    c = 1.0 / sqrt(t * t + 1.0);
                    s = t * c;
                    rotated = 1;
                    sweep_max = fmax(sweep_max, den > 0.0 ? fabs(apq) / den : 1.0);
                }
                cs[tid] = c; sn[tid] = s; pp[tid] = p; qq[tid] = q;
            }
            __syncthreads();
            // A <- J^T A J as independent 2x2 blocks B(k, m) <- R_k^T B R_m, and V <- V J;
            // every entry is read and written by one thread (no intermediate barrier)
            for (int e = tid; e < half * half + half * n; e += EIG_THREADS) {
                if (e < half * half) {
                    const int k = e / half, m = e - k * half;
                    const int pk = pp[k], qk = qq[k], pm = pp[m], qm = qq[m];
                    const double ck = cs[k], sk = sn[k], cm = cs[m], sm = sn[m];
                    const double b00 = A[pk][pm], b01 = A[pk][qm], b10 = A[qk][pm], b11 = A[qk][qm];
                    // columns (right multiply by R_m)
                    const double c00 = cm * b00 - sm * b01, c01 = sm * b00 + cm * b01;
                    const double c10 = cm * b10 - sm * b11, c11 = sm * b10 + cm * b11;
                    // rows (left multiply by R_k^T)
                    double d00 = ck * c00 - sk * c10, d01 = ck * c01 - sk * c11;
                    double d10 = sk * c00 + ck * c10, d11 = sk * c01 + ck * c11;
                    if (k == m && sk != 0.0) { d01 = 0.0; d10 = 0.0; }   // the rotated pair is exactly zeroed
                    A[pk][pm] = d00; A[pk][qm] = d01; A[qk][pm] = d10; A[qk][qm] = d11;
                } else {
                    const int f = e - half * half;
                    const int m = f / n, i = f - m * n;
                    const int pm = pp[m], qm = qq[m];
                    const double cm = cs[m], sm = sn[m];
                    const double vip = V[i][pm], viq = V[i][qm];
                    V[i][pm] = cm * vip - sm * viq;
                    V[i][qm] = sm * vip + cm * viq;
                }
            }
            __syncthreads();
        }
        if (tid < half) maxrel_sh[tid] = sweep_max;
        const int any = rotated;   // every thread reads before anyone resets it
        __syncthreads();
        double mr = 0.0;
        for (int k = 0; k < half; ++k) mr = fmax(mr, maxrel_sh[k]);
        __syncthreads();
        if (tid == 0) sweeps_done = sweep + 1;
        // Jacobi converges quadratically: after a sweep whose rotations were all
        // below 1e-8 (relative) the off-diagonal left is of order 1e-16 of the
        // diagonal.  The FP32 contexts (prox output rounded to FP32) stop at 1e-6,
        // which leaves an off-diagonal of order 1e-12.
        if (!any || mr < (sizeof(TW) == 4 ? 1e-6 : 1e-8)) break;
    }
    if (tid == 0 && diag) diag[0] = (double)sweeps_done;
    // sort eigenvalues in decreasing order (rank by comparison, ties by index)
    if (tid < n) lam[tid] = A[tid][tid];
    __syncthreads();
    if (Vbase) {
        // refinement: the eigenvectors of C are Vbase V (this call decomposed Vbase^T C Vbase)
        for (int e = tid; e < n * n; e += EIG_THREADS) {
            const int i = e / n, j = e - i * n;
            Tm[i][j] = Vbase[i * MAX_L + j];
        }
        __syncthreads();
        for (int e = tid; e < n * n; e += EIG_THREADS) {
            const int i = e / n, j = e - i * n;
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += Tm[i][k] * V[k][j];
            A[i][j] = acc;
        }
        __syncthreads();
        for (int e = tid; e < n * n; e += EIG_THREADS) {
            const int i = e / n, j = e - i * n;
            V[i][j] = A[i][j];
        }
        __syncthreads();
    }
    if (tid < L) {
        int rank = 0;
        const double li = lam[tid];
        for (int j = 0; j < L; ++j) {
            const double lj = lam[j];
            rank += (lj > li || (lj == li && j < tid)) ? 1 : 0;
        }
        ord[rank] = tid;
    }
    __syncthreads();
    if (tid < L) {
        const int src = ord[tid];
        const double sg = sqrt(fmax(lam[src], 0.0));
        const double wj = w[tid];
        double f = (sg > 0.0) ? fmin(1.0, wj / sg) : 1.0;
        if (mode == 1) f = 1.0 - f;
        fac[src] = f;
        sig_out[tid] = sg;
    }
    __syncthreads();
    // store eigenvectors for the next warm start
    for (int e = tid; e < MAX_L * MAX_L; e += EIG_THREADS) {
        const int i = e / MAX_L, j = e - i * MAX_L;
        Vg[e] = (i < n && j < n) ? V[i][j] : ((i == j) ? 1.0 : 0.0);
    }
    // W[a][b] = sum_j V[a][j] f_j V[b][j]
    for (int e = tid; e < MAX_L * MAX_L; e += EIG_THREADS) {
        const int a = e / MAX_L, b = e - a * MAX_L;
        double s = 0.0;
        if (a < L && b < L)
            for (int j = 0; j < L; ++j) s += V[a][j] * fac[j] * V[b][j];
        Wout[e] = (TW)s;
    }
}

typedef float float4_t __attribute__((ext_vector_type(4)));
template <typename T> struct Acc16;
template <> struct Acc16<float> { typedef float4_t type; };
template <> struct Acc16<double> { typedef double4_t type; };
__device__ __forceinline__ float4_t mfma16x16x4(float a, float b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ double4_t mfma16x16x4(double a, double b, double4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Row of the 16 x 16 result held in element r of this lane (its column is
// lane & 15): f32 puts rows 4 (lane >> 4) + r in a lane, f64 rows (lane >> 4) + 4 r.
template <typename T>
__device__ __forceinline__ int mfma16_row(int lane, int r) {
    return sizeof(T) == 4 ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r;
}

// out[b][p] = sum_a W[a][b] Z[a][p], Z = in1 + in2 (in2 may be null): the
// product W^T Z on the matrix cores.  A wave owns 16-pixel column tiles of Z;
// its W^T fragments (b = 16 bb + (lane & 15), a = 4 s + (lane >> 4)) stay in
// registers for all its tiles, Z fragments come straight from memory (the next
// tile's while the current one is multiplied).  W is zero beyond L, so padded
// channels (clamped loads of channel L - 1) add nothing.  out may alias in1: a
// wave reads every channel of a tile before writing it.
constexpr int BP_WAVES = 2048;
template <typename T, bool HAS2>
__global__ __launch_bounds__(256) void k_backproject(const T* in1, const T* __restrict__ in2,
                                                     const T* __restrict__ Wg, T* out, int L, int64_t N) {
    typedef typename Acc16<T>::type acc_t;
    constexpr bool PREF = sizeof(T) == 4;          // register budget allows prefetch in FP32
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * 4 + (threadIdx.x >> 6), nw = gridDim.x * 4;
    const int il = lane & 15, kq = lane >> 4;
    T A[4][MAX_L / 4];
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
        for (int st = 0; st < MAX_L / 4; ++st) A[bb][st] = Wg[(4 * st + kq) * MAX_L + 16 * bb + il];
    const int64_t nt = (N + 15) / 16;
    T B[MAX_L / 4], B2[MAX_L / 4];
    auto load = [&](int64_t t) {
        const int64_t p = t * 16 + il;
        const int64_t pc = p < N ? p : N - 1;
#pragma unroll
        for (int st = 0; st < MAX_L / 4; ++st) {
            const int a = 4 * st + kq;
            const size_t idx = (size_t)(a < L ? a : L - 1) * N + (size_t)pc;
            B[st] = in1[idx];
            if (HAS2) B2[st] = in2[idx];
        }
    };
    if (gw < nt) load(gw);
    for (int64_t t = gw; t < nt; t += nw) {
        T Z[MAX_L / 4];
#pragma unroll
        for (int st = 0; st < MAX_L / 4; ++st) Z[st] = HAS2 ? B[st] + B2[st] : B[st];
        if (PREF && t + nw < nt) load(t + nw);
        acc_t acc[4];
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) acc[bb] = acc_t{};
#pragma unroll
        for (int st = 0; st < MAX_L / 4; ++st)
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) acc[bb] = mfma16x16x4(A[bb][st], Z[st], acc[bb]);
        const int64_t p = t * 16 + il;
        if (p < N) {
#pragma unroll
            for (int bb = 0; bb < 4; ++bb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int b = 16 * bb + mfma16_row<T>(lane, r);
                    if (b < L) out[(size_t)b * N + p] = acc[bb][r];
                }
        }
        if (!PREF && t + nw < nt) load(t + nw);
    }
}

__global__ void k_eye(double* V) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < MAX_L * MAX_L) V[e] = ((e / MAX_L) == (e % MAX_L)) ? 1.0 : 0.0;
}

// Forget the eigenvector warm start (next eigen-decomposition starts from I).
void launch_eig_reset(hs_ctx* c) { k_eye<<<(MAX_L * MAX_L + 255) / 256, 256, 0, c->stream>>>(c->d.eigV); }

template <typename T>
static void gram_lp(hs_ctx*, const T*, const T*, int64_t, int, int) {}   // FP64 contexts: FP64 Gram only
template <>
void gram_lp<float>(hs_ctx* c, const float* P, const float* Xt, int64_t chunk, int nparts, int mode) {
    if (mode == HS_GRAM_F32) {
        if (Xt) k_gram_lp<1, true><<<nparts, 256, 0, c->stream>>>(P, Xt, c->d.gram_part, c->L, c->N, chunk);
        else k_gram_lp<1, false><<<nparts, 256, 0, c->stream>>>(P, Xt, c->d.gram_part, c->L, c->N, chunk);
    } else {
        if (Xt) k_gram_lp<2, true><<<nparts, 256, 0, c->stream>>>(P, Xt, c->d.gram_part, c->L, c->N, chunk);
        else k_gram_lp<2, false><<<nparts, 256, 0, c->stream>>>(P, Xt, c->d.gram_part, c->L, c->N, chunk);
    }
}

template <typename T>
void launch_gram(hs_ctx* c, const T* P, const T* Xt, bool force64) {
    int64_t chunk = (c->N + NGRAM - 1) / NGRAM;
    chunk = (chunk + GR_SLAB - 1) / GR_SLAB * GR_SLAB;
    const int nparts = (int)((c->N + chunk - 1) / chunk);
    const int mode = force64 ? HS_GRAM_F64 : c->gram_mode;
    if (mode != HS_GRAM_F64 && sizeof(T) == 4) gram_lp<T>(c, P, Xt, chunk, nparts, mode);
    else if (Xt) k_gram<T, true><<<nparts, 256, 0, c->stream>>>(P, Xt, c->d.gram_part, c->L, c->N, chunk);
    else k_gram<T, false><<<nparts, 256, 0, c->stream>>>(P, Xt, c->d.gram_part, c->L, c->N, chunk);
    k_gram_reduce<<<(MAX_L * MAX_L + GRR_E - 1) / GRR_E, 256, 0, c->stream>>>(c->d.gram_part, c->d.gram, nparts);
}

static void eig_call(hs_ctx* c, int mode, int warm, double* diag, const double* vbase) {
    if (c->dtype == HS_F32)
        k_eig<float><<<1, EIG_THREADS, 0, c->stream>>>(c->d.gram, c->d.eigV, c->d.eig_sig, c->d.w_nuc,
                                                       (float*)c->d.Wmat, c->L, mode, warm, diag, vbase);
    else
        k_eig<double><<<1, EIG_THREADS, 0, c->stream>>>(c->d.gram, c->d.eigV, c->d.eig_sig, c->d.w_nuc,
                                                        (double*)c->d.Wmat, c->L, mode, warm, diag, vbase);
}

void launch_eig(hs_ctx* c, int mode) {
    // eigV starts as the identity, so the first call is a cold start
    eig_call(c, mode, 1, c->d.scal + 8, nullptr);
}

// The Rayleigh-Ritz refinement of the eigen-decomposition just computed (eigV): the
// Gram of Z V in FP64 (k_gram_rr), decomposed from the identity, the eigenvectors
// composed with V.  W, sigma and the stored eigenvectors are those of the refinement.
template <typename T>
void launch_eig_refine(hs_ctx* c, const T* P, const T* Xt, int mode) {
    int64_t chunk = (c->N + NGRAM - 1) / NGRAM;
    chunk = (chunk + GR_SLAB - 1) / GR_SLAB * GR_SLAB;
    const int nparts = (int)((c->N + chunk - 1) / chunk);
    if (Xt) k_gram_rr<T, true><<<nparts, 256, 0, c->stream>>>(P, Xt, c->d.eigV, c->d.gram_part, c->L, c->N, chunk);
    else k_gram_rr<T, false><<<nparts, 256, 0, c->stream>>>(P, Xt, c->d.eigV, c->d.gram_part, c->L, c->N, chunk);
    k_gram_reduce<<<(MAX_L * MAX_L + GRR_E - 1) / GRR_E, 256, 0, c->stream>>>(c->d.gram_part, c->d.gram, nparts);
    eig_call(c, mode, 0, nullptr, c->d.eigV);
}

bool eig_refined(const hs_ctx* c, bool force64) {
    return c->dtype == HS_F64 || (!force64 && c->gram_mode == HS_GRAM_BF16_SPLIT);
}

template <typename T>
void launch_backproject(hs_ctx* c, T* out, const T* in1, const T* in2) {
    const int64_t nt = (c->N + 15) / 16;
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(BP_WAVES, nt) / 4);
    if (in2) k_backproject<T, true><<<nb, 256, 0, c->stream>>>(in1, in2, (const T*)c->d.Wmat, out, c->L, c->N);
    else k_backproject<T, false><<<nb, 256, 0, c->stream>>>(in1, in2, (const T*)c->d.Wmat, out, c->L, c->N);
}

template void launch_eig_refine<float>(hs_ctx*, const float*, const float*, int);
template void launch_eig_refine<double>(hs_ctx*, const double*, const double*, int);
template void launch_gram<float>(hs_ctx*, const float*, const float*, bool);
template void launch_gram<double>(hs_ctx*, const double*, const double*, bool);
template void launch_backproject<float>(hs_ctx*, float*, const float*, const float*);
template void launch_backproject<double>(hs_ctx*, double*, const double*, const double*);

}  // namespace hs

// ------------------------------------------------ nuclear prox without allocation
// hs_prox_nuclear_noalloc: the nuclear-norm prox of hs_prox_nuclear for callers that
// cannot allocate device memory.  Its scratch (Gram partials, the Gram matrix, the
// eigenvectors and values, the weights and W) is the file-scope device array below,
// one copy per device, held until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.
namespace hs {

constexpr int NA_PARTS = 128;                       // Gram partials (split over pixels)
constexpr size_t NA_MAT = (size_t)MAX_L * MAX_L;    // one 64 x 64 matrix
// doubles: partials, C, V, W, sigma, w
constexpr size_t NA_DOUBLES = NA_PARTS * NA_MAT + 3 * NA_MAT + 2 * MAX_L;
constexpr size_t NA_SCRATCH_BYTES = NA_DOUBLES * sizeof(double);   // 4.29 MB

__device__ __align__(256) double scratch[NA_DOUBLES];

struct NAWeights {
    double w[MAX_L];
};

__global__ void k_na_set_w(NAWeights w, double* dst) {
    const int j = threadIdx.x;
    if (j < MAX_L) dst[j] = w.w[j];
}

static double* na_scratch_ptr(int device, std::string& err) {
    static std::mutex mu;
    static void* ptr[64] = {};
    std::lock_guard<std::mutex> lk(mu);
    if (device < 0 || device >= 64) {
        err = "device ordinal out of range";
        return nullptr;
    }
    if (!ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
            return nullptr;
        }
        ptr[device] = p;
    }
    return (double*)ptr[device];
}

template <typename T>
static void na_launch(double* base, T* X, int64_t N, int L, hipStream_t st) {
    double* part = base;
    double* C = part + NA_PARTS * NA_MAT;
    double* V = C + NA_MAT;
    double* Wm = V + NA_MAT;
    double* sig = Wm + NA_MAT;
    double* w = sig + MAX_L;
    int64_t chunk = (N + NA_PARTS - 1) / NA_PARTS;
    chunk = (chunk + GR_SLAB - 1) / GR_SLAB * GR_SLAB;
    const int nparts = (int)((N + chunk - 1) / chunk);
    k_gram<T, false><<<nparts, 256, 0, st>>>(X, nullptr, part, L, N, chunk);
    k_gram_reduce<<<(MAX_L * MAX_L + GRR_E - 1) / GRR_E, 256, 0, st>>>(part, C, nparts);
    k_eig<T><<<1, EIG_THREADS, 0, st>>>(C, V, sig, w, (T*)Wm, L, 1, 0, nullptr, nullptr);
    if (sizeof(T) == 8) {   // FP64: the Rayleigh-Ritz refinement, as in an FP64 context
        k_gram_rr<T, false><<<nparts, 256, 0, st>>>(X, nullptr, V, part, L, N, chunk);
        k_gram_reduce<<<(MAX_L * MAX_L + GRR_E - 1) / GRR_E, 256, 0, st>>>(part, C, nparts);
        k_eig<T><<<1, EIG_THREADS, 0, st>>>(C, V, sig, w, (T*)Wm, L, 1, 0, nullptr, V);
    }
    const int64_t nt = (N + 15) / 16;
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(BP_WAVES, nt) / 4);
    k_backproject<T, false><<<nb, 256, 0, st>>>(X, nullptr, (const T*)Wm, X, L, N);
}

}  // namespace hs

extern "C" hs_status hs_prox_nuclear_noalloc(void* X, int32_t dtype, int64_t N, int32_t L, const double* w,
                                             double* sigma_out, void* stream, int32_t device) {
    using namespace hs;
    static thread_local std::string err;
    if (!X || (dtype != HS_F32 && dtype != HS_F64) || N < 1) return HS_ERR_INVALID_ARG;
    if (L < 1 || L > MAX_L) return HS_ERR_SHAPE;   // the scratch holds 64 x 64 matrices
    NAWeights wv;
    for (int j = 0; j < MAX_L; ++j) wv.w[j] = 1.0;
    if (w)
        for (int j = 0; j < L; ++j) {
            if (!std::isfinite(w[j]) || w[j] < 0) return HS_ERR_NONFINITE;
            wv.w[j] = w[j];
        }
    if (hipSetDevice(device) != hipSuccess) return HS_ERR_HIP;
    double* base = na_scratch_ptr(device, err);
    if (!base) return HS_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    double* sig = base + NA_PARTS * NA_MAT + 3 * NA_MAT;
    k_na_set_w<<<1, MAX_L, 0, st>>>(wv, sig + MAX_L);
    if (dtype == HS_F32) na_launch<float>(base, (float*)X, N, L, st);
    else na_launch<double>(base, (double*)X, N, L, st);
    if (hipGetLastError() != hipSuccess) return HS_ERR_HIP;
    double sg[MAX_L];
    if (hipMemcpyAsync(sg, sig, MAX_L * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess) return HS_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return HS_ERR_HIP;
    if (sigma_out)
        for (int j = 0; j < L; ++j) sigma_out[j] = sg[j];
    return HS_OK;
}
