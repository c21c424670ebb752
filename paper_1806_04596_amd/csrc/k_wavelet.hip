// SARA dictionary Psi = (Dirac, db1..db8) (Sec. 2.3) and the joint-average-sparsity
// l2,1 dual update (Algorithm 2, Steps 7-8; eq:prox-L21).
//
// Each Daubechies basis is the periodised orthonormal 2-D Mallat transform.  One
// launch covers every (basis, channel) pair of one level and one direction, so a
// level costs two coalesced passes (rows along x, then columns along y) over
// the LL region of all n_db * L images.  Synthesis runs coarse to fine through a
// scratch pyramid and the final sum over bases is a single fused pass.
#include "hs_internal.h"

namespace hs {

// filt: [n_db][2][16] (h then g, zero padded), basis b = db(b+1) with 2(b+1) taps.
template <typename T>
__global__ void k_dwt_rows(const T* __restrict__ X, const T* __restrict__ srcb, T* __restrict__ dst,
                           const T* __restrict__ filt, int L, int nx, int ny, int mx, int my, int from_x) {
    const int half = mx >> 1;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= my * half) return;
    const int l = blockIdx.y, b = blockIdx.z;
    const size_t N = (size_t)nx * ny;
    const int r = e / half, k = e - r * half;
    const T* s = (from_x ? X + (size_t)l * N : srcb + ((size_t)b * L + l) * N) + (size_t)r * nx;
    const T* h = filt + b * 32;
    const T* g = h + 16;
    const int taps = 2 * (b + 1);
    T a = T(0), d = T(0);
    int idx = (2 * k) % mx;
    for (int j = 0; j < taps; ++j) {
        const T x = s[idx];
        a += h[j] * x;
        d += g[j] * x;
        if (++idx == mx) idx = 0;
    }
    T* o = dst + ((size_t)b * L + l) * N + (size_t)r * nx;
    o[k] = a;
    o[half + k] = d;
}

template <typename T>
__global__ void k_dwt_cols(const T* __restrict__ src, T* __restrict__ dst, const T* __restrict__ filt, int L, int nx,
                           int ny, int mx, int my) {
    const int half = my >> 1;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= half * mx) return;
    const int l = blockIdx.y, b = blockIdx.z;
    const size_t N = (size_t)nx * ny;
    const int k = e / mx, c = e - k * mx;
    const T* s = src + ((size_t)b * L + l) * N + c;
    const T* h = filt + b * 32;
    const T* g = h + 16;
    const int taps = 2 * (b + 1);
    T a = T(0), d = T(0);
    int idx = (2 * k) % my;
    for (int j = 0; j < taps; ++j) {
        const T x = s[(size_t)idx * nx];
        a += h[j] * x;
        d += g[j] * x;
        if (++idx == my) idx = 0;
    }
    T* o = dst + ((size_t)b * L + l) * N + c;
    o[(size_t)k * nx] = a;
    o[(size_t)(half + k) * nx] = d;
}

// Inverse along y of level region my x mx.  Rows < my/2 are approximation
// coefficients: for columns < mx/2 they come from the coarser synthesis
// (pyr) unless this is the coarsest level; everything else from C.
template <typename T>
__global__ void k_idwt_cols(const T* __restrict__ C, const T* __restrict__ pyr, T* __restrict__ dst,
                            const T* __restrict__ filt, int L, int nx, int ny, int mx, int my, int coarsest) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= my * mx) return;
    const int l = blockIdx.y, b = blockIdx.z;
    const size_t N = (size_t)nx * ny;
    const size_t off = ((size_t)b * L + l) * N;
    const int m = e / mx, c = e - m * mx;
    const int half = my >> 1;
    const T* h = filt + b * 32;
    const T* g = h + 16;
    const int taps = 2 * (b + 1);
    const T* asrc = (!coarsest && c < (mx >> 1)) ? pyr + off : C + off;
    T x = T(0);
    for (int j = (m & 1); j < taps; j += 2) {
        int q = (m - j) % my;
        if (q < 0) q += my;
        const int k = q >> 1;
        x += h[j] * asrc[(size_t)k * nx + c] + g[j] * C[off + (size_t)(half + k) * nx + c];
    }
    dst[off + (size_t)m * nx + c] = x;
}

template <typename T>
__global__ void k_idwt_rows(const T* __restrict__ src, T* __restrict__ dst, const T* __restrict__ filt, int L, int nx,
                            int ny, int mx, int my) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= my * mx) return;
    const int l = blockIdx.y, b = blockIdx.z;
    const size_t N = (size_t)nx * ny;
    const size_t off = ((size_t)b * L + l) * N;
    const int r = e / mx, m = e - r * mx;
    const int half = mx >> 1;
    const T* h = filt + b * 32;
    const T* g = h + 16;
    const int taps = 2 * (b + 1);
    const T* s = src + off + (size_t)r * nx;
    T x = T(0);
    for (int j = (m & 1); j < taps; j += 2) {
        int q = (m - j) % mx;
        if (q < 0) q += mx;
        const int k = q >> 1;
        x += h[j] * s[k] + g[j] * s[half + k];
    }
    dst[off + (size_t)r * nx + m] = x;
}

// X = C0 + sum_b Y_b  (C0 may be null)
template <typename T>
__global__ void k_psi_sum(const T* __restrict__ Y, const T* __restrict__ C0, T* __restrict__ X, int nb, int64_t LN) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= LN) return;
    T s = C0 ? C0[i] : T(0);
    for (int b = 0; b < nb; ++b) s += Y[(size_t)b * LN + i];
    X[i] = s;
}

// l2,1 on rows of length L at fixed (d, pixel):
//  mode 0 (dual, Step 7): Z = A + Psi_d^dag Xt, A <- Z min(1, thr*wbar/||Z||);
//  mode 1 (prox, eq:prox-L21): Z = A, A <- Z max(||Z|| - thr*wbar, 0)/||Z||.
template <typename T>
__global__ __launch_bounds__(256) void k_l21(T* __restrict__ A, const T* __restrict__ Xt, const T* __restrict__ coef,
                      const T* __restrict__ wbar, double thr, int L, int64_t N, int mode) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int d = blockIdx.y;
    T* Ad = A + (size_t)d * L * N + p;
    const T* Sd = (mode == 0) ? ((d == 0) ? Xt + p : coef + (size_t)(d - 1) * L * N + p) : nullptr;
    T z[MAX_L];
    double n2 = 0.0;
#pragma unroll
    for (int l = 0; l < MAX_L; ++l) {
        if (l < L) {
            T v = Ad[(size_t)l * N];
            if (Sd) v += Sd[(size_t)l * N];
            z[l] = v;
            n2 += (double)v * (double)v;
        }
    }
    const double nrm = sqrt(n2);
    const double t = thr * (wbar ? (double)wbar[(size_t)d * N + p] : 1.0);
    double f;
    if (mode == 0) f = (nrm > t) ? t / nrm : 1.0;
    else f = (nrm > t) ? (nrm - t) / nrm : 0.0;
    const T ft = (T)f;
#pragma unroll
    for (int l = 0; l < MAX_L; ++l)
        if (l < L) Ad[(size_t)l * N] = z[l] * ft;
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Psi_d^dagger for the n_db wavelet bases of X into Cout [n_db][L][N] (coef if null).
template <typename T>
void launch_psi_adj(hs_ctx* c, const T* X, T* Cout) {
    if (c->n_db == 0) return;
    T* out = Cout ? Cout : (T*)c->d.coef;
    T* tmp = (T*)c->d.wtmp;
    const T* filt = (const T*)c->d.filt;
    for (int lev = 0; lev < c->levels; ++lev) {
        const int mx = c->nx >> lev, my = c->ny >> lev;
        dim3 g1(nblk((int64_t)my * (mx / 2), 256), c->L, c->n_db);
        k_dwt_rows<T><<<g1, 256, 0, c->stream>>>(X, out, tmp, filt, c->L, c->nx, c->ny, mx, my, lev == 0 ? 1 : 0);
        dim3 g2(nblk((int64_t)(my / 2) * mx, 256), c->L, c->n_db);
        k_dwt_cols<T><<<g2, 256, 0, c->stream>>>(tmp, out, filt, c->L, c->nx, c->ny, mx, my);
    }
    // detail and approximation coefficients outside the last LL are written by
    // the level that produced them; nothing else to copy.
}

// Xout = C0 + sum_b Psi_b Cdb[b]; C0 (Dirac coefficients) may be null.
template <typename T>
void launch_psi_sum(hs_ctx* c, const T* Cdb, const T* C0, T* Xout) {
    const int64_t LN = (int64_t)c->L * c->N;
    if (c->n_db == 0) {
        k_psi_sum<T><<<nblk(LN, 256), 256, 0, c->stream>>>(nullptr, C0, Xout, 0, LN);
        return;
    }
    T* pyr = (T*)c->d.coef;   // synthesis pyramid (overwrites the analysis scratch)
    T* tmp = (T*)c->d.wtmp;
    const T* filt = (const T*)c->d.filt;
    for (int lev = c->levels - 1; lev >= 0; --lev) {
        const int mx = c->nx >> lev, my = c->ny >> lev;
        dim3 g(nblk((int64_t)my * mx, 256), c->L, c->n_db);
        k_idwt_cols<T><<<g, 256, 0, c->stream>>>(Cdb, pyr, tmp, filt, c->L, c->nx, c->ny, mx, my,
                                                 lev == c->levels - 1 ? 1 : 0);
        k_idwt_rows<T><<<g, 256, 0, c->stream>>>(tmp, pyr, filt, c->L, c->nx, c->ny, mx, my);
    }
    k_psi_sum<T><<<nblk(LN, 256), 256, 0, c->stream>>>(pyr, C0, Xout, c->n_db, LN);
}

template <typename T>
void launch_l21_dual(hs_ctx* c, T* A, const T* Xt, const T* coef, const T* wbar, double thr, int mode) {
    dim3 g(nblk(c->N, 256), c->D);
    k_l21<T><<<g, 256, 0, c->stream>>>(A, Xt, coef, wbar, thr, c->L, c->N, mode);
}

#define HS_INST(T)                                                                   \
    template void launch_psi_adj<T>(hs_ctx*, const T*, T*);                          \
    template void launch_psi_sum<T>(hs_ctx*, const T*, const T*, T*);                \
    template void launch_l21_dual<T>(hs_ctx*, T*, const T*, const T*, const T*, double, int);
HS_INST(float)
HS_INST(double)
#undef HS_INST

}  // namespace hs
