// Measurement operator Phi_l = Theta_l G_l F Z and its adjoint (Sec. 2.1, eq:inverse),
// and the data-fidelity dual update (Algorithm 2: forward operator, dual step, its
// ellipsoid projection by eq:md, and the adjoint).
//
// Design (gfx950):
//  * Hermitian half plane: the image is real, so its transform at -k is the
//    conjugate of that at k.  Only kx in [0, Kx/2] is transformed and stored;
//    a visibility at negative kx is handled at -t with conjugated value.
//  * F Z: register/LDS Stockham passes.  The row pass transforms only the ny
//    rows that Z fills (zero-padding is implicit), two real rows per complex
//    transform; the column pass works on tiles of CT adjacent columns of the
//    half plane so every HBM access is a CT-wide contiguous segment.  The
//    adjoint mirrors it and only writes the rows Z^T keeps.
//  * G (degridding): visibilities are stored tile-major; a work unit stages the
//    (T+8)^2 grid neighbourhood of its tile in LDS and each thread interpolates
//    one visibility (8 + 8 kernel values, 64 taps from LDS).
//  * G^T (gridding): output-stationary on the matrix cores: one wave owns a
//    16 x 16 block of the grid and forms it as the product of the y-kernel
//    matrix and the x-kernel-times-value matrix over the visibilities whose
//    footprints meet the block; no atomics, each grid cell written once.
//    Blocks also cover a 16-cell margin beyond kx = 0 and kx = Kx/2; the
//    adjoint column pass folds the margins back (conjugate mirror cells).
//  * Per-block FP64 sums for the ellipsoid projection are produced by a
//    deterministic segmented scan in the degridding pass and reduced per
//    (block, preconditioner value) bin, so the secular equation of the exact
//    projection is solved over bins instead of visibilities.
#include "hs_internal.h"

namespace hs {

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }

// ------------------------------------------------------------------ FFT core
// Stockham autosort FFT of length n (a power of two, 2..4096) with 16 elements
// per thread.  Each pass has radix R = min(16, n / Ns) (Ns: product of the
// radices before it); a thread owns 16 / R butterflies.  Butterfly j reads
// in[j + k n/R] (k < R), multiplies by w^(k jm) (jm = j mod Ns, w = e^(-2 pi i/(Ns R))),
// takes the R-point DFT in registers and writes out[(j - jm) R + jm + k Ns].
// The first pass reads its inputs from global memory and the last pass writes
// to global memory; LDS only carries data between passes (n = 1024: 3 passes).
// tw[m] = exp(-2 pi i m / n); INV uses the conjugate.

// e^(-2 pi i k / 16) for k < 8 (cos, sin): compile-time twiddles of the register DFTs.
__device__ constexpr double kW16c[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                                        0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613};
__device__ constexpr double kW16s[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                                        1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};

// t * e^(-+2 pi i k / R) for a compile-time k (after unrolling).
template <typename T, bool INV, int R>
__device__ __forceinline__ cplx<T> tw_const(cplx<T> t, int k) {
    if (k == 0) return t;
    if (4 * k == R) return INV ? cplx<T>{-t.im, t.re} : cplx<T>{t.im, -t.re};
    const T c = (T)kW16c[k * (16 / R)], sn = (T)kW16s[k * (16 / R)];
    return INV ? cplx<T>{t.re * c - t.im * sn, t.im * c + t.re * sn} : cplx<T>{t.re * c + t.im * sn, t.im * c - t.re * sn};
}

// In-register DFT of a[0..R-1] (natural order in and out), decimation in time.
template <typename T, bool INV, int R>
__device__ __forceinline__ void dft_reg(cplx<T>* a) {
    if constexpr (R > 1) {
        cplx<T> e[R / 2], o[R / 2];
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            e[k] = a[2 * k];
            o[k] = a[2 * k + 1];
        }
        dft_reg<T, INV, R / 2>(e);
        dft_reg<T, INV, R / 2>(o);
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            const cplx<T> t = tw_const<T, INV, R>(o[k], k);
            a[k] = cadd(e[k], t);
            a[k + R / 2] = csub(e[k], t);
        }
    }
}

// Butterfly m of this thread: j = u + m n/16.
__device__ __forceinline__ int fft_bj(int u, int m, int n) { return u + m * (n >> 4); }

// Twiddles and DFTs of the 16/R butterflies held in a (butterfly m at a[m R ..]).
template <typename T, bool INV, int R>
__device__ __forceinline__ void fft_compute(cplx<T>* a, int u, int n, int Ns, const cplx<T>* __restrict__ tw) {
#pragma unroll
    for (int m = 0; m < 16 / R; ++m) {
        const int j = fft_bj(u, m, n);
        const int jm = j & (Ns - 1);
        if (Ns > 1) {
            const int step = jm * (n / (Ns * R));
#pragma unroll
            for (int k = 1; k < R; ++k) {
                cplx<T> w = tw[k * step];
                if (INV) w.im = -w.im;
                a[m * R + k] = cmul(a[m * R + k], w);
            }
        }
        dft_reg<T, INV, R>(a + m * R);
    }
}

// LDS slot of element q of sequence s: column layout (es = CT, ss = 1) or
// row layout (one pad slot per 16 elements, against stride-R bank conflicts).
template <bool ROWS>
__device__ __forceinline__ int fft_slot(int q, int s, int n, int CT) {
    return ROWS ? s * (n + (n >> 4)) + q + (q >> 4) : q * CT + s;
}

template <typename T, bool ROWS, int R>
__device__ __forceinline__ void fft_load_lds(cplx<T>* a, const cplx<T>* buf, int u, int s, int n, int CT) {
#pragma unroll
    for (int m = 0; m < 16 / R; ++m) {
        const int j = fft_bj(u, m, n);
#pragma unroll
        for (int k = 0; k < R; ++k) a[m * R + k] = buf[fft_slot<ROWS>(j + k * (n / R), s, n, CT)];
    }
}
template <typename T, bool ROWS, int R>
__device__ __forceinline__ void fft_store_lds(const cplx<T>* a, cplx<T>* buf, int u, int s, int n, int Ns, int CT) {
#pragma unroll
    for (int m = 0; m < 16 / R; ++m) {
        const int j = fft_bj(u, m, n);
        const int jm = j & (Ns - 1);
        const int o = (j - jm) * R + jm;
#pragma unroll
        for (int k = 0; k < R; ++k) buf[fft_slot<ROWS>(o + k * Ns, s, n, CT)] = a[m * R + k];
    }
}

// First pass inputs from global: ld(q) gives element q of this thread's sequence.
template <typename T, int R, typename LD>
__device__ __forceinline__ void fft_load_glb(cplx<T>* a, int u, int n, LD ld) {
#pragma unroll
    for (int m = 0; m < 16 / R; ++m) {
        const int j = fft_bj(u, m, n);
#pragma unroll
        for (int k = 0; k < R; ++k) a[m * R + k] = ld(j + k * (n / R));
    }
}
template <typename T, int R, typename ST>
__device__ __forceinline__ void fft_store_glb(const cplx<T>* a, int u, int n, int Ns, ST st) {
#pragma unroll
    for (int m = 0; m < 16 / R; ++m) {
        const int j = fft_bj(u, m, n);
        const int jm = j & (Ns - 1);
        const int o = (j - jm) * R + jm;
#pragma unroll
        for (int k = 0; k < R; ++k) st(o + k * Ns, a[m * R + k]);
    }
}

// The whole transform of this thread's part of sequence s (u: thread index
// within the sequence, N/16 threads per sequence).  The length is a template
// parameter: the radix schedule (16, 16, ..., then the remainder), every index
// and every twiddle stride fold to constants, so only the live data and the
// current pass's twiddles occupy registers.
template <typename T, bool INV, bool ROWS, int N, int NS, typename ST>
__device__ __forceinline__ void fft_pass_ct(cplx<T>* a, cplx<T>* buf, int u, int s, int CT,
                                            const cplx<T>* __restrict__ tw, ST st) {
    constexpr int R = (N / NS) < 16 ? (N / NS) : 16;
    fft_compute<T, INV, R>(a, u, N, NS, tw);
    if constexpr (NS * R == N) {
        fft_store_glb<T, R>(a, u, N, NS, st);
    } else {
        constexpr int NS2 = NS * R;
        constexpr int R2 = (N / NS2) < 16 ? (N / NS2) : 16;
        fft_store_lds<T, ROWS, R>(a, buf, u, s, N, NS, CT);
        __syncthreads();
        fft_load_lds<T, ROWS, R2>(a, buf, u, s, N, CT);
        __syncthreads();
        fft_pass_ct<T, INV, ROWS, N, NS2>(a, buf, u, s, CT, tw, st);
    }
}
template <typename T, bool INV, bool ROWS, int N, typename LD, typename ST>
__device__ __forceinline__ void fft_run_ct(cplx<T>* buf, int u, int s, int CT, const cplx<T>* __restrict__ tw,
                                           LD ld, ST st) {
    static_assert(N >= 16 && (N & (N - 1)) == 0, "power-of-two length of at least 16");
    cplx<T> a[16];
    fft_load_glb<T, 16>(a, u, N, ld);
    fft_pass_ct<T, INV, ROWS, N, 1>(a, buf, u, s, CT, tw, st);
}

// Real-to-complex row pass of F Z.  Rows ja = 2p and jb = 2p + 1 of image l are
// deapodised, placed at (i - nx/2) mod Kx and transformed together as
// z = x_a + i x_b; the halves are separated by the Hermitian symmetry of the
// transform of a real sequence, X_a[k] = (Z[k] + conj Z[-k]) / 2 and
// X_b[k] = -i (Z[k] - conj Z[-k]) / 2, and only k in [0, Kx/2] is kept
// (row stride Hs).  The last FFT pass writes Z to LDS for the separation.
template <typename T, int Kx>
__global__ __launch_bounds__(512) void k_fft_rows_fwd(const T* __restrict__ X, cplx<T>* __restrict__ H,
                                                       const T* __restrict__ sx, const T* __restrict__ sy,
                                                       const cplx<T>* __restrict__ tw, int nx, int ny,
                                                       int Hs, int pairs) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
    const int l = blockIdx.y;
    const int tps = Kx >> 4;                        // threads per sequence
    const int u = threadIdx.x % tps, s = threadIdx.x / tps;
    const int ja = 2 * (blockIdx.x * pairs + s);
    const T* Xa = X + ((size_t)l * ny + ja) * nx;
    const T* Xb = Xa + nx;
    const T sya = sy[ja], syb = sy[ja + 1];
    fft_run_ct<T, false, true, Kx>(buf, u, s, 0, tw,
        [&](int q) {
            int i = q + (nx >> 1);
            if (i >= Kx) i -= Kx;
            if (i >= nx) return cplx<T>{T(0), T(0)};
            const T w = sx[i];
            return cplx<T>{Xa[i] * w * sya, Xb[i] * w * syb};
        },
        [&](int q, const cplx<T>& v) { buf[fft_slot<true>(q, s, Kx, 0)] = v; });
    __syncthreads();
    const int Kh = Kx >> 1;
    cplx<T>* Ha = H + ((size_t)l * ny + ja) * Hs;
    cplx<T>* Hb = Ha + Hs;
    for (int k = u; k <= Kh; k += tps) {
        const cplx<T> zk = buf[fft_slot<true>(k, s, Kx, 0)];
        const cplx<T> zm = buf[fft_slot<true>((Kx - k) & (Kx - 1), s, Kx, 0)];
        Ha[k] = {(zk.re + zm.re) * T(0.5), (zk.im - zm.im) * T(0.5)};
        Hb[k] = {(zk.im + zm.im) * T(0.5), (zm.re - zk.re) * T(0.5)};
    }
}

// Column tile of work-group b (of nb): work-groups b and b + 8 run on the same
// XCD (work-groups are dispatched round-robin over the 8 XCDs, each with its
// own L2) and take adjacent tiles, so both halves of a 128-byte line of a grid
// row are read through one L2.  Tiles past the last full group of 16 keep
// their index.
__device__ __forceinline__ int xcd_pair_tile(int b, int nb) {
    if (b >= (nb & ~15)) return b;
    const int q = b >> 4, r = b & 15;
    return (q << 4) + ((r & 7) << 1) + (r >> 3);
}

// Work item of work-group b (of n) when consecutive items are dealt to the 8
// XCDs in groups of G: work-groups are dispatched round-robin over the XCDs
// (b mod 8 names the XCD, each has its own L2), and within each run of 8G
// work-groups XCD x takes items [xG, xG + G) of the run, so neighbouring items
// (which share input) meet in one L2.  G = 1 is the identity; the items of the
// last incomplete run keep their index.  A bijection of [0, n).
__device__ __forceinline__ int xcd_group_item(int b, int n, int G) {
    if (G <= 1 || b >= (n / (8 * G)) * 8 * G) return b;
    const int s = b >> 3, k = s / G;
    return k * 8 * G + (b & 7) * G + (s - k * G);
}

// Column pass of F over the half plane: columns kx in [0, Kx/2] in tiles of CT
// adjacent columns (the last tile is partly idle), rows placed at
// (j - ny/2) mod Ky.  The grid row has Wg cells, kx = 0 at cell T.
template <typename T> struct NV2;
template <> struct NV2<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct NV2<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <typename T>
__device__ __forceinline__ cplx<T> ldnt_c(const cplx<T>* p) {
    const typename NV2<T>::type v = __builtin_nontemporal_load(reinterpret_cast<const typename NV2<T>::type*>(p));
    return cplx<T>{v[0], v[1]};
}
template <typename T>
__device__ __forceinline__ void stnt_c(cplx<T>* p, const cplx<T>& c) {
    typename NV2<T>::type v;
    v[0] = c.re; v[1] = c.im;
    __builtin_nontemporal_store(v, reinterpret_cast<typename NV2<T>::type*>(p));
}

template <typename T, int Ky, bool NT>
__global__ __launch_bounds__(512) void k_fft_cols_fwd(const cplx<T>* __restrict__ H, cplx<T>* __restrict__ G,
                                                       const cplx<T>* __restrict__ tw, int ny, int Kh,
                                                       int Hs, int Wg, int CT) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
    const int l = blockIdx.y;
    const int s = threadIdx.x & (CT - 1), u = threadIdx.x / CT;
    const int c = xcd_pair_tile(blockIdx.x, gridDim.x) * CT + s;
    const bool live = c <= Kh;
    const cplx<T>* Hl = H + (size_t)l * ny * Hs + c;
    cplx<T>* Gl = G + (size_t)l * Ky * Wg + GR_MARGIN + c;
    // NT: the grid rows go out as non-temporal stores (the launcher picks it when a
    // tile's row segment is at least 64 bytes; narrower segments reach memory as
    // partial lines and are slower that way)
    fft_run_ct<T, false, false, Ky>(buf, u, s, CT, tw,
        [&](int q) {
            int j = q + (ny >> 1);
            if (j >= Ky) j -= Ky;
            return (live && j < ny) ? Hl[(size_t)j * Hs] : cplx<T>{T(0), T(0)};
        },
        [&](int q, const cplx<T>& v) {
            if (live) {
                if constexpr (NT) stnt_c(Gl + (size_t)q * Wg, v);
                else Gl[(size_t)q * Wg] = v;
            }
        });
}

// Adjoint column pass over the half plane: inverse (unnormalised) DFT along y
// of the folded grid, keeping the rows Z^T reads.  Gridding leaves the
// contributions that fall beyond kx = 0 or kx = Kx/2 in the margins of the
// grid row; the Hermitian part of the full-plane grid is (g[k] + conj g[-k]) / 2,
// so columns within GR_FOLD of either edge add the conjugate of their mirror
// cell as they are loaded (the factor 1/2 is applied by the row pass).
constexpr int GR_FOLD = 4;
template <typename T, int Ky>
__global__ __launch_bounds__(512) void k_fft_cols_adj(const cplx<T>* __restrict__ G, cplx<T>* __restrict__ H,
                                                       const cplx<T>* __restrict__ tw, int ny, int Kh,
                                                       int Hs, int Wg, int CT) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
    const int l = blockIdx.y;
    const int s = threadIdx.x & (CT - 1), u = threadIdx.x / CT;
    const int c = xcd_pair_tile(blockIdx.x, gridDim.x) * CT + s;
    const bool live = c <= Kh;
    const bool fold = c <= GR_FOLD || (c >= Kh - GR_FOLD && live);
    const int mx = c <= GR_FOLD ? -c : 2 * Kh - c;
    const cplx<T>* G0 = G + (size_t)l * Ky * Wg + GR_MARGIN;   // kx = 0
    cplx<T>* Hl = H + (size_t)l * ny * Hs + c;
    fft_run_ct<T, true, false, Ky>(buf, u, s, CT, tw,
        [&](int q) {
            if (!live) return cplx<T>{T(0), T(0)};
            cplx<T> g = G0[(size_t)q * Wg + c];
            if (fold) {
                const cplx<T> h = G0[(size_t)(q == 0 ? 0 : Ky - q) * Wg + mx];
                g.re += h.re;
                g.im -= h.im;
            }
            return g;
        },
        [&](int q, const cplx<T>& v) {
            int j = q + (ny >> 1);
            if (j >= Ky) j -= Ky;
            if (live && j < ny) Hl[(size_t)j * Hs] = v;
        });
}

// Complex-to-real adjoint row pass: rows ja = 2p and jb = 2p + 1 hold the half
// spectra A, B (k in [0, Kx/2]) of two real rows; Z[k] = A[k] + i B[k] with
// A[k] = conj A[Kx - k] beyond Kx/2 (and the real parts at k = 0 and Kx/2,
// which is what the real part of the full inverse transform keeps) gives
// x_a + i x_b in one inverse DFT.  Crop, deapodise, times 1/2.
template <typename T, int Kx>
__global__ __launch_bounds__(512) void k_fft_rows_adj(const cplx<T>* __restrict__ H, T* __restrict__ X,
                                                       const T* __restrict__ sx, const T* __restrict__ sy,
                                                       const cplx<T>* __restrict__ tw, int nx, int ny,
                                                       int Hs, int pairs) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
    const int l = blockIdx.y;
    const int tps = Kx >> 4;
    const int u = threadIdx.x % tps, s = threadIdx.x / tps;
    const int ja = 2 * (blockIdx.x * pairs + s);
    const int Kh = Kx >> 1;
    const cplx<T>* Ha = H + ((size_t)l * ny + ja) * Hs;
    const cplx<T>* Hb = Ha + Hs;
    T* Xa = X + ((size_t)l * ny + ja) * nx;
    T* Xb = Xa + nx;
    const T sya = sy[ja] * T(0.5), syb = sy[ja + 1] * T(0.5);
    fft_run_ct<T, true, true, Kx>(buf, u, s, 0, tw,
        [&](int q) {
            const bool up = q > Kh;
            const int k = up ? Kx - q : q;
            cplx<T> a = Ha[k], b = Hb[k];
            if (up) {
                a.im = -a.im;
                b.im = -b.im;
            } else if (q == 0 || q == Kh) {
                a.im = T(0);
                b.im = T(0);
            }
            return cplx<T>{a.re - b.im, a.im + b.re};
        },
        [&](int q, const cplx<T>& v) {
            int i = q + (nx >> 1);
            if (i >= Kx) i -= Kx;
            if (i < nx) {
                const T w = sx[i];
                __builtin_nontemporal_store(v.re * w * sya, Xa + i);
                __builtin_nontemporal_store(v.im * w * syb, Xb + i);
            }
        });
}

template <typename KF>
static void set_lds(KF kern, size_t bytes) {
    if (bytes > 65536) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Row pairs per workgroup for the row passes (power of two, 2 * pairs dividing
// ny, Kx * pairs <= 8192: <= 512 threads).
static int row_group(const hs_ctx* c) {
    int p = 1;
    while (4 * p <= c->ny && (c->ny % (4 * p)) == 0 && c->Kx * p * 2 <= 8192) p *= 2;
    return p;
}
// Columns per tile for the column passes (16 elements per thread, <= 512 threads, LDS <= 128 KiB):
// the tuned value when set, else the widest that fits.
static bool col_tile_fits(const hs_ctx* c, int ct, size_t csz) {
    return ct >= 1 && ct <= 16 && (ct & (ct - 1)) == 0 && ct <= c->Kh && (size_t)c->Ky * ct * csz <= 131072 &&
           c->Ky * ct <= 8192;
}
template <typename T>
static int col_group(const hs_ctx* c) {
    if (c->fft_ct > 0 && col_tile_fits(c, c->fft_ct, sizeof(cplx<T>))) return c->fft_ct;
    int ct = 1;
    while (col_tile_fits(c, ct * 2, sizeof(cplx<T>))) ct *= 2;
    return ct;
}
int fft_col_tile(const hs_ctx* c) {
    return c->dtype == HS_F32 ? col_group<float>(c) : col_group<double>(c);
}
bool fft_col_tile_ok(const hs_ctx* c, int ct) {
    return col_tile_fits(c, ct, c->dtype == HS_F32 ? sizeof(cplx<float>) : sizeof(cplx<double>));
}
static size_t row_lds(const hs_ctx* c, int rows, size_t csz) {
    return (size_t)rows * (c->Kx + (c->Kx >> 4)) * csz;
}

// Allow up to 160 KiB of dynamic LDS for every FFT instantiation (set once,
// outside any stream capture).
// Transform lengths (Kx = 2 nx, Ky = 2 ny with nx, ny powers of two in 16..2048).
#define HS_FFT_LEN_SWITCH(n, BODY)                         \
    switch (n) {                                           \
        case 32: { constexpr int NN = 32; BODY; } break;   \
        case 64: { constexpr int NN = 64; BODY; } break;   \
        case 128: { constexpr int NN = 128; BODY; } break; \
        case 256: { constexpr int NN = 256; BODY; } break; \
        case 512: { constexpr int NN = 512; BODY; } break; \
        case 1024: { constexpr int NN = 1024; BODY; } break; \
        case 2048: { constexpr int NN = 2048; BODY; } break; \
        default: { constexpr int NN = 4096; BODY; } break; \
    }

template <typename T, int NN>
static void fft_attrs_len() {
    const size_t b = 160 * 1024;
    set_lds(k_fft_rows_fwd<T, NN>, b);
    set_lds(k_fft_cols_fwd<T, NN, false>, b);
    set_lds(k_fft_cols_fwd<T, NN, true>, b);
    set_lds(k_fft_cols_adj<T, NN>, b);
    set_lds(k_fft_rows_adj<T, NN>, b);
}
template <typename T>
static void fft_attrs_one() {
    for (int n = 32; n <= 4096; n *= 2) HS_FFT_LEN_SWITCH(n, (fft_attrs_len<T, NN>()))
}
void fft_init_attrs() {
    static bool done = false;
    if (done) return;
    fft_attrs_one<float>();
    fft_attrs_one<double>();
    done = true;
}

// The transforms of channels l0 .. l0 + L - 1 (the channel index of each work-group
// is relative to the offset base pointers).
template <typename T>
void launch_fft_rows_fwd(hs_ctx* c, const T* X, int L, int l0) {
    const int p = row_group(c);
    dim3 grid(c->ny / (2 * p), L);
    HS_FFT_LEN_SWITCH(c->Kx, (k_fft_rows_fwd<T, NN><<<grid, c->Kx * p / 16, row_lds(c, p, sizeof(cplx<T>)), c->stream>>>(
        X + (size_t)l0 * c->N, (cplx<T>*)c->d.H + (size_t)l0 * c->ny * c->Hs, (const T*)c->d.sx, (const T*)c->d.sy,
        (const cplx<T>*)c->d.tw_x, c->nx, c->ny, c->Hs, p)))
}
template <typename T>
void launch_fft_cols_fwd(hs_ctx* c, int L, int l0) {
    const int ct = col_group<T>(c);
    const bool nt = ct * (int)sizeof(cplx<T>) >= 64;
    dim3 grid((c->Wh + ct - 1) / ct, L);
    const cplx<T>* H = (const cplx<T>*)c->d.H + (size_t)l0 * c->ny * c->Hs;
    cplx<T>* G = (cplx<T>*)c->d.grid + (size_t)l0 * c->Ky * c->Wg;
    const size_t lds = (size_t)c->Ky * ct * sizeof(cplx<T>);
    if (nt)
        HS_FFT_LEN_SWITCH(c->Ky, (k_fft_cols_fwd<T, NN, true><<<grid, c->Ky * ct / 16, lds, c->stream>>>(
            H, G, (const cplx<T>*)c->d.tw_y, c->ny, c->Kh, c->Hs, c->Wg, ct)))
    else
        HS_FFT_LEN_SWITCH(c->Ky, (k_fft_cols_fwd<T, NN, false><<<grid, c->Ky * ct / 16, lds, c->stream>>>(
            H, G, (const cplx<T>*)c->d.tw_y, c->ny, c->Kh, c->Hs, c->Wg, ct)))
}
template <typename T>
void launch_fft_cols_adj(hs_ctx* c, int L, int l0) {
    const int ct = col_group<T>(c);
    dim3 grid((c->Wh + ct - 1) / ct, L);
    HS_FFT_LEN_SWITCH(c->Ky, (k_fft_cols_adj<T, NN><<<grid, c->Ky * ct / 16, (size_t)c->Ky * ct * sizeof(cplx<T>), c->stream>>>(
        (const cplx<T>*)c->d.grid + (size_t)l0 * c->Ky * c->Wg, (cplx<T>*)c->d.H + (size_t)l0 * c->ny * c->Hs,
        (const cplx<T>*)c->d.tw_y, c->ny, c->Kh, c->Hs, c->Wg, ct)))
}
template <typename T>
void launch_fft_rows_adj(hs_ctx* c, T* Xout, int L, int l0) {
    const int p = row_group(c);
    dim3 grid(c->ny / (2 * p), L);
    HS_FFT_LEN_SWITCH(c->Kx, (k_fft_rows_adj<T, NN><<<grid, c->Kx * p / 16, row_lds(c, p, sizeof(cplx<T>)), c->stream>>>(
        (const cplx<T>*)c->d.H + (size_t)l0 * c->ny * c->Hs, Xout + (size_t)l0 * c->N, (const T*)c->d.sx,
        (const T*)c->d.sy, (const cplx<T>*)c->d.tw_x, c->nx, c->ny, c->Hs, p)))
}

// Work-list range of channel lc (lc < 0: every channel).
static inline void chan_range(const std::vector<int64_t>& off, int lc, int64_t& b, int64_t& n) {
    if (lc < 0) { b = 0; n = off.back(); }
    else { b = off[lc]; n = off[lc + 1] - off[lc]; }
}

// ------------------------------------------------------------- KB kernel
// The eight kernel values phi(f + 3 - j), j = 0..7, of a fractional offset f from
// the per-tap polynomials of the plan (taps 0..3; tap 7 - j is tap j at -t):
// 2 x (the even and odd Horner chains in t^2) per pair of taps, the coefficients
// uniform across lanes (scalar operands).
template <typename T>
__device__ __forceinline__ void kb_weights(T f, const KBPoly<T>& P, T* w) {
    constexpr int NE = KBPoly<T>::NE, NO = KBPoly<T>::NO;
    const T t = f - T(0.5);
    const T t2 = t * t;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        T e = P.e[j][NE - 1];
#pragma unroll
        for (int k = NE - 2; k >= 0; --k) e = e * t2 + P.e[j][k];
        T o = P.o[j][NO - 1];
#pragma unroll
        for (int k = NO - 2; k >= 0; --k) o = o * t2 + P.o[j][k];
        const T to = t * o;
        w[j] = e + to;
        w[KB_J - 1 - j] = e - to;
    }
}

// ------------------------------------------------------------- degridding
// Stage the (T+8)^2 window of the half-plane grid around tile origin (ox, oy):
// g0 points at kx = 0 of the channel's grid (rows of Wg cells).  Cells beyond the
// half plane (kx < 0 or kx > Kx/2) are the conjugates of their reflections
// (Hermitian symmetry of the transform of a real image); y is periodic.
// The staged grid window of a degridding tile: TT + 8 rows of TT + 8 cells at a row
// stride of TT + 8 + DEG_PAD cells (the padding moves neighbouring rows to other LDS
// banks).
constexpr int DEG_PAD = 1;
__host__ __device__ constexpr int deg_stride(int TT) { return TT + 8 + DEG_PAD; }

template <typename T>
__device__ __forceinline__ void stage_tile(cplx<T>* tileS, const cplx<T>* g0, int ox, int oy, int TT, int Kh, int Ky,
                                           int Wg) {
    const int W = TT + 8, S = deg_stride(TT);
    for (int e = threadIdx.x; e < W * W; e += blockDim.x) {
        const int ry = e / W, rx = e - ry * W;
        int gy = oy - 3 + ry;
        if (gy < 0) gy += Ky;
        if (gy >= Ky) gy -= Ky;
        const int gx = ox - 3 + rx;
        cplx<T> v;
        if (gx >= 0 && gx <= Kh) {
            v = g0[(size_t)gy * Wg + gx];
        } else {
            const int mx = gx < 0 ? -gx : 2 * Kh - gx;
            const int my = gy == 0 ? 0 : Ky - gy;
            const cplx<T> w = g0[(size_t)my * Wg + mx];
            v = {w.re, -w.im};
        }
        tileS[ry * S + rx] = v;
    }
}

template <typename T>
__device__ __forceinline__ cplx<T> interp(const cplx<T>* tileS, int W, int lx, int ly, T fx, T fy,
                                          const KBPoly<T>& kb) {
    T wx[KB_J], wy[KB_J];
    kb_weights(fx, kb, wx);
    kb_weights(fy, kb, wy);
    cplx<T> acc{T(0), T(0)};
#pragma unroll
    for (int jy = 0; jy < KB_J; ++jy) {
        const cplx<T>* row = tileS + (ly + jy) * W + lx;
        T rr = T(0), ri = T(0);
#pragma unroll
        for (int jx = 0; jx < KB_J; ++jx) {
            const cplx<T> gv = row[jx];
            rr += wx[jx] * gv.re;
            ri += wx[jx] * gv.im;
        }
        acc.re += wy[jy] * rr;
        acc.im += wy[jy] * ri;
    }
    return acc;
}

// out[dst] = theta * mult * (G ghat)(vis), dst = perm[pos] (caller order, PERM) or
// pos; mult is applied when MULT.  The optional operands are template switches,
// so the loop body has no branches after the interpolation.
template <typename T, bool PERM, bool MULT>
__global__ __launch_bounds__(DEG_THREADS) void k_degrid_plain(
    const DegridUnit* __restrict__ units, const int32_t* __restrict__ cell, const cplx<T>* __restrict__ frac,
    const cplx<T>* __restrict__ grid, const T* __restrict__ theta, const T* __restrict__ mult,
    const int32_t* __restrict__ perm, cplx<T>* __restrict__ out, int Kh, int Ky, int Wg, int TT, int tiles_x,
    KBPoly<T> kb, int xg) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* tileS = reinterpret_cast<cplx<T>*>(smem_raw);
    // units are in tile order per channel: grouping keeps the halo a tile shares
    // with its neighbours in one L2
    const DegridUnit u = units[xcd_group_item(blockIdx.x, gridDim.x, xg)];
    const int ox = (u.tile % tiles_x) * TT, oy = (u.tile / tiles_x) * TT;
    stage_tile(tileS, grid + (size_t)u.l * Ky * Wg + GR_MARGIN, ox, oy, TT, Kh, Ky, Wg);
    __syncthreads();
    const int W = deg_stride(TT);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // chunk j of the unit (DEG_CHUNK visibilities) is walked by wave j mod 4
    for (int j = wave; j * DEG_CHUNK < u.count; j += DEG_THREADS / DEG_CHUNK) {
        const int i = j * DEG_CHUNK + lane;
        if (i < u.count) {
            const int pos = u.start + i;
            const int cc = cell[pos];
            const int cx = cc & 0x7FFF, cy = cc >> 16;
            const cplx<T> f = frac[pos];
            cplx<T> a = interp(tileS, W, cx - ox, cy - oy, f.re, f.im, kb);
            if (cc & 0x8000) a.im = -a.im;   // reflected visibility: conjugate of the value at -t
            T s = theta[pos];
            if constexpr (MULT) s *= mult[pos];
            a.re *= s;
            a.im *= s;
            if constexpr (PERM) out[perm[pos]] = a;
            else out[pos] = a;
        }
    }
}

// Phase 1 of the data dual (Algorithm 2): g = Theta G u, d = v + U (g - y)
// (= vbar - U y) stored in v; per-run FP64 sums of |d|^2 and |y - g|^2.
// Segmented inclusive sums of two FP64 values over the 64 lanes of a wave (lane
// `head` starts this lane's segment), by DPP lane moves instead of LDS permutes:
// row shifts by 1, 2, 4, 8 sum each 16-lane row from max(head, row start), then
// the last lane of row 0 is broadcast into row 1 (and that of row 2 into row 3),
// and the last lane of row 1, by then complete, into rows 2 and 3; a lane adds a
// moved value only when its segment reaches back to the source lane.  Lanes that
// a move does not reach receive zero.
template <int CTRL, int RMASK>
__device__ __forceinline__ double dpp_f64(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, RMASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, RMASK, 0xF, true);
    return __hiloint2double(hi, lo);
}
template <int CTRL, int RMASK>
__device__ __forceinline__ void seg_step(double& a0, double& a1, bool take) {
    const double y0 = dpp_f64<CTRL, RMASK>(a0), y1 = dpp_f64<CTRL, RMASK>(a1);
    if (take) {
        a0 += y0;
        a1 += y1;
    }
}
__device__ __forceinline__ void seg_scan2(double& a0, double& a1, int lane, int head) {
    seg_step<0x111, 0xF>(a0, a1, (lane & 15) >= 1 && lane - 1 >= head);    // row_shr:1
    seg_step<0x112, 0xF>(a0, a1, (lane & 15) >= 2 && lane - 2 >= head);    // row_shr:2
    seg_step<0x114, 0xF>(a0, a1, (lane & 15) >= 4 && lane - 4 >= head);    // row_shr:4
    seg_step<0x118, 0xF>(a0, a1, (lane & 15) >= 8 && lane - 8 >= head);    // row_shr:8
    // row_bcast:15 into rows 1 and 3 (sources: lanes 15 and 47)
    seg_step<0x142, 0xA>(a0, a1, ((lane >> 4) & 1) && head <= (lane & ~15) - 1);
    // row_bcast:31 into rows 2 and 3 (source: lane 31)
    seg_step<0x143, 0xC>(a0, a1, lane >= 32 && head <= 31);
}

template <typename T>
__global__ __launch_bounds__(DEG_THREADS) void k_degrid_dual(
    const DegridUnit* __restrict__ units, const int32_t* __restrict__ cell, const cplx<T>* __restrict__ frac,
    const cplx<T>* __restrict__ grid, const T* __restrict__ theta, const T* __restrict__ uprec,
    const cplx<T>* __restrict__ yv, const int32_t* __restrict__ vbin, cplx<T>* __restrict__ v,
    const int32_t* __restrict__ chunk_run, const int32_t* __restrict__ run_slot, double* __restrict__ run_sum, int Kh, int Ky, int Wg, int TT, int tiles_x,
    KBPoly<T> kb, int xg) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* tileS = reinterpret_cast<cplx<T>*>(smem_raw);
    // units are in tile order per channel: grouping keeps the halo a tile shares
    // with its neighbours in one L2
    const DegridUnit u = units[xcd_group_item(blockIdx.x, gridDim.x, xg)];
    const int ox = (u.tile % tiles_x) * TT, oy = (u.tile / tiles_x) * TT;
    stage_tile(tileS, grid + (size_t)u.l * Ky * Wg + GR_MARGIN, ox, oy, TT, Kh, Ky, Wg);
    __syncthreads();
    const int W = deg_stride(TT);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long le = lane == 63 ? ~0ull : ((2ull << lane) - 1);   // lanes <= this one
    // chunk j of the unit (DEG_CHUNK visibilities) is walked by wave j mod 4
    for (int j = wave; j * DEG_CHUNK < u.count; j += DEG_THREADS / DEG_CHUNK) {
        const int i = j * DEG_CHUNK + lane;
        const bool act = i < u.count;
        double a0 = 0.0, a1 = 0.0;
        int bin = -1;
        if (act) {
            const int pos = u.start + i;
            const int cc = cell[pos];
            const int cx = cc & 0x7FFF, cy = cc >> 16;
            const cplx<T> f = frac[pos];
            cplx<T> g = interp(tileS, W, cx - ox, cy - oy, f.re, f.im, kb);
            if (cc & 0x8000) g.im = -g.im;   // reflected visibility
            const T th = theta[pos];
            g.re *= th;
            g.im *= th;
            const cplx<T> yy = yv[pos];
            const T uu = uprec[pos];
            const cplx<T> vv = v[pos];
            const cplx<T> r{yy.re - g.re, yy.im - g.im};
            const cplx<T> d{vv.re - uu * r.re, vv.im - uu * r.im};
            v[pos] = d;
            a0 = (double)d.re * (double)d.re + (double)d.im * (double)d.im;
            a1 = (double)r.re * (double)r.re + (double)r.im * (double)r.im;
            bin = vbin[pos];
        }
        // runs of equal bin within the chunk: segmented inclusive sums by shuffles
        const int bprev = __shfl_up(bin, 1);
        const unsigned long long heads = __ballot(act && (lane == 0 || bin != bprev));
        const int head = 63 - __builtin_clzll(heads & le);   // first lane of this lane's run
        seg_scan2(a0, a1, lane, head);
        const bool last = lane == 63 || !act || ((heads >> (lane + 1)) & 1ull) || (i + 1 >= u.count);
        if (act && last) {
            const int slot = run_slot[chunk_run[u.chunk0 + j] + __popcll(heads & le) - 1];
            run_sum[2 * (size_t)slot] = a0;
            run_sum[2 * (size_t)slot + 1] = a1;
        }
    }
}

// Bin sums (fixed order, one wave per bin): S[bin] = sum of its runs, which
// the degridding stored in the bin's contiguous slot range.
__global__ void k_bin_reduce(const int32_t* __restrict__ bin_run_ptr, const double* __restrict__ run_sum,
                             double* __restrict__ S, int nbins) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wave >= nbins) return;
    const int r0 = bin_run_ptr[wave], r1 = bin_run_ptr[wave + 1];
    double a = 0.0, b = 0.0;
    for (int k = r0 + lane; k < r1; k += 64) {
        a += run_sum[2 * (size_t)k];
        b += run_sum[2 * (size_t)k + 1];
    }
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
    }
    if (lane == 0) {
        S[2 * (size_t)wave] = a;
        S[2 * (size_t)wave + 1] = b;
    }
}

__device__ __forceinline__ double wave_sum(double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// Root of f(lam) = sum_c S_c/(u_c + lam)^2 - eps^2 per block (exact ellipsoid
// projection, eq:prox with the metric U), one wave per block; Newton from
// lam = 0, monotone for this convex decreasing f.  Also the residual norms rho
// and the adaptive l2 bounds of Algorithm 2 (Sec. 3.6) when enabled.
__global__ void k_block_roots(const int32_t* __restrict__ blk_bin_ptr, const double* __restrict__ S,
                              const double* __restrict__ bin_u, double* __restrict__ bin_f, int u_f32,
                              double* __restrict__ eps, double* __restrict__ lam_out,
                              double* __restrict__ rho2, int32_t* __restrict__ vartheta, const double* __restrict__ scal,
                              int nblk, int adaptive, double lam1, double lam2, double lam3, int vbar) {
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wave >= nblk) return;
    const int c0 = blk_bin_ptr[wave], c1 = blk_bin_ptr[wave + 1];
    const double e = eps[wave];
    const double e2 = e * e;
    double f0 = 0.0, tot = 0.0, r2 = 0.0;
    for (int k = c0 + lane; k < c1; k += 64) {
        const double s = S[2 * (size_t)k], uu = bin_u[k];
        f0 += s / (uu * uu);
        tot += s;
        r2 += S[2 * (size_t)k + 1];
    }
    f0 = wave_sum(f0);
    tot = wave_sum(tot);
    r2 = wave_sum(r2);
    double lam = 0.0;
    if (f0 > e2) {
        if (e2 <= 0.0) {
            lam = INFINITY;
        } else {
            double hi = sqrt(tot) / e;
            for (int it = 0; it < 200; ++it) {
                double f = 0.0, fp = 0.0;
                for (int k = c0 + lane; k < c1; k += 64) {
                    const double s = S[2 * (size_t)k], q = 1.0 / (bin_u[k] + lam);
                    const double q2 = q * q;
                    f += s * q2;
                    fp += s * q2 * q;
                }
                f = wave_sum(f) - e2;
                fp = -2.0 * wave_sum(fp);
                if (f <= 1e-15 * e2) break;
                double nl = lam - f / fp;
                if (!(nl > lam)) break;
                if (nl > hi) nl = hi;
                if (nl - lam <= 1e-16 * nl) { lam = nl; break; }
                lam = nl;
            }
        }
    }
    // the projection's factor for each bin of the block, v = d lam/(u + lam), with u as
    // the visibilities hold it (rounded to FP32 in an FP32 context)
    for (int k = c0 + lane; k < c1; k += 64) {
        const double uu = u_f32 ? (double)(float)bin_u[k] : bin_u[k];
        bin_f[k] = lam == 0.0 ? 0.0 : (isinf(lam) ? 1.0 : lam / (uu + lam));
    }
    if (lane == 0) {
        lam_out[wave] = lam;
        rho2[wave] = r2;
        if (adaptive) {
            const double beta_prev = scal[0];
            const double t = scal[1] + 1.0;
            const double rho = sqrt(r2);
            if (beta_prev < lam1 && (t - (double)vartheta[wave]) > (double)vbar && fabs(rho - e) / e > lam2) {
                eps[wave] = lam3 * rho + (1.0 - lam3) * e;
                vartheta[wave] = (int32_t)t;
            }
        }
    }
}

// Phase 2 (the projection of Algorithm 2): v = d * lam/(u + lam) (= vbar - U q); lam = inf gives v = d.
// The factor is the same for all visibilities of a bin (one u per bin, one lam per
// block), so k_block_roots forms it once per bin.
template <typename T>
__global__ void k_dual_apply(cplx<T>* __restrict__ v, const int32_t* __restrict__ vbin, const double* __restrict__ bin_f,
                             int64_t M) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const T f = (T)bin_f[vbin[i]];
    cplx<T> d = v[i];
    d.re *= f;
    d.im *= f;
    v[i] = d;
}

// The same, two visibilities per thread (v + 2i 16-byte aligned for FP32: the
// caller passes an even start).
template <typename T>
__global__ void k_dual_apply2(cplx<T>* __restrict__ v, const int32_t* __restrict__ vbin,
                              const double* __restrict__ bin_f, int64_t M) {
    const int64_t i = 2 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i + 1 < M) {
        const int2 b = *reinterpret_cast<const int2*>(vbin + i);
        const T f0 = (T)bin_f[b.x], f1 = (T)bin_f[b.y];
        cplx<T> d0 = v[i], d1 = v[i + 1];
        d0.re *= f0;
        d0.im *= f0;
        d1.re *= f1;
        d1.im *= f1;
        v[i] = d0;
        v[i + 1] = d1;
    } else if (i < M) {
        const T f = (T)bin_f[vbin[i]];
        cplx<T> d = v[i];
        d.re *= f;
        d.im *= f;
        v[i] = d;
    }
}

// ---------------------------------------------------------- gridding (pull)
// Output-stationary gridding on the matrix cores.  One wave owns a GB x GB
// (16 x 16) output block and consumes every visibility whose 8 x 8 footprint
// meets it (the plan lists them, in plan order).  For entries e with first-tap
// offset (dy_e, dx_e) from the block origin, kernel values wy_e, wx_e and value
// v_e, the block is
//     G[i][j] = sum_e wy_e(i - dy_e) wx_e(j - dx_e) v_e
// (terms outside the footprint are zero), i.e. the product A B of the 16 x E
// matrix A[i][e] = wy_e(i - dy_e) and the E x 16 matrix B[e][j] = wx_e(j - dx_e) v_e.
// Each 16x16x4 MFMA takes four entries: lane (i, k) = (lane & 15, lane >> 4)
// supplies A[i][k] and B[k][i] from the staged values of entry 4q + k; the real
// and imaginary parts of v are two products with a shared A.  The accumulators
// stay in registers; each grid cell is written once (no atomics, fixed order).
// Entries come in batches of 64: lane e stages entry e's kernel values, offsets
// and value in LDS.  Blocks with many entries are split; their partial blocks
// are summed in fixed order.
typedef float grid_f4 __attribute__((ext_vector_type(4)));
typedef double grid_d4 __attribute__((ext_vector_type(4)));
template <typename T> struct GridAcc;
template <> struct GridAcc<float> { typedef grid_f4 type; };
template <> struct GridAcc<double> { typedef grid_d4 type; };
__device__ __forceinline__ grid_f4 grid_mfma(float a, float b, grid_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ grid_d4 grid_mfma(double a, double b, grid_d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Row of the 16 x 16 result held in element r of this lane (column lane & 15):
// f32 puts rows 4 (lane >> 4) + r in a lane, f64 rows (lane >> 4) + 4 r.
template <typename T>
__device__ __forceinline__ int grid_mfma_row(int lane, int r) {
    return sizeof(T) == 4 ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r;
}

// Orders this wave's LDS accesses around a wave-local exchange (the LDS
// operations of one wave complete in issue order).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Staged operands of one entry: its eight kernel values with a zero on each side,
// so that an operand is a single LDS read at a clamped index (no masks).
constexpr int GR_WS = KB_J + 2;
constexpr int GR_BATCH = 64;   // entries staged per batch (one lane per entry)

template <typename T>
__global__ __launch_bounds__(64) void k_grid_pull(
    const GridUnit* __restrict__ units, const int32_t* __restrict__ glist, const int32_t* __restrict__ cell,
    const cplx<T>* __restrict__ frac, const cplx<T>* __restrict__ vals, const T* __restrict__ weight,
    cplx<T>* __restrict__ grid, cplx<T>* __restrict__ partial, int Ky, int Wg, int nbx, KBPoly<T> kb, int xg) {
    typedef typename GridAcc<T>::type acc_t;
    // entry e: sA[e][1 + j] = wy_e(j), sB[e][1 + j] = wx_e(j) v_e, zeros at 0 and KB_J + 1;
    // sd[e] = (dy, dx), the offsets of its first tap from the block origin
    __shared__ T sA[GR_BATCH * GR_WS];
    __shared__ cplx<T> sB[GR_BATCH * GR_WS];
    __shared__ int2 sd[GR_BATCH];
    // gridding units are in block order (row-major per channel), and a visibility
    // is listed by up to four neighbouring blocks: grouping keeps neighbours on one L2
    const GridUnit u = units[xcd_group_item(blockIdx.x, gridDim.x, xg)];
    const int lane = threadIdx.x, il = lane & 15, kq = lane >> 4;
    // staging: lane e evaluates both dimensions of entry e of the batch
    const int se = lane;
    const int bx0 = (u.tile % nbx - 1) * GB, by0 = (u.tile / nbx) * GB;   // bx0 = -GB for the margin block
    const int32_t* gl = glist + u.g0;
    const int n = u.gn;
    sA[se * GR_WS] = T(0);
    sA[se * GR_WS + KB_J + 1] = T(0);
    sB[se * GR_WS] = cplx<T>{T(0), T(0)};
    sB[se * GR_WS + KB_J + 1] = cplx<T>{T(0), T(0)};
    // two accumulator pairs (even and odd groups of four entries), so that
    // consecutive products do not wait on each other
    acc_t are0{}, aim0{}, are1{}, aim1{};
    // software pipeline: the next batch's entry data are loaded while this batch
    // is gridded, and the list positions of the one after
    int cc_n = 0;
    cplx<T> f_n{T(0), T(0)};
    cplx<T> val_n{T(0), T(0)};
    T w_n = T(1);
    auto fetch = [&](int p) {
        if (p >= 0) {
            cc_n = cell[p];
            f_n = frac[p];
            val_n = vals[p];
            if (weight) w_n = weight[p];
        }
    };
    int pos_n = se < n ? gl[se] : -1;
    fetch(pos_n);
    int pos_nn = GR_BATCH + se < n ? gl[GR_BATCH + se] : -1;
    for (int base = 0; base < n; base += GR_BATCH) {
        const int pos = pos_n;
        const int cc = cc_n;
        const cplx<T> f = f_n;
        cplx<T> val = val_n;
        const T wt = w_n;
        pos_n = pos_nn;
        fetch(pos_n);
        pos_nn = base + 2 * GR_BATCH + se < n ? gl[base + 2 * GR_BATCH + se] : -1;
        int dy = 2 * GB, dx = 2 * GB;   // an empty slot: every tap falls outside the block
        T wx8[KB_J], wy8[KB_J];
        if (pos >= 0) {
            dy = (cc >> 16) - 3 - by0;
            if (dy < -(KB_J - 1)) dy += Ky;
            if (dy > GB - 1) dy -= Ky;
            dx = (cc & 0x7FFF) - 3 - bx0;   // the half plane has no wrap in x
            kb_weights(f.re, kb, wx8);
            kb_weights(f.im, kb, wy8);
        } else {
#pragma unroll
            for (int j = 0; j < KB_J; ++j) wx8[j] = wy8[j] = T(0);
        }
        if (weight) {
            val.re *= wt;
            val.im *= wt;
        }
        const T vr = val.re, vi = (cc & 0x8000) ? -val.im : val.im;   // reflected: conjugate value
#pragma unroll
        for (int j = 0; j < KB_J; ++j) {
            sA[se * GR_WS + 1 + j] = wy8[j];
            sB[se * GR_WS + 1 + j] = cplx<T>{wx8[j] * vr, wx8[j] * vi};
        }
        sd[se] = int2{dy, dx};
        wave_lds_sync();
        const int ng = (min(GR_BATCH, n - base) + 3) >> 2;
        // row il of A is wy_e(il - dy_e) and column il of B is wx_e(il - dx_e) v_e:
        // the tap index clamped to [-1, KB_J] reads a zero outside the footprint
        auto step = [&](int q, acc_t& are, acc_t& aim) {
            const int e = 4 * q + kq;
            const int2 d = sd[e];
            const int iy = min(max(il - d.x, -1), KB_J) + 1;
            const int ix = min(max(il - d.y, -1), KB_J) + 1;
            const T a = sA[e * GR_WS + iy];
            const cplx<T> b = sB[e * GR_WS + ix];
            are = grid_mfma(a, b.re, are);
            aim = grid_mfma(a, b.im, aim);
        };
        int q = 0;
        for (; q + 1 < ng; q += 2) {
            step(q, are0, aim0);
            step(q + 1, are1, aim1);
        }
        if (q < ng) step(q, are0, aim0);
        wave_lds_sync();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = grid_mfma_row<T>(lane, r);
        const cplx<T> v{are0[r] + are1[r], aim0[r] + aim1[r]};
        if (u.nsplit == 1)
            stnt_c(grid + (size_t)u.l * Ky * Wg + (size_t)(by0 + row) * Wg + GR_MARGIN + bx0 + il, v);
        else
            partial[(size_t)(u.partial + u.split) * GB * GB + row * GB + il] = v;
    }
}

template <typename T>
__global__ void k_grid_merge(const SplitTile* __restrict__ splits, const cplx<T>* __restrict__ partial,
                             cplx<T>* __restrict__ grid, int Ky, int Wg, int nbx) {
    const SplitTile s = splits[blockIdx.x];
    const int bx0 = (s.tile % nbx - 1) * GB, by0 = (s.tile / nbx) * GB;
    cplx<T>* g = grid + (size_t)s.l * Ky * Wg + GR_MARGIN;
    for (int e = threadIdx.x; e < GB * GB; e += blockDim.x) {
        cplx<T> acc{T(0), T(0)};
        for (int k = 0; k < s.nsplit; ++k) {
            const cplx<T> p = partial[(size_t)(s.partial + k) * GB * GB + e];
            acc.re += p.re;
            acc.im += p.im;
        }
        const int ry = e / GB, rx = e - ry * GB;
        g[(size_t)(by0 + ry) * Wg + bx0 + rx] = acc;
    }
}

// ------------------------------------------------------------- reorderings
template <typename T>
__global__ void k_gather_user(const cplx<T>* __restrict__ in_user, const int32_t* __restrict__ perm,
                              const T* __restrict__ theta, cplx<T>* __restrict__ out, int64_t M) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    cplx<T> v = in_user[perm[i]];
    if (theta) {
        const T t = theta[i];
        v.re *= t;
        v.im *= t;
    }
    out[i] = v;
}

template <typename T>
__global__ void k_scatter_user(const cplx<T>* __restrict__ in, const int32_t* __restrict__ perm,
                               cplx<T>* __restrict__ out_user, int64_t M) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    out_user[perm[i]] = in[i];
}

// ------------------------------------------------- exact ball projection (one block)
// z <- argmin_{||q - y|| <= eps} (q - z)^H U (q - z) over the visibilities of one
// block, without bins: FP64 block reductions and Newton from lambda = 0.
__device__ __forceinline__ double wg_sum(double v, double* sh) {
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    return s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_proj_block(cplx<T>* __restrict__ z, const int32_t* __restrict__ vis_pos,
                                                    const cplx<T>* __restrict__ yv, const T* __restrict__ uprec,
                                                    const double* __restrict__ eps_blk, int blk, int64_t pos0,
                                                    int64_t Mb) {
    __shared__ double sh[4];
    const double e = eps_blk[blk];
    double r2 = 0.0, a2 = 0.0;
    for (int64_t i = threadIdx.x; i < Mb; i += blockDim.x) {
        const int g = vis_pos[pos0 + i];
        const cplx<T> zz = z[i], yy = yv[g];
        const double dr = (double)zz.re - (double)yy.re, di = (double)zz.im - (double)yy.im;
        const double uu = (double)uprec[g];
        r2 += dr * dr + di * di;
        a2 += uu * uu * (dr * dr + di * di);
    }
    r2 = wg_sum(r2, sh);
    a2 = wg_sum(a2, sh);
    if (r2 <= e * e) return;   // already inside: q = z
    double lam = 0.0;
    if (e > 0.0) {
        const double hi = sqrt(a2) / e;
        for (int it = 0; it < 200; ++it) {
            double f = 0.0, fp = 0.0;
            for (int64_t i = threadIdx.x; i < Mb; i += blockDim.x) {
                const int g = vis_pos[pos0 + i];
                const cplx<T> zz = z[i], yy = yv[g];
                const double dr = (double)zz.re - (double)yy.re, di = (double)zz.im - (double)yy.im;
                const double uu = (double)uprec[g];
                const double q = 1.0 / (uu + lam);
                const double t = uu * uu * (dr * dr + di * di) * q * q;
                f += t;
                fp += t * q;
            }
            f = wg_sum(f, sh) - e * e;
            fp = -2.0 * wg_sum(fp, sh);
            if (f <= 1e-15 * e * e) break;
            double nl = lam - f / fp;
            if (!(nl > lam)) break;
            if (nl > hi) nl = hi;
            if (nl - lam <= 1e-16 * nl) { lam = nl; break; }
            lam = nl;
        }
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < Mb; i += blockDim.x) {
        const int g = vis_pos[pos0 + i];
        const cplx<T> zz = z[i], yy = yv[g];
        const double uu = (double)uprec[g];
        const double f = (e > 0.0) ? uu / (uu + lam) : 0.0;
        z[i] = {(T)((double)yy.re + f * ((double)zz.re - (double)yy.re)),
                (T)((double)yy.im + f * ((double)zz.im - (double)yy.im))};
    }
}

// ------------------------------------------------------------------ launchers
// Kernel-argument form of the plan's per-tap coefficients ([4][deg + 1] in t).
template <typename T>
static KBPoly<T> kbpoly(const hs_ctx* c) {
    KBPoly<T> p{};
    constexpr int n = KBDeg<T>::n + 1;
    for (int j = 0; j < 4; ++j) {
        for (int k = 0; k < KBPoly<T>::NE; ++k) p.e[j][k] = (T)c->kb_c[(size_t)j * n + 2 * k];
        for (int k = 0; k < KBPoly<T>::NO; ++k) p.o[j][k] = (T)c->kb_c[(size_t)j * n + 2 * k + 1];
    }
    return p;
}

static inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
void launch_degrid_plain(hs_ctx* c, cplx<T>* out_user, int lc) {
    int64_t u0, nu;
    chan_range(c->dunit_off, lc, u0, nu);
    if (nu == 0) return;
    const size_t lds = (size_t)(c->T + 8) * deg_stride(c->T) * sizeof(cplx<T>);
    k_degrid_plain<T, true, false><<<(unsigned)nu, DEG_THREADS, lds, c->stream>>>(
        c->d.dunits + u0, c->d.vis_cell, (const cplx<T>*)c->d.vis_frac, (const cplx<T>*)c->d.grid,
        (const T*)c->d.vis_theta, nullptr, c->d.vis_perm, out_user, c->Kh, c->Ky, c->Wg, c->T, c->tiles_x,
        kbpoly<T>(c), c->deg_group);
}

// Degrid into grid order with an extra per-visibility factor (used by the power iteration).
template <typename T>
void launch_degrid_grid_order(hs_ctx* c, cplx<T>* out, const T* mult, int lc) {
    int64_t u0, nu;
    chan_range(c->dunit_off, lc, u0, nu);
    if (nu == 0) return;
    const size_t lds = (size_t)(c->T + 8) * deg_stride(c->T) * sizeof(cplx<T>);
    auto launch = [&](auto kern) {
        kern<<<(unsigned)nu, DEG_THREADS, lds, c->stream>>>(
            c->d.dunits + u0, c->d.vis_cell, (const cplx<T>*)c->d.vis_frac, (const cplx<T>*)c->d.grid,
            (const T*)c->d.vis_theta, mult, nullptr, out, c->Kh, c->Ky, c->Wg, c->T, c->tiles_x, kbpoly<T>(c),
            c->deg_group);
    };
    if (mult) launch(k_degrid_plain<T, false, true>);
    else launch(k_degrid_plain<T, false, false>);
}

template <typename T>
void launch_degrid_dual_v(hs_ctx* c, cplx<T>* v, int lc) {
    int64_t u0, nu;
    chan_range(c->dunit_off, lc, u0, nu);
    if (nu == 0) return;
    const size_t lds = (size_t)(c->T + 8) * deg_stride(c->T) * sizeof(cplx<T>);
    k_degrid_dual<T><<<(unsigned)nu, DEG_THREADS, lds, c->stream>>>(
        c->d.dunits + u0, c->d.vis_cell, (const cplx<T>*)c->d.vis_frac, (const cplx<T>*)c->d.grid,
        (const T*)c->d.vis_theta, (const T*)c->d.vis_u, (const cplx<T>*)c->d.vis_y, c->d.vis_bin, v,
        c->d.chunk_run, c->d.run_slot, c->d.run_sum, c->Kh, c->Ky, c->Wg, c->T, c->tiles_x, kbpoly<T>(c),
        c->deg_group);
}

template <typename T>
void launch_bins_and_roots(hs_ctx* c, int lc) {
    int64_t b0, nbn;
    chan_range(c->bin_off, lc, b0, nbn);
    const int64_t k0 = lc < 0 ? 0 : c->blk_off[lc];
    const int64_t nk = lc < 0 ? c->nblk : c->blk_off[lc + 1] - c->blk_off[lc];
    if (nbn > 0)
        k_bin_reduce<<<nblocks(nbn * 64, 256), 256, 0, c->stream>>>(c->d.bin_run_ptr + b0, c->d.run_sum,
                                                                     c->d.bin_S + 2 * b0, (int)nbn);
    if (nk > 0)
        k_block_roots<<<nblocks(nk * 64, 256), 256, 0, c->stream>>>(
            c->d.blk_bin_ptr + k0, c->d.bin_S, c->d.bin_u, c->d.bin_f, c->dtype == HS_F32 ? 1 : 0, c->d.blk_eps + k0,
            c->d.blk_lambda + k0, c->d.blk_rho2 + k0, c->d.blk_vartheta + k0,
            c->d.scal, (int)nk, c->adaptive ? 1 : 0, c->lam1, c->lam2, c->lam3, c->vartheta_bar);
}

template <typename T>
void launch_dual_apply_v(hs_ctx* c, cplx<T>* v, int lc) {
    int64_t m0, nm;
    chan_range(c->chan_off, lc, m0, nm);
    if (nm == 0) return;
    if (m0 % 2 == 0)
        k_dual_apply2<T><<<nblocks((nm + 1) / 2, 256), 256, 0, c->stream>>>(v + m0, c->d.vis_bin + m0, c->d.bin_f, nm);
    else
        k_dual_apply<T><<<nblocks(nm, 256), 256, 0, c->stream>>>(v + m0, c->d.vis_bin + m0, c->d.bin_f, nm);
}

template <typename T>
void launch_grid_pull(hs_ctx* c, const cplx<T>* vals, const T* weight, int lc) {
    int64_t g0, ng, s0, ns;
    chan_range(c->gunit_off, lc, g0, ng);
    chan_range(c->split_off, lc, s0, ns);
    if (ng > 0)
        k_grid_pull<T><<<(unsigned)ng, 64, 0, c->stream>>>(
            c->d.gunits + g0, c->d.glist, c->d.vis_cell, (const cplx<T>*)c->d.vis_frac, vals, weight,
            (cplx<T>*)c->d.grid, (cplx<T>*)c->d.gpartial, c->Ky, c->Wg, c->gtiles_x, kbpoly<T>(c), c->grid_group);
    if (ns > 0)
        k_grid_merge<T><<<(unsigned)ns, 256, 0, c->stream>>>(
            c->d.splits + s0, (const cplx<T>*)c->d.gpartial, (cplx<T>*)c->d.grid, c->Ky, c->Wg, c->gtiles_x);
}

template <typename T>
void launch_proj_block(hs_ctx* c, int64_t pos0, int64_t Mb, int blk, cplx<T>* z) {
    k_proj_block<T><<<1, 256, 0, c->stream>>>(z, c->d.vis_pos, (const cplx<T>*)c->d.vis_y, (const T*)c->d.vis_u,
                                             c->d.blk_eps, blk, pos0, Mb);
}

template <typename T>
void launch_gather_user(hs_ctx* c, const cplx<T>* in_user, cplx<T>* out_grid, bool times_theta) {
    if (c->Mtot == 0) return;
    k_gather_user<T><<<nblocks(c->Mtot, 256), 256, 0, c->stream>>>(
        in_user, c->d.vis_perm, times_theta ? (const T*)c->d.vis_theta : nullptr, out_grid, c->Mtot);
}

template <typename T>
void launch_scatter_user(hs_ctx* c, const cplx<T>* in_grid, cplx<T>* out_user) {
    if (c->Mtot == 0) return;
    k_scatter_user<T><<<nblocks(c->Mtot, 256), 256, 0, c->stream>>>(in_grid, c->d.vis_perm, out_user, c->Mtot);
}

#define HS_INST(T)                                                                          \
    template void launch_fft_rows_fwd<T>(hs_ctx*, const T*, int, int);                      \
    template void launch_fft_cols_fwd<T>(hs_ctx*, int, int);                                \
    template void launch_fft_cols_adj<T>(hs_ctx*, int, int);                                \
    template void launch_fft_rows_adj<T>(hs_ctx*, T*, int, int);                            \
    template void launch_degrid_plain<T>(hs_ctx*, cplx<T>*, int);                           \
    template void launch_degrid_grid_order<T>(hs_ctx*, cplx<T>*, const T*, int);            \
    template void launch_degrid_dual_v<T>(hs_ctx*, cplx<T>*, int);                          \
    template void launch_bins_and_roots<T>(hs_ctx*, int);                                   \
    template void launch_dual_apply_v<T>(hs_ctx*, cplx<T>*, int);                           \
    template void launch_proj_block<T>(hs_ctx*, int64_t, int64_t, int, cplx<T>*);           \
    template void launch_grid_pull<T>(hs_ctx*, const cplx<T>*, const T*, int);              \
    template void launch_gather_user<T>(hs_ctx*, const cplx<T>*, cplx<T>*, bool);           \
    template void launch_scatter_user<T>(hs_ctx*, const cplx<T>*, cplx<T>*);
HS_INST(float)
HS_INST(double)
#undef HS_INST

}  // namespace hs
