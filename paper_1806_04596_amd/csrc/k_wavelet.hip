// SARA dictionary Psi = (Dirac, db1..db8) (Sec. 2.3) and the joint-average-sparsity
// l2,1 dual update (Algorithm 2; eq:prox-L21).
//
// Each Daubechies basis is the periodised orthonormal 2-D Mallat transform.  One
// launch covers every (basis, channel) pair of one level and one direction, so a
// level costs two coalesced passes (rows along x, then columns along y) over
// the LL region of all n_db * L images.  Synthesis runs coarse to fine through a
// scratch pyramid and the final sum over bases is a single fused pass.
#include "hs_internal.h"

namespace hs {

// filt: [n_db][2][16] (h then g, zero padded), basis b = db(b+1) with 2(b+1) taps.
//
// Analysis, one launch per level: a work item is a TB x TB tile of each of the
// four subbands of one channel (and one basis, below level 0); its
// (2TB + 14)^2 input window (periodic wrap) is staged in LDS, filtered along
// rows then columns in LDS, and the three detail subbands go to their Mallat
// positions; the approximation goes to a compact buffer for the next level (or
// to its Mallat place at the last level).  At level 0 the input X is shared by
// every basis, so one item loops over the bases and reads X once.  Work-groups
// loop over items and load the next item's window into registers while the
// current one is filtered.
constexpr int WV_TB = 16;   // analysis output tile per subband
constexpr int WV_TO = 32;   // synthesis output tile
constexpr int WV_HALO = 14; // 2 * 8 - 2
constexpr int WV_W = WV_TO / 2 + 8;   // synthesis coefficient window per subband
constexpr int64_t IDWT_MIN_WG = 2048;  // smallest synthesis grid worth looping bases for

// Tile of work item t (of n): work-groups are dispatched round-robin over the 8
// XCDs, each with its own L2, so t mod 8 names the XCD; when n is a multiple of 8
// each XCD takes a contiguous band of n/8 tiles (whole tile rows), so the halo a
// tile shares with its neighbours is read through the same L2.
__device__ __forceinline__ int xcd_band(int t, int n) {
    return (n & 7) ? t : (t & 7) * (n >> 3) + (t >> 3);
}

// k mod n for 0 <= k < 2n + W (one subtraction in the usual case; small
// coarse levels fall back to the remainder).
__device__ __forceinline__ int wrap_idx(int k, int n) {
    if (k >= n) k -= n;
    if (k >= n) k %= n;
    return k;
}

// Filter taps of basis b (db(b+1): NT = 2(b+1) taps); the loops below are
// unrolled per NT, so the coefficients are uniform (scalar) operands.
#define WV_DISPATCH(b, FN, ...)                         \
    switch (b) {                                        \
        case 0: FN<T, 2>(__VA_ARGS__); break;           \
        case 1: FN<T, 4>(__VA_ARGS__); break;           \
        case 2: FN<T, 6>(__VA_ARGS__); break;           \
        case 3: FN<T, 8>(__VA_ARGS__); break;           \
        case 4: FN<T, 10>(__VA_ARGS__); break;          \
        case 5: FN<T, 12>(__VA_ARGS__); break;          \
        case 6: FN<T, 14>(__VA_ARGS__); break;          \
        default: FN<T, 16>(__VA_ARGS__); break;         \
    }

constexpr int WV_WI = 2 * WV_TB + WV_HALO;   // analysis input window edge

// Analysis rows: a | d for every needed input row (2 TB + NT - 2 rows).
template <typename T, int NT>
__device__ __forceinline__ void dwt_rows(const T* __restrict__ f, const T (*inS)[WV_WI + 1], T (*tmpS)[2 * WV_TB + 1]) {
    constexpr int TB = WV_TB, NR = 2 * TB + NT - 2;
    T h[NT], g[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        h[j] = f[j];
        g[j] = f[16 + j];
    }
    for (int e = threadIdx.x; e < NR * TB; e += blockDim.x) {
        const int r = e / TB, kx = e - r * TB;
        T a = T(0), d = T(0);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const T x = inS[r][2 * kx + j];
            a += h[j] * x;
            d += g[j] * x;
        }
        tmpS[r][kx] = a;
        tmpS[r][TB + kx] = d;
    }
}

// Analysis columns: the four subbands of output (ky, kx), written to their places.
template <typename T, int NT>
__device__ __forceinline__ void dwt_cols(const T* __restrict__ f, const T (*tmpS)[2 * WV_TB + 1], T* __restrict__ cb,
                                         T* __restrict__ llb, int ky0, int kx0, int hx, int hy, int nx, int last) {
    constexpr int TB = WV_TB;
    T h[NT], g[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        h[j] = f[j];
        g[j] = f[16 + j];
    }
    for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) {
        const int ky = e / TB, kx = e - ky * TB;
        T aa = T(0), da = T(0), ad = T(0), dd = T(0);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const T lo = tmpS[2 * ky + j][kx], hi = tmpS[2 * ky + j][TB + kx];
            aa += h[j] * lo;
            da += g[j] * lo;
            ad += h[j] * hi;
            dd += g[j] * hi;
        }
        const int gy = ky0 + ky, gx = kx0 + kx;
        if (gy < hy && gx < hx) {
            cb[(size_t)gy * nx + hx + gx] = ad;
            cb[(size_t)(hy + gy) * nx + gx] = da;
            cb[(size_t)(hy + gy) * nx + hx + gx] = dd;
            if (last) cb[(size_t)gy * nx + gx] = aa;
            else llb[(size_t)gy * hx + gx] = aa;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_dwt_level(const T* __restrict__ X, const T* __restrict__ llin,
                                                   T* __restrict__ coef, T* __restrict__ llout,
                                                   const T* __restrict__ filt, int L, int nx, int ny, int mx, int my,
                                                   int lev0, int last, int n_db) {
    constexpr int TB = WV_TB, WI = WV_WI, NW = (WI * WI + 255) / 256;
    __shared__ T inS[WI][WI + 1];
    __shared__ T tmpS[WI][2 * TB + 1];
    const int hx = mx >> 1, hy = my >> 1;
    const int ntx = (hx + TB - 1) / TB, nty = (hy + TB - 1) / TB, ntiles = ntx * nty;
    const size_t N = (size_t)nx * ny;
    const int tid = threadIdx.x;
    // work items: (tile, channel) at level 0 (all bases share the window), else (tile, channel, basis)
    const int nitems = ntiles * L * (lev0 ? 1 : n_db);
    T win[NW];
    auto fetch = [&](int item) {
        const int tile = xcd_band(item % ntiles, ntiles), rest = item / ntiles;
        const int l = rest % L, b = rest / L;
        const int ky0 = (tile / ntx) * TB, kx0 = (tile % ntx) * TB;
        const T* src = lev0 ? X + (size_t)l * N : llin + ((size_t)b * L + l) * (size_t)my * mx;
        const int stride = lev0 ? nx : mx;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int e = tid + 256 * k;
            if (e < WI * WI) {
                const int r = e / WI, cc = e - r * WI;
                const int gy = wrap_idx(2 * ky0 + r, my), gx = wrap_idx(2 * kx0 + cc, mx);
                win[k] = src[(size_t)gy * stride + gx];
            }
        }
    };
    int item = blockIdx.x;
    if (item < nitems) fetch(item);
    for (; item < nitems; item += gridDim.x) {
        const int tile = xcd_band(item % ntiles, ntiles), rest = item / ntiles;
        const int l = rest % L;
        const int ky0 = (tile / ntx) * TB, kx0 = (tile % ntx) * TB;
        const int b_first = lev0 ? 0 : rest / L;
        const int b_last = lev0 ? n_db : b_first + 1;
        __syncthreads();   // the previous item is done with inS and tmpS
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int e = tid + 256 * k;
            if (e < WI * WI) inS[e / WI][e % WI] = win[k];
        }
        __syncthreads();
        if (item + (int)gridDim.x < nitems) fetch(item + gridDim.x);   // in flight during the filters
        for (int b = b_first; b < b_last; ++b) {
            if (b != b_first) __syncthreads();
            const T* f = filt + b * 32;
            WV_DISPATCH(b, dwt_rows, f, inS, tmpS)
            __syncthreads();
            T* cb = coef + ((size_t)b * L + l) * N;
            T* llb = llout + ((size_t)b * L + l) * (size_t)hy * hx;
            WV_DISPATCH(b, dwt_cols, f, tmpS, cb, llb, ky0, kx0, hx, hy, nx, last)
        }
    }
}

// Synthesis, one launch per level (coarse to fine): a workgroup owns a TO x TO
// tile of the synthesised region, stages windows of the four subbands
// (approximation from the coarser synthesis, or from C at the coarsest level),
// inverts along y then x in LDS, and writes a compact approximation for the
// next finer level.  At level 0 it loops over the bases and writes
// Xout = C0 + sum_b Psi_b C_b once.  Outputs 2p and 2p + 1 of a filter pass
// read the same coefficients (even taps for the first, odd for the second).
// Each thread owns a short run of adjacent outputs: it reads the coefficients
// the run needs once into registers and forms every output as a chain of
// FMAs, so the inner loops carry no index arithmetic.

// Column (y) inverse: thread t < 192 owns x-subband sx, window column wx and
// the output rows 2p, 2p + 1 for p in [p0, p0 + 4).
constexpr int IDWT_YP = 4;
template <typename T, int NT>
__device__ __forceinline__ void idwt_y(const T* __restrict__ f, const T (*S)[WV_W][WV_W + 1],
                                       T (*Tm)[WV_TO][WV_W + 1], int sx, int wx, int p0) {
    constexpr int NH = NT / 2, NR = NH + IDWT_YP - 1;
    T a[NR], d[NR];
    const int r0 = p0 + 9 - NH;   // first window row of the run
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        a[k] = S[sx][r0 + k][wx];
        d[k] = S[2 + sx][r0 + k][wx];
    }
#pragma unroll
    for (int j = 0; j < IDWT_YP; ++j) {
        T xe = T(0), xo = T(0);
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const int k = j - i + NH - 1;   // row p0 + j - i + 8
            xe = fma(f[2 * i], a[k], xe);
            xe = fma(f[16 + 2 * i], d[k], xe);
            xo = fma(f[2 * i + 1], a[k], xo);
            xo = fma(f[16 + 2 * i + 1], d[k], xo);
        }
        Tm[sx][2 * (p0 + j)][wx] = xe;
        Tm[sx][2 * (p0 + j) + 1][wx] = xo;
    }
}

// Row (x) inverse: thread t owns output row m and columns 2q0 .. 2q0 + 3.
template <typename T, int NT>
__device__ __forceinline__ void idwt_x(const T* __restrict__ f, const T (*Tm)[WV_TO][WV_W + 1], int m, int q0,
                                       T (&res)[4]) {
    constexpr int NH = NT / 2, NC = NH + 1;
    T a[NC], d[NC];
    const int c0 = q0 + 9 - NH;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        a[k] = Tm[0][m][c0 + k];
        d[k] = Tm[1][m][c0 + k];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        T xe = T(0), xo = T(0);
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const int k = j - i + NH - 1;   // column q0 + j - i + 8
            xe = fma(f[2 * i], a[k], xe);
            xe = fma(f[16 + 2 * i], d[k], xe);
            xo = fma(f[2 * i + 1], a[k], xo);
            xo = fma(f[16 + 2 * i + 1], d[k], xo);
        }
        res[2 * j] = xe;
        res[2 * j + 1] = xo;
    }
}

template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 6))) void k_idwt_level(const T* __restrict__ C, const T* __restrict__ llin,
                                                    T* __restrict__ out, const T* __restrict__ C0,
                                                    const T* __restrict__ filt, int L, int nx, int ny, int mx, int my,
                                                    int coarsest, int final_level, int n_db, int bpw) {
    constexpr int TO = WV_TO, W = WV_W;
    static_assert(TO * TO == 4 * 256, "four outputs per thread");
    static_assert(2 * W * (TO / 2) == IDWT_YP * 192, "y runs on three waves");
    __shared__ T S[4][W][W + 1];           // subband (sy*2 + sx)
    __shared__ T Tm[2][TO][W + 1];         // after the column inverse, per x-subband
    const int hx = mx >> 1, hy = my >> 1;
    const int ntx = (mx + TO - 1) / TO;
    const int tile = xcd_band(blockIdx.x, gridDim.x);
    const int m0y = (tile / ntx) * TO, m0x = (tile % ntx) * TO;
    const int l = blockIdx.y;
    const size_t N = (size_t)nx * ny;
    const int tid = threadIdx.x;
    int kylo = (m0y / 2 - 8) % hy;
    if (kylo < 0) kylo += hy;
    int kxlo = (m0x / 2 - 8) % hx;
    if (kxlo < 0) kxlo += hx;
    // thread roles in the two filter passes
    const bool ylive = tid < 192;
    const int yc = tid % 48, ysx = yc / W, ywx = yc - ysx * W, yp0 = (tid / 48) * IDWT_YP;
    const int xm = tid >> 3, xq0 = 2 * (tid & 7);
    T acc[4] = {T(0), T(0), T(0), T(0)};
    const int b_first = final_level ? 0 : (int)blockIdx.z * bpw;
    const int b_last = final_level ? n_db : min(b_first + bpw, n_db);
    // This thread's window elements: the same offsets in every basis, computed once.
    // Element i comes from the coarser approximation (llin) when it is in subband 0
    // below the coarsest level, else from the coefficient image.
    constexpr int NE = (4 * W * W + 255) / 256;
    int off[NE];
    unsigned from_ll = 0u, live = 0u;
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        const int e = tid + 256 * i;
        off[i] = 0;
        if (e < 4 * W * W) {
            const int sb = e / (W * W), rem = e - sb * (W * W);
            const int r = rem / W, cc = rem - r * W;
            const int sy = sb >> 1, sx = sb & 1;
            const int ky = wrap_idx(kylo + r, hy), kx = wrap_idx(kxlo + cc, hx);
            live |= 1u << i;
            if (sb == 0 && !coarsest) {
                from_ll |= 1u << i;
                off[i] = ky * hx + kx;
            } else {
                off[i] = (sy * hy + ky) * nx + sx * hx + kx;
            }
        }
    }
    // the window of the next basis is loaded into registers while this one is filtered
    T nxt[NE];
    auto fetch = [&](int b) {
        const T* Cb = C + ((size_t)b * L + l) * N;
        const T* LLb = coarsest ? Cb : llin + ((size_t)b * L + l) * (size_t)hy * hx;
#pragma unroll
        for (int i = 0; i < NE; ++i)
            if ((live >> i) & 1u) nxt[i] = ((from_ll >> i) & 1u) ? LLb[off[i]] : Cb[off[i]];
    };
    fetch(b_first);
    for (int b = b_first; b < b_last; ++b) {
        T* Sf = &S[0][0][0];
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            const int e = tid + 256 * i;
            if ((live >> i) & 1u) {
                const int sb = e / (W * W), rem = e - sb * (W * W);
                Sf[(sb * W + rem / W) * (W + 1) + rem % W] = nxt[i];
            }
        }
        __syncthreads();
        if (b + 1 < b_last) fetch(b + 1);
        const T* f = filt + b * 32;
        if (ylive) {
            WV_DISPATCH(b, idwt_y, f, S, Tm, ysx, ywx, yp0)
        }
        __syncthreads();
        T res[4];
        WV_DISPATCH(b, idwt_x, f, Tm, xm, xq0, res)
        if (final_level) {
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] += res[k];
        } else {
            const int gy = m0y + xm, gx = m0x + 2 * xq0;
            T* o = out + ((size_t)b * L + l) * (size_t)my * mx + (size_t)gy * mx + gx;
            if (gy < my) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (gx + k < mx) o[k] = res[k];
            }
        }
        __syncthreads();
    }
    if (final_level) {
        // mx is a power of two, so for mx >= 4 the four outputs are all in or all out
        const int gy = m0y + xm, gx = m0x + 2 * xq0;
        const size_t idx = (size_t)l * N + (size_t)gy * nx + gx;
        if (gy < my && mx >= 4 && gx < mx) {
            T v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = (C0 ? C0[idx + k] : T(0)) + acc[k];
#pragma unroll
            for (int k = 0; k < 4; ++k) out[idx + k] = v[k];
        } else if (gy < my) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (gx + k < mx) out[idx + k] = (C0 ? C0[idx + k] : T(0)) + acc[k];
        }
    }
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
//  mode 0 (dual update): Z = A + Psi_d^dag Xt, A <- Z min(1, thr*wbar/||Z||);
//  mode 1 (prox, eq:prox-L21): Z = A, A <- Z max(||Z|| - thr*wbar, 0)/||Z||;
//  mode 2 (dual of the per-channel weighted l1 of the SARA variant, eq:min-sara):
//         Z = A + Psi_d^dag Xt, A <- clip(Z, -thr*wbar, thr*wbar) element by element,
//         one weight per channel and coefficient (wbar [D][L][N]).
template <typename T, bool HAS_S>
__global__ __launch_bounds__(256) void k_l21(T* __restrict__ A, const T* __restrict__ Xt, const T* __restrict__ coef,
                      const T* __restrict__ wbar, double thr, int L, int64_t N, int mode) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int d = blockIdx.y;
    T* Ad = A + (size_t)d * L * N + p;
    const T* Sd = HAS_S ? ((d == 0) ? Xt + p : coef + (size_t)(d - 1) * L * N + p) : nullptr;
    if (mode == 2) {
        // SARA variant: weighted l1 per channel (weights wbar[d][l][p]), Z - soft(Z) =
        // clip(Z, -t, t) element by element
        for (int l = 0; l < L; ++l) {
            const T t = (T)(thr * (wbar ? (double)wbar[((size_t)d * L + l) * N + p] : 1.0));
            const T v = Ad[(size_t)l * N] + (HAS_S ? Sd[(size_t)l * N] : T(0));
            Ad[(size_t)l * N] = v > t ? t : (v < -t ? -t : v);
        }
        return;
    }
    // every channel's loads are issued together (clamped channel index; channels
    // >= L are never used), then the row norm and the shrink
    T z[MAX_L], z2[MAX_L];
#pragma unroll
    for (int l = 0; l < MAX_L; ++l) {
        const size_t o = (size_t)(l < L ? l : L - 1) * N;
        z[l] = Ad[o];
        if (HAS_S) z2[l] = Sd[o];
    }
    double n2 = 0.0;
#pragma unroll
    for (int l = 0; l < MAX_L; ++l) {
        if (l < L) {
            if (HAS_S) z[l] += z2[l];
            n2 += (double)z[l] * (double)z[l];
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
// Intermediate approximations live in two compact slots of wtmp.
template <typename T>
void launch_psi_adj(hs_ctx* c, const T* X, T* Cout, int nl) {
    if (c->n_db == 0) return;
    const int L = nl > 0 ? nl : c->L;   // channels of X and Cout (the scratch slots hold c->L)
    T* out = Cout ? Cout : (T*)c->d.coef;
    T* slotA = (T*)c->d.wtmp;
    T* slotB = slotA + (size_t)c->n_db * c->L * (c->N / 4);
    const T* filt = (const T*)c->d.filt;
    const T* llin = nullptr;
    for (int lev = 0; lev < c->levels; ++lev) {
        const int mx = c->nx >> lev, my = c->ny >> lev;
        const int hx = mx / 2, hy = my / 2;
        const int tiles = ((hy + WV_TB - 1) / WV_TB) * ((hx + WV_TB - 1) / WV_TB);
        T* llout = (lev % 2 == 0) ? slotA : slotB;
        const int last = (lev == c->levels - 1) ? 1 : 0;
        const int items = tiles * L * (lev == 0 ? 1 : c->n_db);
        dim3 g(std::min(items, 4096));
        k_dwt_level<T><<<g, 256, 0, c->stream>>>(X, llin, out, llout, filt, L, c->nx, c->ny, mx, my,
                                                 lev == 0 ? 1 : 0, last, c->n_db);
        llin = llout;
    }
}

// Xout = C0 + sum_b Psi_b Cdb[b]; C0 (Dirac coefficients) may be null.
template <typename T>
void launch_psi_sum(hs_ctx* c, const T* Cdb, const T* C0, T* Xout, int nl) {
    const int L = nl > 0 ? nl : c->L;   // channels of the coefficients and Xout
    const int64_t LN = (int64_t)L * c->N;
    if (c->n_db == 0) {
        k_psi_sum<T><<<nblk(LN, 256), 256, 0, c->stream>>>(nullptr, C0, Xout, 0, LN);
        return;
    }
    T* slotA = (T*)c->d.wtmp;
    T* slotB = slotA + (size_t)c->n_db * c->L * (c->N / 4);
    const T* filt = (const T*)c->d.filt;
    const T* llin = nullptr;
    for (int lev = c->levels - 1; lev >= 0; --lev) {
        const int mx = c->nx >> lev, my = c->ny >> lev;
        const int tiles = ((my + WV_TO - 1) / WV_TO) * ((mx + WV_TO - 1) / WV_TO);
        const int fin = (lev == 0) ? 1 : 0;
        T* out = fin ? Xout : ((lev % 2 == 1) ? slotA : slotB);
        // bases per work-group: as many as keep the grid at IDWT_MIN_WG or more, so the
        // next basis's window is fetched while this one is filtered
        int bpw = 1;
        while (!fin && bpw < c->n_db && (int64_t)tiles * L * ((c->n_db + 2 * bpw - 1) / (2 * bpw)) >= IDWT_MIN_WG)
            bpw *= 2;
        const int nz = fin ? 1 : (c->n_db + bpw - 1) / bpw;
        dim3 g(tiles, L, nz);
        k_idwt_level<T><<<g, 256, 0, c->stream>>>(Cdb, llin, out, C0, filt, L, c->nx, c->ny, mx, my,
                                                  lev == c->levels - 1 ? 1 : 0, fin, c->n_db, bpw);
        llin = out;
    }
}

template <typename T>
void launch_l21_dual(hs_ctx* c, T* A, const T* Xt, const T* coef, const T* wbar, double thr, int mode) {
    dim3 g(nblk(c->N, 256), c->D);
    if (mode != 1) k_l21<T, true><<<g, 256, 0, c->stream>>>(A, Xt, coef, wbar, thr, c->L, c->N, mode);
    else k_l21<T, false><<<g, 256, 0, c->stream>>>(A, Xt, coef, wbar, thr, c->L, c->N, mode);
}

#define HS_INST(T)                                                                   \
    template void launch_psi_adj<T>(hs_ctx*, const T*, T*, int);                     \
    template void launch_psi_sum<T>(hs_ctx*, const T*, const T*, T*, int);           \
    template void launch_l21_dual<T>(hs_ctx*, T*, const T*, const T*, const T*, double, int);
HS_INST(float)
HS_INST(double)
#undef HS_INST

}  // namespace hs
