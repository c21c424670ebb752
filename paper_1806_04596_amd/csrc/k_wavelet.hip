// SARA dictionary Psi = (Dirac, db1..db8) (Sec. 2.3) and the joint-average-sparsity
// l2,1 dual update (Algorithm 2; eq:prox-L21).
//
// Each Daubechies basis is the periodised orthonormal 2-D Mallat transform.  One
// launch covers every (basis, channel) pair of one level and one direction; a
// work-group filters one tile along rows then columns in LDS, so each level reads
// its input and writes its output once (plus the tile halos, read through the
// L2).  Synthesis runs coarse to fine through a scratch pyramid, and its finest
// level sums the bases and the Dirac term in the same pass.
#include "hs_internal.h"

namespace hs {

// filt: [n_db][2][16] (h then g, zero padded), basis b = db(b+1) with 2(b+1) taps.
//
// Analysis, one launch per level: a work item is a TB x TB tile of each of the
// four subbands of one channel (and one basis, below level 0); its
// (2TB + NT - 2)^2 input window (periodic wrap) is staged in LDS with 16-byte
// loads, filtered along rows then columns in LDS, and the three detail subbands
// go to their Mallat positions; the approximation goes to a compact buffer for
// the next level (or to its Mallat place at the last level).  At level 0 the
// input X is shared by every basis, so one item loops over the bases and reads X
// once.  Work-groups loop over items and load the next item's window into
// registers while the current one is filtered.
//
// Both filter passes are register-blocked: a thread reads the inputs of a run of
// adjacent outputs once (16-byte LDS reads along rows) and forms every output of
// the run as an FMA chain with uniform (scalar) taps, so the unrolled loops carry
// no index arithmetic.  Row pass: runs of 4 outputs (a and d) along a row.
// Column pass: runs of TB^2/128 outputs down a column, one task per thread.
constexpr int WV_HALO = 14; // 2 * 8 - 2
constexpr int64_t IDWT_MIN_WG = 2048;  // smallest synthesis grid worth looping bases for

template <typename T> struct Pack16;
template <> struct Pack16<float> { using type = float4; static constexpr int n = 4; };
template <> struct Pack16<double> { using type = double2; static constexpr int n = 2; };

// 16-byte LDS / global accesses of n = 16 / sizeof(T) consecutive elements
template <typename T>
__device__ __forceinline__ void ld16(const T* p, T* out) {
    const typename Pack16<T>::type v = *reinterpret_cast<const typename Pack16<T>::type*>(p);
    if constexpr (Pack16<T>::n == 4) { out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w; }
    else { out[0] = v.x; out[1] = v.y; }
}
template <typename T>
__device__ __forceinline__ void st16(T* p, const T* in) {
    typename Pack16<T>::type v;
    if constexpr (Pack16<T>::n == 4) { v.x = in[0]; v.y = in[1]; v.z = in[2]; v.w = in[3]; }
    else { v.x = in[0]; v.y = in[1]; }
    *reinterpret_cast<typename Pack16<T>::type*>(p) = v;
}

// Analysis tiling per precision: TB outputs per subband and dimension, LDS row
// strides SI (input window) and ST (row-filtered a | d), multiples of 16 bytes.
template <typename T> struct DwtCfg;
template <> struct DwtCfg<float> { static constexpr int TB = 32, SI = 84, ST = 68; };
template <> struct DwtCfg<double> { static constexpr int TB = 16, SI = 50, ST = 34; };

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

// Analysis rows: a | d for every window row the column pass needs (2 TB + NT - 2
// rows).  Task (r, q): outputs 4q .. 4q + 3 of row r from inputs 8q .. 8q + NT + 5.
template <typename T, int NT>
__device__ __forceinline__ void dwt_rows(const T* __restrict__ f, const T* inS, T* tmpS) {
    using C = DwtCfg<T>;
    constexpr int TB = C::TB, R = 4, RUNS = TB / R, NR = 2 * TB + NT - 2;
    constexpr int VW = Pack16<T>::n, NX = 2 * R + NT - 2, NXV = (NX + VW - 1) / VW * VW;
    static_assert(2 * R * (RUNS - 1) + NXV <= C::SI, "row reads stay inside the padded row");
    for (int t = threadIdx.x; t < NR * RUNS; t += 256) {
        const int r = t / RUNS, q = t % RUNS;
        const T* src = inS + r * C::SI + 2 * R * q;
        T x[NXV];
#pragma unroll
        for (int k = 0; k < NXV; k += VW) ld16(src + k, x + k);
        T a[R], d[R];
#pragma unroll
        for (int o = 0; o < R; ++o) {
            T sa = T(0), sd = T(0);
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                sa = fma(f[j], x[2 * o + j], sa);
                sd = fma(f[16 + j], x[2 * o + j], sd);
            }
            a[o] = sa;
            d[o] = sd;
        }
        T* dst = tmpS + r * C::ST + R * q;
#pragma unroll
        for (int k = 0; k < R; k += VW) {
            st16(dst + k, a + k);
            st16(dst + TB + k, d + k);
        }
    }
}

// Analysis columns: thread t owns column c = t mod 2TB of the row-filtered tile (a
// for c < TB, d above) and the run of RC = TB^2/128 output rows starting at
// RC (t / 2TB); the low-pass of the run goes to LL (a) or to the (low y, high x)
// subband (d), the high-pass to (high y, low x) or (high y, high x).
template <typename T, int NT>
__device__ __forceinline__ void dwt_cols(const T* __restrict__ f, const T* tmpS, T* __restrict__ cb,
                                         T* __restrict__ llb, int ky0, int kx0, int hx, int hy, int nx, int last) {
    using C = DwtCfg<T>;
    constexpr int TB = C::TB, RC = TB * TB / 128, NX = 2 * RC + NT - 2;
    static_assert(2 * TB * (TB / RC) == 256, "one column task per thread");
    const int c = threadIdx.x % (2 * TB), q = threadIdx.x / (2 * TB);
    const bool hi = c >= TB;
    const int gx = kx0 + (hi ? c - TB : c);
    T x[NX];
#pragma unroll
    for (int k = 0; k < NX; ++k) x[k] = tmpS[(2 * RC * q + k) * C::ST + c];
    T lo[RC], hg[RC];
#pragma unroll
    for (int o = 0; o < RC; ++o) {
        T sl = T(0), sh = T(0);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            sl = fma(f[j], x[2 * o + j], sl);
            sh = fma(f[16 + j], x[2 * o + j], sh);
        }
        lo[o] = sl;
        hg[o] = sh;
    }
    if (gx >= hx) return;
    // low-pass destination: LL (compact slot, or its Mallat place at the last level)
    // for a columns, the (low y, high x) detail for d columns
    T* p1 = hi ? cb + hx + gx : (last ? cb + gx : llb + gx);
    const int s1 = (!hi && !last) ? hx : nx;
    T* p2 = cb + (size_t)hy * nx + (hi ? hx : 0) + gx;
    const int gy0 = ky0 + RC * q;
#pragma unroll
    for (int o = 0; o < RC; ++o) {
        if (gy0 + o < hy) {
            __builtin_nontemporal_store(lo[o], p1 + (size_t)(gy0 + o) * s1);
            __builtin_nontemporal_store(hg[o], p2 + (size_t)(gy0 + o) * nx);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_dwt_level(const T* __restrict__ X, const T* __restrict__ llin,
                                                   T* __restrict__ coef, T* __restrict__ llout,
                                                   const T* __restrict__ filt, int L, int nx, int ny, int mx, int my,
                                                   int lev0, int last, int n_db) {
    using C = DwtCfg<T>;
    constexpr int TB = C::TB, VW = Pack16<T>::n;
    constexpr int WMAX = 2 * TB + WV_HALO;            // widest window edge (16 taps)
    constexpr int NG = (WMAX + VW - 1) / VW;          // 16-byte groups per window row
    constexpr int NW = (WMAX * NG + 255) / 256;       // groups per thread
    static_assert(NG * VW <= C::SI, "window rows fit the LDS row");
    __shared__ __align__(16) T inS[WMAX * C::SI];
    __shared__ __align__(16) T tmpS[WMAX * C::ST];
    const int hx = mx >> 1, hy = my >> 1;
    const int ntx = (hx + TB - 1) / TB, nty = (hy + TB - 1) / TB, ntiles = ntx * nty;
    const size_t N = (size_t)nx * ny;
    const int tid = threadIdx.x;
    // work items: (tile, channel) at level 0 (all bases share the window), else (tile, channel, basis)
    const int nitems = ntiles * L * (lev0 ? 1 : n_db);
    T win[NW * VW];
    auto fetch = [&](int item) {
        const int tile = xcd_band(item % ntiles, ntiles), rest = item / ntiles;
        const int l = rest % L, b = rest / L;
        const int ky0 = (tile / ntx) * TB, kx0 = (tile % ntx) * TB;
        const T* src = lev0 ? X + (size_t)l * N : llin + ((size_t)b * L + l) * (size_t)my * mx;
        const int stride = lev0 ? nx : mx;
        const int rows = 2 * TB + 2 * (lev0 ? n_db : b + 1) - 2;   // window rows this item filters
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int e = tid + 256 * k;
            const int r = e / NG, g = e - r * NG;
            if (r < rows) {
                const T* row = src + (size_t)wrap_idx(2 * ky0 + r, my) * stride;
                if (mx >= VW) {
                    // mx and the group start are multiples of VW: a group never straddles the wrap
                    ld16(row + wrap_idx(2 * kx0 + VW * g, mx), win + VW * k);
                } else {
#pragma unroll
                    for (int i = 0; i < VW; ++i) win[VW * k + i] = row[wrap_idx(2 * kx0 + VW * g + i, mx)];
                }
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
        const int rows = 2 * TB + 2 * (lev0 ? n_db : b_first + 1) - 2;
        __syncthreads();   // the previous item is done with inS and tmpS
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int e = tid + 256 * k;
            const int r = e / NG, g = e - r * NG;
            if (r < rows) st16(inS + r * C::SI + VW * g, win + VW * k);
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
// (approximation from the coarser synthesis, or from C at the coarsest level)
// with 16-byte loads, inverts along y then x in LDS, and writes a compact
// approximation for the next finer level.  At level 0 it loops over the bases and
// writes Xout = C0 + sum_b Psi_b C_b once.  Outputs 2p and 2p + 1 of a filter
// pass read the same coefficients (even taps for the first, odd for the second).
// Each thread owns a run of adjacent outputs: it reads the coefficients the run
// needs once into registers and forms every output as a chain of FMAs, so the
// inner loops carry no index arithmetic.
//
// LDS layout: S[sy][r][sx * W + c] holds the W x W window of subband (sy, sx), the
// two x-subbands side by side in one row, so the column pass walks one contiguous
// range of lanes per row; Tm[m][sx * W + c] holds the column-inverted rows, the
// low-x half then the high-x half, read by the row pass with 16-byte reads.
template <typename T> struct IdwtCfg;
// TO output tile edge, P output pairs per column task, Q output pairs per row task,
// row strides SW (S) and ST (Tm), multiples of 16 bytes; NTH threads per work-group
// and WPE, the waves per SIMD the register allocation is held to
template <> struct IdwtCfg<float> { static constexpr int TO = 64, P = 4, Q = 4, SW = 84, ST = 84, NTH = 256, WPE = 3; };
template <> struct IdwtCfg<double> { static constexpr int TO = 32, P = 2, Q = 2, SW = 50, ST = 50, NTH = 256, WPE = 4; };

// Column (y) inverse: task (run, column) forms rows 2p, 2p + 1 for the P values of
// p in the run, in one window column of either x-subband; only the columns the row
// pass reads are formed (window columns 9 - NH .. W - 1 of each half).
template <typename T, int NT>
__device__ __forceinline__ void idwt_y(const T* __restrict__ f, const T* S, T* Tm) {
    using C = IdwtCfg<T>;
    constexpr int TO = C::TO, W = TO / 2 + 8, P = C::P, RUNS = TO / 2 / P, NH = NT / 2;
    constexpr int C0 = 9 - NH, NCOL = W - C0, NA = NH + P - 1;
    for (int t = threadIdx.x; t < RUNS * 2 * NCOL; t += C::NTH) {
        const int run = t / (2 * NCOL), idx = t - run * 2 * NCOL;
        const int cc = idx < NCOL ? C0 + idx : W + C0 + (idx - NCOL);
        const int r0 = P * run + C0;
        T a[NA], d[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            a[k] = S[(r0 + k) * C::SW + cc];
            d[k] = S[(W + r0 + k) * C::SW + cc];
        }
#pragma unroll
        for (int j = 0; j < P; ++j) {
            T xe = T(0), xo = T(0);
#pragma unroll
            for (int i = 0; i < NH; ++i) {
                const int k = j - i + NH - 1;   // window row p + 8 - i
                xe = fma(f[2 * i], a[k], xe);
                xe = fma(f[16 + 2 * i], d[k], xe);
                xo = fma(f[2 * i + 1], a[k], xo);
                xo = fma(f[16 + 2 * i + 1], d[k], xo);
            }
            Tm[(2 * (P * run + j)) * C::ST + cc] = xe;
            Tm[(2 * (P * run + j) + 1) * C::ST + cc] = xo;
        }
    }
}

// Row (x) inverse: task (m, q) forms output columns 2p, 2p + 1 of row m for the Q
// values of p in run q, from window columns Qq .. Qq + Q + 7 of both halves.
template <typename T, int NT>
__device__ __forceinline__ void idwt_x(const T* __restrict__ f, const T* Tm, int t, T* res) {
    using C = IdwtCfg<T>;
    constexpr int TO = C::TO, W = TO / 2 + 8, Q = C::Q, XR = TO / 2 / Q, NH = NT / 2, VW = Pack16<T>::n;
    constexpr int NA = Q + 8;
    static_assert(NA % VW == 0 && W % VW == 0 && Q % VW == 0, "16-byte row reads");
    const int m = t / XR, q = t - (t / XR) * XR;
    const T* row = Tm + m * C::ST + Q * q;
    T a[NA], d[NA];
#pragma unroll
    for (int k = 0; k < NA; k += VW) {
        ld16(row + k, a + k);
        ld16(row + W + k, d + k);
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        T xe = T(0), xo = T(0);
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const int k = j + 8 - i;   // window column p + 8 - i
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
__global__ __launch_bounds__(IdwtCfg<T>::NTH, IdwtCfg<T>::WPE) void k_idwt_level(const T* __restrict__ C, const T* __restrict__ llin,
                                                    T* __restrict__ out, const T* __restrict__ C0,
                                                    const T* __restrict__ filt, int L, int nx, int ny, int mx, int my,
                                                    int coarsest, int final_level, int n_db, int bpw) {
    using Cf = IdwtCfg<T>;
    constexpr int TO = Cf::TO, W = TO / 2 + 8, Q = Cf::Q, XR = TO / 2 / Q, VW = Pack16<T>::n;
    constexpr int G = W / VW;                       // 16-byte groups per subband window row
    constexpr int NG = 4 * W * G;                   // groups of the four windows
    constexpr int NTH = Cf::NTH;
    constexpr int NE = (NG + NTH - 1) / NTH;        // groups per thread
    constexpr int NXT = TO * XR / NTH;              // row-pass tasks per thread
    static_assert(TO * XR % NTH == 0 && 2 * W <= Cf::SW && 2 * W <= Cf::ST, "tiling");
    __shared__ __align__(16) T S[2 * W * Cf::SW];
    __shared__ __align__(16) T Tm[TO * Cf::ST];
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
    // Group e = ((sy W + r) 2 + sx) G + g: VW elements of window row r of subband
    // (sy, sx), columns VW g ..; the same offsets serve every basis, so they are
    // formed once.  A group comes from the coarser approximation (llin) when it is
    // in subband (0, 0) below the coarsest level, else from the coefficient image.
    const bool vec = hx >= VW;   // hx and the group starts are multiples of VW
    int goff[NE], loff[NE];
    unsigned from_ll = 0u;
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        const int e = tid + NTH * i;
        const int rr = e / G, g = e - rr * G;
        const int sx = rr & 1, row = rr >> 1, sy = row / W, r = row - sy * W;
        loff[i] = row * Cf::SW + sx * W + VW * g;
        const int ky = wrap_idx(kylo + r, hy), kx = vec ? wrap_idx(kxlo + VW * g, hx) : 0;
        if (sy == 0 && sx == 0 && !coarsest) {
            from_ll |= 1u << i;
            goff[i] = ky * hx + kx;
        } else {
            goff[i] = (sy * hy + ky) * nx + sx * hx + kx;
        }
    }
    // the window of the next basis is loaded into registers while this one is filtered
    T nxt[NE * VW];
    auto fetch = [&](int b) {
        const T* Cb = C + ((size_t)b * L + l) * N;
        const T* LLb = coarsest ? Cb : llin + ((size_t)b * L + l) * (size_t)hy * hx;
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            if (tid + NTH * i < NG) {
                const T* src = ((from_ll >> i) & 1u) ? LLb : Cb;
                if (vec) {
                    ld16(src + goff[i], nxt + VW * i);
                } else {
                    // coarse levels narrower than one group: element by element
                    const int e = tid + NTH * i, g = e % G;
#pragma unroll
                    for (int k = 0; k < VW; ++k) nxt[VW * i + k] = src[goff[i] + wrap_idx(kxlo + VW * g + k, hx)];
                }
            }
        }
    };
    T acc[NXT * 2 * Q];
#pragma unroll
    for (int k = 0; k < NXT * 2 * Q; ++k) acc[k] = T(0);
    const int b_first = final_level ? 0 : (int)blockIdx.z * bpw;
    const int b_last = final_level ? n_db : min(b_first + bpw, n_db);
    fetch(b_first);
    for (int b = b_first; b < b_last; ++b) {
#pragma unroll
        for (int i = 0; i < NE; ++i)
            if (tid + NTH * i < NG) st16(S + loff[i], nxt + VW * i);
        __syncthreads();
        if (b + 1 < b_last) fetch(b + 1);
        const T* f = filt + b * 32;
        WV_DISPATCH(b, idwt_y, f, S, Tm)
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NXT; ++u) {
            const int t = tid + NTH * u;
            T res[2 * Q];
            WV_DISPATCH(b, idwt_x, f, Tm, t, res)
            if (final_level) {
#pragma unroll
                for (int k = 0; k < 2 * Q; ++k) acc[2 * Q * u + k] += res[k];
            } else {
                const int gy = m0y + t / XR, gx = m0x + 2 * Q * (t % XR);
                T* o = out + ((size_t)b * L + l) * (size_t)my * mx + (size_t)gy * mx + gx;
                if (gy < my) {
                    if (gx + 2 * Q <= mx) {
#pragma unroll
                        for (int k = 0; k < 2 * Q; k += VW) st16(o + k, res + k);
                    } else {
#pragma unroll
                        for (int k = 0; k < 2 * Q; ++k)
                            if (gx + k < mx) o[k] = res[k];
                    }
                }
            }
        }
        __syncthreads();
    }
    if (final_level) {
#pragma unroll
        for (int u = 0; u < NXT; ++u) {
            const int t = tid + NTH * u;
            const int gy = m0y + t / XR, gx = m0x + 2 * Q * (t % XR);
            if (gy >= my) continue;
            const size_t idx = (size_t)l * N + (size_t)gy * nx + gx;
            T* a = acc + 2 * Q * u;
            if (gx + 2 * Q <= mx) {
                if (C0) {
#pragma unroll
                    for (int k = 0; k < 2 * Q; k += VW) {
                        T c0[VW];
                        ld16(C0 + idx + k, c0);
#pragma unroll
                        for (int i = 0; i < VW; ++i) a[k + i] += c0[i];
                    }
                }
#pragma unroll
                for (int k = 0; k < 2 * Q; k += VW) st16(out + idx + k, a + k);
            } else {
#pragma unroll
                for (int k = 0; k < 2 * Q; ++k)
                    if (gx + k < mx) out[idx + k] = (C0 ? C0[idx + k] : T(0)) + a[k];
            }
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
        z[l] = __builtin_nontemporal_load(Ad + o);
        if (HAS_S) z2[l] = __builtin_nontemporal_load(Sd + o);
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
        if (l < L) __builtin_nontemporal_store(z[l] * ft, Ad + (size_t)l * N);
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
        constexpr int TB = DwtCfg<T>::TB;
        const int tiles = ((hy + TB - 1) / TB) * ((hx + TB - 1) / TB);
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
        constexpr int TO = IdwtCfg<T>::TO;
        const int tiles = ((my + TO - 1) / TO) * ((mx + TO - 1) / TO);
        const int fin = (lev == 0) ? 1 : 0;
        T* out = fin ? Xout : ((lev % 2 == 1) ? slotA : slotB);
        // bases per work-group: as many as keep the grid at IDWT_MIN_WG or more, so the
        // next basis's window is fetched while this one is filtered
        int bpw = 1;
        while (!fin && bpw < c->n_db && (int64_t)tiles * L * ((c->n_db + 2 * bpw - 1) / (2 * bpw)) >= IDWT_MIN_WG)
            bpw *= 2;
        const int nz = fin ? 1 : (c->n_db + bpw - 1) / bpw;
        dim3 g(tiles, L, nz);
        k_idwt_level<T><<<g, IdwtCfg<T>::NTH, 0, c->stream>>>(Cdb, llin, out, C0, filt, L, c->nx, c->ny, mx, my,
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
