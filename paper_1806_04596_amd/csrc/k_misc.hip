// Primal update (Algorithm 2), FP64 reductions, power-iteration
// helpers (Sec. 3.4 step sizes) and the reweighting of Algorithm 1
// (eq:weights-l21).
#include "hs_internal.h"

namespace hs {

static inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename S, typename D>
__global__ void k_convert(D* __restrict__ dst, const S* __restrict__ src, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (D)src[i];
}

template <typename S, typename D>
void launch_convert(hipStream_t s, D* dst, const S* src, int64_t n) {
    if (n > 0) k_convert<S, D><<<nb(n, 256), 256, 0, s>>>(dst, src, n);
}
template void launch_convert<float, double>(hipStream_t, double*, const float*, int64_t);

template <typename T>
__global__ void k_axpby(T* y, const T* x, T a, T b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i] + b * y[i];
}

__device__ __forceinline__ double block_sum_256(double v, double* sh) {
    const int tid = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0) s = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return s;
}

// Primal update: G = k1 P + k2 At + k3 D (P or At null: that prior is off);
// X <- max(X - tau G, 0); Xt <- 2X_new - X_old;
// FP64 partial sums of ||X_new - X_old||^2 and ||X_new||^2 per block (fixed grid).
// 16 bytes of T.
template <typename T>
struct Vec16 {
    T v[16 / sizeof(T)];
};

template <typename T, bool HAS_P, bool HAS_AT>
__global__ __launch_bounds__(256) void k_primal(T* __restrict__ X, T* __restrict__ Xt, const T* __restrict__ P,
                                                const T* __restrict__ At, const T* __restrict__ D, T k1, T k2, T k3,
                                                T tau, int64_t n, double* __restrict__ part) {
    // n is a multiple of 16 / sizeof(T): every operand is read and written in
    // 16-byte vectors, two per array in flight per thread and step
    constexpr int V = 16 / sizeof(T), U = 2;
    __shared__ double sh[4];
    double dd = 0.0, xx = 0.0;
    const int64_t nv = n / V;
    const Vec16<T>* Dv = reinterpret_cast<const Vec16<T>*>(D);
    const Vec16<T>* Pv = reinterpret_cast<const Vec16<T>*>(P);
    const Vec16<T>* Av = reinterpret_cast<const Vec16<T>*>(At);
    Vec16<T>* Xv = reinterpret_cast<Vec16<T>*>(X);
    Vec16<T>* Xtv = reinterpret_cast<Vec16<T>*>(Xt);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < nv; i0 += U * stride) {
        Vec16<T> d[U], pp[U], aa[U], xo[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * stride < nv ? i0 + u * stride : i0;
            d[u] = Dv[i];
            if (HAS_P) pp[u] = Pv[i];
            if (HAS_AT) aa[u] = Av[i];
            xo[u] = Xv[i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (i0 + u * stride >= nv) break;
            Vec16<T> xn, xt;
#pragma unroll
            for (int k = 0; k < V; ++k) {
                T g = k3 * d[u].v[k];
                if (HAS_P) g += k1 * pp[u].v[k];
                if (HAS_AT) g += k2 * aa[u].v[k];
                const T x0 = xo[u].v[k];
                T x1 = x0 - tau * g;
                x1 = x1 > T(0) ? x1 : T(0);
                xn.v[k] = x1;
                xt.v[k] = T(2) * x1 - x0;
                const double df = (double)x1 - (double)x0;
                dd += df * df;
                xx += (double)x1 * (double)x1;
            }
            Xv[i0 + u * stride] = xn;
            Xtv[i0 + u * stride] = xt;
        }
    }
    dd = block_sum_256(dd, sh);
    xx = block_sum_256(xx, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = dd;
        part[2 * blockIdx.x + 1] = xx;
    }
}

// beta (the relative variation of Algorithm 2) into scal[0]; iteration counter scal[1] += 1.  One wave:
// lane-strided partial sums, then a fixed butterfly (deterministic).
__global__ void k_finish_beta(const double* __restrict__ part, double* __restrict__ scal, int nparts) {
    const int lane = threadIdx.x;
    double dd = 0.0, xx = 0.0;
    for (int k = lane; k < nparts; k += 64) {
        dd += part[2 * k];
        xx += part[2 * k + 1];
    }
    for (int off = 32; off > 0; off >>= 1) {
        dd += __shfl_xor(dd, off);
        xx += __shfl_xor(xx, off);
    }
    if (lane == 0) {
        scal[0] = (xx > 0.0) ? sqrt(dd / xx) : 0.0;
        scal[1] += 1.0;
        scal[2] = dd;
        scal[3] = xx;
    }
}

// Per-channel sums of squares: part[l][chunk].
template <typename T>
__global__ __launch_bounds__(256) void k_chan_sumsq(const T* __restrict__ X, int64_t N, double* __restrict__ part) {
    __shared__ double sh[4];
    const int l = blockIdx.y;
    const T* x = X + (size_t)l * N;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = (double)x[i];
        s += v * v;
    }
    s = block_sum_256(s, sh);
    if (threadIdx.x == 0) part[(size_t)l * gridDim.x + blockIdx.x] = s;
}

__global__ void k_chan_finish(const double* __restrict__ part, double* __restrict__ out, int L, int nch) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= L) return;
    double s = 0.0;
    for (int k = 0; k < nch; ++k) s += part[(size_t)l * nch + k];
    out[l] = sqrt(s);
}

// x[l] *= 1/norm[l] (zero norms leave the channel unchanged)
template <typename T>
__global__ void k_chan_scale(T* __restrict__ X, const double* __restrict__ nrm, int64_t N) {
    const int l = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double s = nrm[l];
    if (s > 0.0) X[(size_t)l * N + i] = (T)((double)X[(size_t)l * N + i] / s);
}

// Per-channel maximum of X: block partials, then out[l] = max over the partials.
template <typename T>
__global__ __launch_bounds__(256) void k_chan_max(const T* __restrict__ X, int64_t N, double* __restrict__ part) {
    __shared__ double sh[4];
    const int l = blockIdx.y;
    const T* x = X + (size_t)l * N;
    double m = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, (double)x[i]);
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[(size_t)l * gridDim.x + blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

__global__ void k_chan_max_finish(const double* __restrict__ part, double* __restrict__ out, int L, int nch) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= L) return;
    double m = -INFINITY;
    for (int k = 0; k < nch; ++k) m = fmax(m, part[(size_t)l * nch + k]);
    out[l] = m;
}

// X[l][center] = 1 for every channel (a unit source at the phase centre; X zeroed before).
template <typename T>
__global__ void k_set_center(T* __restrict__ X, int L, int64_t N, int64_t center) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < L) X[(size_t)l * N + center] = T(1);
}

// ||Psi^dag X||_{2,1} partials: basis d = blockIdx.y (0: Dirac = X itself, else coef[d-1]);
// sum over pixels of the l2 norm over the L channels, FP64, fixed reduction order.
template <typename T>
__global__ __launch_bounds__(256) void k_l21_norm(const T* __restrict__ X, const T* __restrict__ coef, int L,
                                                  int64_t N, double* __restrict__ part) {
    __shared__ double sh[4];
    const int d = blockIdx.y;
    const T* S = (d == 0) ? X : coef + (size_t)(d - 1) * L * N;
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        double n2 = 0.0;
        for (int l = 0; l < L; ++l) {
            const double v = (double)S[(size_t)l * N + p];
            n2 += v * v;
        }
        acc += sqrt(n2);
    }
    acc = block_sum_256(acc, sh);
    if (threadIdx.x == 0) part[(size_t)d * gridDim.x + blockIdx.x] = acc;
}

// Squared l2 norms of the rows of Psi^dag X (Sec. 2.3: a row is one coefficient of one
// basis across the channels) over a chunk of nl channels, in FP64: X is the chunk's Dirac
// basis [nl][N], coef its n_db wavelet bases [n_db][nl][N].  S[d][p] receives the sum
// (acc = 0) or adds it (acc = 1); the channels are summed in order.
template <typename T>
__global__ void k_l21_rowsq(const T* __restrict__ X, const T* __restrict__ coef, int nl, int64_t N,
                            double* __restrict__ S, int acc) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int d = blockIdx.y;
    const T* src = (d == 0) ? X + p : coef + (size_t)(d - 1) * nl * N + p;
    double n2 = 0.0;
    for (int l = 0; l < nl; ++l) {
        const double v = (double)src[(size_t)l * N];
        n2 += v * v;
    }
    double* out = S + (size_t)d * N + p;
    *out = acc ? *out + n2 : n2;
}

// Gradient of sum_r wbar_r ||c_r|| with respect to the coefficients of a chunk of nl
// channels: c <- scale * wbar_r * c / ||c_r|| with ||c_r||^2 = S[d][p] from k_l21_rowsq
// over all channels (0 on a zero row, the subgradient of least norm).  wbar may be null.
template <typename T>
__global__ void k_l21_rowscale(T* __restrict__ X, T* __restrict__ coef, int nl, int64_t N,
                               const double* __restrict__ S, const T* __restrict__ wbar, double scale) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int d = blockIdx.y;
    const double n2 = S[(size_t)d * N + p];
    double f = n2 > 0.0 ? scale / sqrt(n2) : 0.0;
    if (wbar) f *= (double)wbar[(size_t)d * N + p];
    T* dst = (d == 0) ? X + p : coef + (size_t)(d - 1) * nl * N + p;
    for (int l = 0; l < nl; ++l) dst[(size_t)l * N] = (T)(f * (double)dst[(size_t)l * N]);
}

// Partials of sum_{d,p} wbar[d][p] sqrt(S[d][p]) (the weighted l2,1 norm from the row
// sums of squares), FP64, fixed reduction order; wbar may be null.
template <typename T>
__global__ __launch_bounds__(256) void k_l21_from_rowsq(const double* __restrict__ S, const T* __restrict__ wbar,
                                                        int64_t N, double* __restrict__ part) {
    __shared__ double sh[4];
    const int d = blockIdx.y;
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        const double r = sqrt(S[(size_t)d * N + p]);
        acc += wbar ? (double)wbar[(size_t)d * N + p] * r : r;
    }
    acc = block_sum_256(acc, sh);
    if (threadIdx.x == 0) part[(size_t)d * gridDim.x + blockIdx.x] = acc;
}

// eq:weights-l21: wbar[d][p] = gb / (gb + ||(Psi^dag X)_{d,p}||) over the L channels.
template <typename T>
__global__ void k_reweight_l21(const T* __restrict__ X, const T* __restrict__ coef, T* __restrict__ wbar, double gb,
                               int L, int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int d = blockIdx.y;
    const T* S = (d == 0) ? X + p : coef + (size_t)(d - 1) * L * N + p;
    double n2 = 0.0;
    for (int l = 0; l < L; ++l) {
        const double v = (double)S[(size_t)l * N];
        n2 += v * v;
    }
    wbar[(size_t)d * N + p] = (T)(gb / (gb + sqrt(n2)));
}

// SARA's reweighted l1 (Sec. 2.3): wbar[d][l][p] = gb / (gb + |(Psi_d^dag x_l)_p|), per channel.
template <typename T>
__global__ void k_reweight_l1(const T* __restrict__ X, const T* __restrict__ coef, T* __restrict__ wbar, double gb,
                              int L, int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int d = blockIdx.y, l = blockIdx.z;
    const T v = (d == 0) ? X[(size_t)l * N + p] : coef[((size_t)(d - 1) * L + l) * N + p];
    wbar[((size_t)d * L + l) * N + p] = (T)(gb / (gb + fabs((double)v)));
}

template <typename T>
void launch_fill(hipStream_t s, T* p, T v, int64_t n) {
    if (n > 0) k_fill<T><<<nb(n, 256), 256, 0, s>>>(p, v, n);
}
template <typename T>
void launch_axpby(hipStream_t s, T* y, const T* x, T a, T b, int64_t n) {
    if (n > 0) k_axpby<T><<<nb(n, 256), 256, 0, s>>>(y, x, a, b, n);
}

template <typename T>
void launch_primal(hs_ctx* c, const T* Atsum, const T* Dimg, bool use_p) {
    const int64_t n = (int64_t)c->L * c->N;
    int grid = (int)std::min<int64_t>(NRED, (n + 255) / 256);
    if (grid < 1) grid = 1;
    const T* P = use_p ? (const T*)c->d.P : nullptr;
#define HS_PRIMAL(HP, HA)                                                                                         \
    k_primal<T, HP, HA><<<grid, 256, 0, c->stream>>>((T*)c->d.X, (T*)c->d.Xt, P, Atsum, Dimg, (T)c->k1, (T)c->k2, \
                                                     (T)c->k3, (T)c->tau, n, c->d.red_part)
    if (P && Atsum) HS_PRIMAL(true, true);
    else if (P) HS_PRIMAL(true, false);
    else if (Atsum) HS_PRIMAL(false, true);
    else HS_PRIMAL(false, false);
#undef HS_PRIMAL
    k_finish_beta<<<1, 64, 0, c->stream>>>(c->d.red_part, c->d.scal, grid);
}

// Per-channel l2 norms of X into out[L] (device doubles).
template <typename T>
void launch_chan_norms(hs_ctx* c, const T* X, double* out) {
    const int nch = 64;
    dim3 g(nch, c->L);
    k_chan_sumsq<T><<<g, 256, 0, c->stream>>>(X, c->N, c->d.red_part);
    k_chan_finish<<<1, 64, 0, c->stream>>>(c->d.red_part, out, c->L, nch);
}

template <typename T>
void launch_chan_scale(hs_ctx* c, T* X, const double* nrm) {
    dim3 g(nb(c->N, 256), c->L);
    k_chan_scale<T><<<g, 256, 0, c->stream>>>(X, nrm, c->N);
}

template <typename T>
void launch_chan_max(hs_ctx* c, const T* X, double* out) {
    const int nch = 64;
    dim3 g(nch, c->L);
    k_chan_max<T><<<g, 256, 0, c->stream>>>(X, c->N, c->d.red_part);
    k_chan_max_finish<<<1, 64, 0, c->stream>>>(c->d.red_part, out, c->L, nch);
}

template <typename T>
void launch_set_center(hs_ctx* c, T* X) {
    k_set_center<T><<<1, 64, 0, c->stream>>>(X, c->L, c->N, (int64_t)(c->ny / 2) * c->nx + c->nx / 2);
}

// Partials of ||Psi^dag X||_{2,1} (X: Dirac basis, coef: the n_db wavelet bases) into
// red_part[0 .. D * 64); returns the number of partials.
template <typename T>
int launch_l21_norm(hs_ctx* c, const T* X, const T* coef) {
    const int nch = 64;
    dim3 g(nch, c->D);
    k_l21_norm<T><<<g, 256, 0, c->stream>>>(X, coef, c->L, c->N, c->d.red_part);
    return nch * c->D;
}

template <typename T>
void launch_l21_rowsq(hs_ctx* c, const T* X, const T* coef, int nl, double* S, bool acc) {
    dim3 g(nb(c->N, 256), c->D);
    k_l21_rowsq<T><<<g, 256, 0, c->stream>>>(X, coef, nl, c->N, S, acc ? 1 : 0);
}

template <typename T>
void launch_l21_rowscale(hs_ctx* c, T* X, T* coef, int nl, const double* S, const T* wbar, double scale) {
    dim3 g(nb(c->N, 256), c->D);
    k_l21_rowscale<T><<<g, 256, 0, c->stream>>>(X, coef, nl, c->N, S, wbar, scale);
}

// Partials of sum wbar sqrt(S) into red_part[0 .. D * 64); returns their number.
template <typename T>
int launch_l21_from_rowsq(hs_ctx* c, const double* S, const T* wbar) {
    const int nch = 64;
    dim3 g(nch, c->D);
    k_l21_from_rowsq<T><<<g, 256, 0, c->stream>>>(S, wbar, c->N, c->d.red_part);
    return nch * c->D;
}

template <typename T>
void launch_reweight_l21(hs_ctx* c, const T* X, const T* coef, T* wbar, double gb) {
    dim3 g(nb(c->N, 256), c->D);
    k_reweight_l21<T><<<g, 256, 0, c->stream>>>(X, coef, wbar, gb, c->L, c->N);
}

template <typename T>
void launch_reweight_l1(hs_ctx* c, const T* X, const T* coef, T* wbar, double gb) {
    dim3 g(nb(c->N, 256), c->D, c->L);
    k_reweight_l1<T><<<g, 256, 0, c->stream>>>(X, coef, wbar, gb, c->L, c->N);
}

#define HS_INST(T)                                                                 \
    template void launch_l21_rowsq<T>(hs_ctx*, const T*, const T*, int, double*, bool);                 \
    template void launch_l21_rowscale<T>(hs_ctx*, T*, T*, int, const double*, const T*, double);        \
    template int launch_l21_from_rowsq<T>(hs_ctx*, const double*, const T*);                           \
    template void launch_reweight_l1<T>(hs_ctx*, const T*, const T*, T*, double);  \
    template void launch_fill<T>(hipStream_t, T*, T, int64_t);                     \
    template void launch_axpby<T>(hipStream_t, T*, const T*, T, T, int64_t);       \
    template void launch_primal<T>(hs_ctx*, const T*, const T*, bool);             \
    template void launch_chan_norms<T>(hs_ctx*, const T*, double*);                \
    template void launch_chan_scale<T>(hs_ctx*, T*, const double*);                \
    template void launch_chan_max<T>(hs_ctx*, const T*, double*);                  \
    template void launch_set_center<T>(hs_ctx*, T*);                               \
    template int launch_l21_norm<T>(hs_ctx*, const T*, const T*);                  \
    template void launch_reweight_l21<T>(hs_ctx*, const T*, const T*, T*, double);
HS_INST(float)
HS_INST(double)
template void launch_fill<int32_t>(hipStream_t, int32_t*, int32_t, int64_t);
#undef HS_INST

}  // namespace hs
