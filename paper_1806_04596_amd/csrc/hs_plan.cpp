// Host-side plan: visibility order and bins, work lists, kernel/FFT/wavelet tables.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <numeric>

#include "hs_internal.h"

namespace hs {

// ------------------------------------------------------------------- kernel
// Kaiser-Bessel kernel of width J = 8 on a 2x oversampled grid, shape
// parameter from Beatty et al. (2005): beta = pi sqrt((J/s)^2 (s-1/2)^2 - 0.8).
static long double kb_beta_ld() {
    const long double J = KB_J, s = 2.0L;
    const long double pi = 3.141592653589793238462643383279502884L;
    return pi * std::sqrt((J / s) * (J / s) * (s - 0.5L) * (s - 0.5L) - 0.8L);
}

// Taylor terms of I0(beta sqrt(w)) = sum_k (beta^2 w / 4)^k / (k!)^2.
static void i0_terms(long double beta, std::vector<long double>& t, int n) {
    t.resize(n);
    const long double q = beta * beta / 4.0L;
    t[0] = 1.0L;
    for (int k = 1; k < n; ++k) t[k] = t[k - 1] * q / ((long double)k * (long double)k);
}

static long double i0_of_beta() {
    std::vector<long double> t;
    i0_terms(kb_beta_ld(), t, 200);
    long double s = 0.0L;
    for (int k = 199; k >= 0; --k) s += t[k];
    return s;
}

// Chebyshev interpolant of phi(f + 3 - j) for f in [0, 1] (tap j), converted to
// monomial coefficients in t = f - 1/2 (coefficients below 1 in magnitude, so the
// Horner evaluation is well conditioned).  phi is the entire function
// I0(beta sqrt(w))/I0(beta) of w = 1 - (2d/J)^2, so the interpolant converges
// faster than geometrically.
void kb_taps(int deg, std::vector<double>& coef) {
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double b = kb_beta_ld();
    std::vector<long double> t;
    i0_terms(b, t, 200);
    const long double I0 = i0_of_beta();
    auto phi = [&](long double d) {
        const long double w = 1.0L - (2.0L * d / KB_J) * (2.0L * d / KB_J);
        if (w < 0) return 0.0L;
        long double acc = 0.0L;
        for (int k = 199; k >= 0; --k) acc = acc * w + t[k];
        return acc / I0;
    };
    const int n = deg + 1;
    coef.assign((size_t)4 * n, 0.0);
    for (int j = 0; j < 4; ++j) {
        // Chebyshev coefficients in u = 2t on [-1, 1]
        std::vector<long double> cc(n, 0.0L);
        for (int q = 0; q < n; ++q) {
            long double sum = 0.0L;
            for (int k = 0; k < n; ++k) {
                const long double th = pi * ((long double)k + 0.5L) / (long double)n;
                const long double u = std::cos(th);
                sum += phi(0.5L * (u + 1.0L) + 3.0L - j) * std::cos((long double)q * th);
            }
            cc[q] = sum * 2.0L / (long double)n;
        }
        cc[0] *= 0.5L;
        // Chebyshev -> monomial in u: T_0 = 1, T_1 = u, T_{q+1} = 2 u T_q - T_{q-1}
        std::vector<long double> m(n, 0.0L), T0(n, 0.0L), T1(n, 0.0L);
        T0[0] = 1.0L;
        m[0] += cc[0];
        if (n > 1) {
            T1[1] = 1.0L;
            m[1] += cc[1];
        }
        for (int q = 2; q < n; ++q) {
            std::vector<long double> Tn(n, 0.0L);
            for (int k = 0; k < n; ++k) {
                if (k + 1 < n) Tn[k + 1] += 2.0L * T1[k];
                Tn[k] -= T0[k];
            }
            for (int k = 0; k < n; ++k) m[k] += cc[q] * Tn[k];
            T0 = T1;
            T1 = Tn;
        }
        // u = 2t
        long double p2 = 1.0L;
        for (int k = 0; k < n; ++k, p2 *= 2.0L) coef[(size_t)j * n + k] = (double)(m[k] * p2);
    }
}

// Continuous Fourier transform of the normalised kernel (closed form).
double kb_ft(double xi) {
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double b = kb_beta_ld();
    const long double z = b * b - (pi * KB_J * (long double)xi) * (pi * KB_J * (long double)xi);
    long double v;
    if (z > 0) {
        const long double r = std::sqrt(z);
        v = KB_J * std::sinh(r) / r;
    } else if (z < 0) {
        const long double r = std::sqrt(-z);
        v = KB_J * std::sin(r) / r;
    } else {
        v = KB_J;
    }
    return (double)(v / i0_of_beta());
}

// ----------------------------------------------------------------- Daubechies
// db-K low-pass by spectral factorisation: roots of P_K(y) = sum_{k<K} C(K-1+k,k) y^k
// (Durand-Kerner in long double), z-roots inside the unit circle, then
// sqrt(2) ((1+z^-1)/2)^K prod (1 - r z^-1)/(1 - r).
void daubechies_host(int K, double* h) {
    typedef std::complex<long double> cld;
    std::vector<long double> a(K);  // coefficients, a[k] for y^k
    for (int k = 0; k < K; ++k) {
        long double c = 1.0L;
        for (int i = 1; i <= k; ++i) c = c * (long double)(K - 1 + i) / (long double)i;
        a[k] = c;
    }
    const int deg = K - 1;
    std::vector<cld> roots(deg);
    if (deg > 0) {
        std::vector<cld> m(deg + 1);
        for (int k = 0; k <= deg; ++k) m[k] = a[k] / a[deg];  // monic
        for (int i = 0; i < deg; ++i) roots[i] = std::pow(cld(0.4L, 0.9L), (long double)i);
        auto peval = [&](cld x) {
            cld s = m[deg];
            for (int k = deg - 1; k >= 0; --k) s = s * x + m[k];
            return s;
        };
        for (int it = 0; it < 5000; ++it) {
            long double delta = 0.0L;
            for (int i = 0; i < deg; ++i) {
                cld den = 1.0L;
                for (int j = 0; j < deg; ++j)
                    if (j != i) den *= (roots[i] - roots[j]);
                const cld step = peval(roots[i]) / den;
                roots[i] -= step;
                delta = std::max(delta, std::abs(step));
            }
            if (delta < 1e-30L) break;
        }
    }
    std::vector<cld> poly(1, cld(1.0L, 0.0L));
    auto conv = [&](cld c0, cld c1) {
        std::vector<cld> out(poly.size() + 1, cld(0, 0));
        for (size_t i = 0; i < poly.size(); ++i) {
            out[i] += poly[i] * c0;
            out[i + 1] += poly[i] * c1;
        }
        poly.swap(out);
    };
    for (int k = 0; k < K; ++k) conv(cld(0.5L, 0), cld(0.5L, 0));
    for (int i = 0; i < deg; ++i) {
        const cld y = roots[i];
        const cld b = 1.0L - 2.0L * y;
        const cld s = std::sqrt(b * b - 1.0L);
        cld z = b + s;
        if (std::abs(z) >= 1.0L) z = b - s;
        conv(cld(1.0L, 0) / (1.0L - z), -z / (1.0L - z));
    }
    const long double r2 = std::sqrt(2.0L);
    for (int k = 0; k < 2 * K; ++k) h[k] = (double)(r2 * poly[k].real());
}

// ------------------------------------------------------------------- binning
static inline int region_class(int o, int T) {
    if (o < KB_J / 2 - 1) return 0;
    if (o >= T - KB_J / 2) return 2;
    return 1;
}

struct ChanOrder {
    std::vector<int64_t> perm;        // position -> input index
    std::vector<int64_t> region_ptr;  // [ntiles*9 + 1]
    std::vector<int32_t> bin_local;   // per input index
    std::vector<int32_t> cx, cy;      // per input index (half-plane cell)
    std::vector<int32_t> refl;        // per input index: reflected to -t
    std::vector<double> fx, fy;       // per input index
    std::vector<double> bin_val;      // value of every bin, block by block (ascending within a block)
    std::vector<int64_t> blk_bin_ptr; // [nb + 1]: bins of block b are [ptr[b], ptr[b + 1])
};

// Cell, fraction and reflection of one visibility in the Hermitian half plane:
// t = (u Kx, v Ky) reduced mod K (exact: K is a power of two and u is
// float32-representable); when t_x mod Kx > Kx/2 the visibility is reflected
// to -t (phi is even, so its model value is the conjugate of the value at -t).
// The taps of t are floor(t) - 3 .. floor(t) + 4; their mirror images are the
// taps of cell -floor(t) - 1 = ceil(-t) - 1 with fraction 1 - f in (0, 1], so a
// reflected visibility sees exactly the mirrored cells, also on a grid node.
struct HalfCell {
    int32_t cx, cy, refl;
    double fx, fy;
};
static inline HalfCell half_cell(double u, double v, int Kx, int Ky) {
    const double tX = u * (double)Kx;   // one correctly rounded product, as the definition
    const double tY = v * (double)Ky;
    const double flx = std::floor(tX), fly = std::floor(tY);
    int64_t ix = (int64_t)flx % Kx, iy = (int64_t)fly % Ky;
    if (ix < 0) ix += Kx;
    if (iy < 0) iy += Ky;
    const double fx = tX - flx, fy = tY - fly;
    HalfCell h{(int32_t)ix, (int32_t)iy, 0, fx, fy};
    if (ix > Kx / 2 || (ix == Kx / 2 && fx > 0.0)) {
        h.refl = 1;
        h.cx = (int32_t)(Kx - 1 - ix);
        h.cy = (int32_t)(Ky - 1 - iy);
        h.fx = 1.0 - fx;   // exact: fx is a multiple of ulp(tX)
        h.fy = 1.0 - fy;
    }
    return h;
}

static void order_channel(int64_t M, const double* uv, const double* u, int nb, const int64_t* bp, int nx, int ny,
                          int T, ChanOrder& o) {
    const int Kx = 2 * nx, Ky = 2 * ny;
    const int tx = nx / T + 1, ty = Ky / T;   // visibility tiles over kx in [0, Kx/2 + T)
    const int64_t ntr = (int64_t)tx * ty * 9;
    o.cx.resize(M);
    o.cy.resize(M);
    o.fx.resize(M);
    o.fy.resize(M);
    o.refl.resize(M);
    std::vector<int64_t> key(M);
    std::vector<int32_t> loc(M);   // cell within the tile, raster order
    for (int64_t m = 0; m < M; ++m) {
        const HalfCell h = half_cell(uv[2 * m], uv[2 * m + 1], Kx, Ky);
        o.cx[m] = h.cx;
        o.cy[m] = h.cy;
        o.fx[m] = h.fx;
        o.fy[m] = h.fy;
        o.refl[m] = h.refl;
        const int64_t tile = (h.cy / T) * tx + (h.cx / T);
        const int reg = 3 * region_class(h.cy % T, T) + region_class(h.cx % T, T);
        key[m] = tile * 9 + reg;
        loc[m] = (h.cy % T) * T + (h.cx % T);
    }
    // bins: the (block, preconditioner value) pairs that occur, block by block; a
    // visibility's bin is its block's first bin + the rank of its value among the
    // block's distinct values.  At most M + nb bins, whatever the values.
    o.bin_local.assign(M, 0);
    o.bin_val.clear();
    o.blk_bin_ptr.assign(1, 0);
    for (int b = 0; b < nb; ++b) {
        const int64_t m0 = bp[b], m1 = bp[b + 1];
        std::vector<double> vals;
        if (u) {
            vals.assign(u + m0, u + m1);
            std::sort(vals.begin(), vals.end());
            vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
        } else if (m1 > m0) {
            vals.assign(1, 1.0);
        }
        const int64_t off = o.blk_bin_ptr.back();
        for (int64_t m = m0; m < m1; ++m) {
            const int64_t cls = u ? (int64_t)(std::lower_bound(vals.begin(), vals.end(), u[m]) - vals.begin()) : 0;
            o.bin_local[m] = (int32_t)(off + cls);
        }
        o.bin_val.insert(o.bin_val.end(), vals.begin(), vals.end());
        o.blk_bin_ptr.push_back(off + (int64_t)vals.size());
    }
    // stable counting sorts: by cell within the tile, then by bin, then by (tile,
    // region).  Within a (tile, region, bin) group the visibilities come in raster
    // order of their cells, so neighbouring lanes of the degridding read
    // neighbouring grid cells.
    const int64_t nbins = std::max<int64_t>(o.blk_bin_ptr.back(), 1);
    const int64_t nloc = (int64_t)T * T;
    std::vector<int64_t> cnt(std::max<int64_t>(std::max<int64_t>(nbins, ntr), nloc) + 1, 0);
    std::vector<int64_t> tmp0(M), tmp(M);
    for (int64_t m = 0; m < M; ++m) cnt[loc[m] + 1]++;
    for (int64_t k = 0; k < nloc; ++k) cnt[k + 1] += cnt[k];
    for (int64_t m = 0; m < M; ++m) tmp0[cnt[loc[m]]++] = m;
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int64_t m = 0; m < M; ++m) cnt[o.bin_local[m] + 1]++;
    for (int64_t k = 0; k < nbins; ++k) cnt[k + 1] += cnt[k];
    for (int64_t k = 0; k < M; ++k) {
        const int64_t m = tmp0[k];
        tmp[cnt[o.bin_local[m]]++] = m;
    }
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int64_t m = 0; m < M; ++m) cnt[key[m] + 1]++;
    for (int64_t k = 0; k < ntr; ++k) cnt[k + 1] += cnt[k];
    o.region_ptr.assign(cnt.begin(), cnt.begin() + ntr + 1);
    o.perm.resize(M);
    for (int64_t k = 0; k < M; ++k) {
        const int64_t m = tmp[k];
        o.perm[cnt[key[m]]++] = m;
    }
}

hs_status build_plan(hs_ctx* c) {
    const int L = c->L;
    for (int l = 0; l < L; ++l)
        if (!c->ch[l].set) return fail(c, HS_ERR_INVALID_ARG, "hs_plan: channel " + std::to_string(l) + " not set");
    int T = c->tune_tile ? c->tune_tile : c->desc.tile;
    if (T == 0) {
        T = 32;
        while (T > 8 && (c->Kx / T < 3 || c->Ky / T < 3 || c->Kx % T || c->Ky % T)) T /= 2;
    }
    if (T < 8 || T > 32 || (T & (T - 1)) || c->Kx % T || c->Ky % T || c->Kx / T < 3 || c->Ky / T < 3)
        return fail(c, HS_ERR_SHAPE, "hs_plan: tile must be a power of two in 8..32 with >= 3 tiles per dimension");
    c->T = T;
    c->Kh = c->Kx / 2;
    c->Wh = c->Kh + 1;
    c->Wg = c->Kh + 2 * GR_MARGIN;
    c->Hs = c->Kh + 16;
    c->tiles_x = c->Kh / T + 1;
    c->tiles_y = c->Ky / T;
    c->ntiles = c->tiles_x * c->tiles_y;
    c->gtiles_x = c->Kh / GB + 2;   // blocks cover kx in [-GB, Kx/2 + GB)
    c->ngtiles = c->gtiles_x * (c->Ky / GB);
    // offsets
    c->chan_off.assign(L + 1, 0);
    c->blk_off.assign(L + 1, 0);
    for (int l = 0; l < L; ++l) {
        c->chan_off[l + 1] = c->chan_off[l] + c->ch[l].M;
        c->blk_off[l + 1] = c->blk_off[l] + c->ch[l].nb;
    }
    c->Mtot = c->chan_off[L];
    c->nblk = c->blk_off[L];
    if (c->Mtot >= (int64_t)INT32_MAX) return fail(c, HS_ERR_SHAPE, "hs_plan: more than 2^31-1 visibilities");
    const int64_t M = c->Mtot;
    c->h_cell.assign(M, 0);
    c->h_frac.assign(2 * M, 0.0);
    c->h_y.assign(2 * M, 0.0);
    c->h_theta.assign(M, 0.0);
    c->h_u.assign(M, 0.0);
    c->h_bin.assign(M, 0);
    c->h_perm.assign(M, 0);
    c->h_pos_of.assign(M, 0);
    c->h_bin_u.clear();
    c->h_blk_bin_ptr.assign(1, 0);
    c->h_blk_eps.clear();
    c->dunits.clear();
    c->h_chunk_run.clear();
    c->gunits.clear();
    c->splits.clear();
    c->h_glist.clear();
    std::vector<std::pair<int32_t, int32_t>> run_bin;  // (bin, run)
    int64_t nruns = 0, npartial = 0;
    int64_t bin_base = 0;
    const int unit_max = DEG_THREADS * c->deg_batches;
    c->dunit_off.assign(1, 0);
    c->gunit_off.assign(1, 0);
    c->split_off.assign(1, 0);
    c->bin_off.assign(1, 0);
    for (int l = 0; l < L; ++l) {
        const Channel& ch = c->ch[l];
        ChanOrder o;
        order_channel(ch.M, ch.uv.data(), ch.has_u ? ch.u.data() : nullptr, ch.nb, ch.bp.data(), c->nx, c->ny, T, o);
        const int64_t base = c->chan_off[l];
        for (int64_t k = 0; k < ch.M; ++k) {
            const int64_t m = o.perm[k];
            const int64_t g = base + k;
            c->h_cell[g] = (o.cy[m] << 16) | (o.refl[m] << 15) | o.cx[m];
            c->h_frac[2 * g] = o.fx[m];
            c->h_frac[2 * g + 1] = o.fy[m];
            c->h_theta[g] = ch.theta[m];
            c->h_y[2 * g] = ch.theta[m] * ch.y[2 * m];
            c->h_y[2 * g + 1] = ch.theta[m] * ch.y[2 * m + 1];
            c->h_u[g] = ch.has_u ? ch.u[m] : 1.0;
            c->h_bin[g] = (int32_t)(bin_base + o.bin_local[m]);
            c->h_perm[g] = (int32_t)(base + m);
            c->h_pos_of[base + m] = g;
        }
        // bins and blocks
        c->h_bin_u.insert(c->h_bin_u.end(), o.bin_val.begin(), o.bin_val.end());
        for (int b = 0; b < ch.nb; ++b) {
            c->h_blk_bin_ptr.push_back((int32_t)(bin_base + o.blk_bin_ptr[b + 1]));
            c->h_blk_eps.push_back(ch.eps[b]);
        }
        const int64_t nbins_l = o.blk_bin_ptr.back();
        if (bin_base + nbins_l >= (int64_t)INT32_MAX) return fail(c, HS_ERR_SHAPE, "hs_plan: too many bins");
        // degridding units and their runs
        for (int t = 0; t < c->ntiles; ++t) {
            const int64_t s = o.region_ptr[(int64_t)t * 9], e = o.region_ptr[(int64_t)t * 9 + 9];
            for (int64_t p = s; p < e; p += unit_max) {
                DegridUnit du{};
                du.l = l;
                du.tile = t;
                du.start = (int32_t)(base + p);
                du.count = (int32_t)std::min<int64_t>(unit_max, e - p);
                du.run_base = (int32_t)nruns;
                du.chunk0 = (int32_t)c->h_chunk_run.size();
                for (int64_t b0 = 0; b0 < du.count; b0 += DEG_CHUNK) {
                    const int64_t b1 = std::min<int64_t>(du.count, b0 + DEG_CHUNK);
                    c->h_chunk_run.push_back((int32_t)nruns);
                    int32_t prev = -1;
                    for (int64_t i = b0; i < b1; ++i) {
                        const int32_t bin = c->h_bin[base + p + i];
                        if (i == b0 || bin != prev) {
                            run_bin.push_back({bin, (int32_t)nruns});
                            ++nruns;
                        }
                        prev = bin;
                    }
                }
                c->dunits.push_back(du);
            }
        }
        // gridding units (every block gets at least one: empty blocks write
        // zeros).  Every visibility is listed by each GB x GB block its 8 x 8
        // footprint meets (one to four; periodic in y), in plan order (stable
        // counting sort by block).
        {
            const int nbx = c->gtiles_x, nby = c->Ky / GB, Ky = c->Ky;
            auto blocks_of = [&](int64_t g, int32_t* out) -> int {
                const int32_t cl = c->h_cell[g];
                const int x0 = (cl & 0x7FFF) - 3 + GB;   // first tap, in block units shifted by one block
                int ya = (cl >> 16) - 3;
                if (ya < 0) ya += Ky;
                int yb = ya + 7;
                if (yb >= Ky) yb -= Ky;
                const int bx[2] = {x0 / GB, (x0 + 7) / GB}, by[2] = {ya / GB, yb / GB};
                int n = 0;
                for (int i = 0; i < (by[1] != by[0] ? 2 : 1); ++i)
                    for (int j = 0; j < (bx[1] != bx[0] ? 2 : 1); ++j) out[n++] = by[i] * nbx + bx[j];
                return n;
            };
            std::vector<int64_t> bcnt((size_t)nbx * nby + 1, 0);
            int32_t ids[4];
            for (int64_t k = 0; k < ch.M; ++k) {
                const int n = blocks_of(base + k, ids);
                for (int i = 0; i < n; ++i) {
                    if (ids[i] < 0 || ids[i] >= nbx * nby) return fail(c, HS_ERR_INVALID_ARG, "hs_plan: internal error in gridding blocks");
                    ++bcnt[ids[i] + 1];
                }
            }
            for (int b = 0; b < nbx * nby; ++b) bcnt[b + 1] += bcnt[b];
            const int64_t g0 = (int64_t)c->h_glist.size(), E = bcnt[(size_t)nbx * nby];
            if (g0 + E > INT32_MAX) return fail(c, HS_ERR_SHAPE, "hs_plan: too many gridding entries");
            c->h_glist.resize(g0 + E);
            std::vector<int64_t> fill(bcnt.begin(), bcnt.end() - 1);
            for (int64_t k = 0; k < ch.M; ++k) {
                const int n = blocks_of(base + k, ids);
                for (int i = 0; i < n; ++i) c->h_glist[g0 + fill[ids[i]]++] = (int32_t)(base + k);
            }
            for (int t = 0; t < nbx * nby; ++t) {
                const int64_t s0 = bcnt[t], e0 = bcnt[t + 1], En = e0 - s0;
                const int nsplit = (int)std::max<int64_t>(1, (En + c->grid_split - 1) / c->grid_split);
                for (int sp = 0; sp < nsplit; ++sp) {
                    GridUnit gu{};
                    gu.l = l;
                    gu.tile = t;
                    gu.split = sp;
                    gu.nsplit = nsplit;
                    gu.partial = (int32_t)npartial;
                    const int64_t a = (sp * En) / nsplit, e = ((sp + 1) * En) / nsplit;
                    gu.g0 = (int32_t)(g0 + s0 + a);
                    gu.gn = (int32_t)(e - a);
                    c->gunits.push_back(gu);
                }
                if (nsplit > 1) {
                    c->splits.push_back(SplitTile{l, t, (int32_t)npartial, nsplit});
                    npartial += nsplit;
                }
            }
        }
        bin_base += nbins_l;
        c->dunit_off.push_back((int64_t)c->dunits.size());
        c->gunit_off.push_back((int64_t)c->gunits.size());
        c->split_off.push_back((int64_t)c->splits.size());
        c->bin_off.push_back(bin_base);
    }
    c->nbins = bin_base;
    c->nruns = nruns;
    c->npartial = npartial;
    // Run sums are stored grouped by bin (increasing run index within a bin):
    // run r goes to slot run_slot[r], and bin k owns slots [bin_run_ptr[k], bin_run_ptr[k + 1]).
    c->h_bin_run_ptr.assign(c->nbins + 1, 0);
    for (auto& pr : run_bin) c->h_bin_run_ptr[pr.first + 1]++;
    for (int64_t k = 0; k < c->nbins; ++k) c->h_bin_run_ptr[k + 1] += c->h_bin_run_ptr[k];
    c->h_run_slot.assign(nruns, 0);
    {
        std::vector<int32_t> fillp(c->h_bin_run_ptr.begin(), c->h_bin_run_ptr.end() - 1);
        for (auto& pr : run_bin) c->h_run_slot[pr.second] = fillp[pr.first]++;
    }
    // kernel polynomials per tap (Chebyshev interpolants, rounding-level accurate)
    c->kb_terms = (c->dtype == HS_F64 ? KBDeg<double>::n : KBDeg<float>::n) + 1;
    kb_taps(c->kb_terms - 1, c->kb_c);
    if (c->dtype == HS_F32) kb_taps(KBDeg<double>::n, c->kb_c64);
    return HS_OK;
}

}  // namespace hs

// --------------------------------------------------------- host utilities (C ABI)
extern "C" hs_status hs_density_precond(int64_t M, const double* uv, int32_t nx, int32_t ny, double* out) {
    if (M < 0 || nx <= 0 || ny <= 0 || (M > 0 && (!uv || !out))) return HS_ERR_INVALID_ARG;
    std::vector<int64_t> key(M);
    for (int64_t m = 0; m < M; ++m) {
        if (!std::isfinite(uv[2 * m]) || !std::isfinite(uv[2 * m + 1])) return HS_ERR_NONFINITE;
        int64_t cx = (int64_t)std::floor(uv[2 * m] * (double)nx) % nx;
        int64_t cy = (int64_t)std::floor(uv[2 * m + 1] * (double)ny) % ny;
        if (cx < 0) cx += nx;
        if (cy < 0) cy += ny;
        key[m] = cy * nx + cx;
    }
    std::vector<int64_t> sorted(key);
    std::sort(sorted.begin(), sorted.end());
    for (int64_t m = 0; m < M; ++m) {
        const auto r = std::equal_range(sorted.begin(), sorted.end(), key[m]);
        out[m] = 1.0 / (double)(r.second - r.first);
    }
    return HS_OK;
}

extern "C" hs_status hs_visibility_order(int64_t M, const double* uv, const double* precond, int32_t nblocks,
                                         const int64_t* block_ptr, int32_t nx, int32_t ny, int32_t tile,
                                         int64_t* perm, int64_t* region_ptr) {
    if (M < 0 || nx < 16 || ny < 16 || nblocks < 1 || !block_ptr || !perm || !region_ptr || (M > 0 && !uv))
        return HS_ERR_INVALID_ARG;
    const int Kx = 2 * nx, Ky = 2 * ny;
    if (tile < 8 || tile > 64 || (tile & (tile - 1)) || Kx % tile || Ky % tile || Kx / tile < 3 || Ky / tile < 3)
        return HS_ERR_SHAPE;
    if (block_ptr[0] != 0 || block_ptr[nblocks] != M) return HS_ERR_INVALID_ARG;
    for (int b = 0; b < nblocks; ++b)
        if (block_ptr[b + 1] < block_ptr[b]) return HS_ERR_INVALID_ARG;
    hs::ChanOrder o;
    hs::order_channel(M, uv, precond, nblocks, block_ptr, nx, ny, tile, o);
    std::copy(o.perm.begin(), o.perm.end(), perm);
    std::copy(o.region_ptr.begin(), o.region_ptr.end(), region_ptr);
    return HS_OK;
}

extern "C" hs_status hs_daubechies_filter(int32_t K, double* h) {
    if (K < 1 || K > hs::MAX_DB || !h) return HS_ERR_INVALID_ARG;
    hs::daubechies_host(K, h);
    return HS_OK;
}
