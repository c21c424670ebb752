// Host-side driver of the C-ABI for an AddressSanitizer build of the library (host
// code instrumented, device code unchanged).  It exercises every entry point that
// runs without a GPU: the host utilities on ragged, empty and edge-case inputs, the
// argument checks of hs_create, and the status strings.  Exit status 0 when every
// call returned what it should; the sanitizer aborts on any invalid host access.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "hypersara.h"

static int fails = 0;
#define EXPECT(cond)                                                   \
    do {                                                               \
        if (!(cond)) {                                                 \
            std::printf("FAILED: %s (line %d)\n", #cond, __LINE__);    \
            ++fails;                                                   \
        }                                                              \
    } while (0)

static void order_case(std::mt19937_64& rng, int64_t M, int nx, int ny, int tile, int nblocks, int precond) {
    std::uniform_real_distribution<double> U(-0.75, 0.75);
    std::vector<double> uv(2 * (size_t)M + 1), pre((size_t)M + 1);
    for (int64_t m = 0; m < 2 * M; ++m) uv[m] = U(rng);
    if (M > 0) {
        uv[0] = 0.0;
        uv[1] = -0.5;   // on a grid node and on the fold
    }
    std::vector<int64_t> bp(nblocks + 1);
    for (int b = 0; b <= nblocks; ++b) bp[b] = (b * M) / nblocks;
    const int64_t nreg = (int64_t)(nx / tile + 1) * (2 * ny / tile) * 9 + 1;
    std::vector<int64_t> perm((size_t)M + 1), rp(nreg);
    const double* pp = nullptr;
    if (precond == 1) {
        EXPECT(hs_density_precond(M, uv.data(), nx, ny, pre.data()) == HS_OK);
        pp = pre.data();
    } else if (precond == 2) {
        std::uniform_real_distribution<double> P(0.1, 1.0);
        for (int64_t m = 0; m < M; ++m) pre[m] = P(rng);
        pp = pre.data();
    }
    EXPECT(hs_visibility_order(M, uv.data(), pp, nblocks, bp.data(), nx, ny, tile, perm.data(), rp.data()) == HS_OK);
    // a permutation, and the region pointers span it
    std::vector<char> seen((size_t)M + 1, 0);
    for (int64_t k = 0; k < M; ++k) {
        EXPECT(perm[k] >= 0 && perm[k] < M);
        if (perm[k] >= 0 && perm[k] < M) seen[perm[k]]++;
    }
    for (int64_t m = 0; m < M; ++m) EXPECT(seen[m] == 1);
    EXPECT(rp[0] == 0 && rp[nreg - 1] == M);
}

int main() {
    std::mt19937_64 rng(7);
    const int shapes[][3] = {{16, 16, 8}, {64, 64, 16}, {128, 64, 8}, {64, 128, 32}, {32, 32, 8}};
    for (const auto& sh : shapes)
        for (int pre = 0; pre < 3; ++pre)
            for (int64_t M : {0, 1, 7, 1000, 4097}) order_case(rng, M, sh[0], sh[1], sh[2], M > 0 ? 3 : 1, pre);
    // Daubechies filters: unit norm, and the status of out-of-range orders
    for (int K = 1; K <= 8; ++K) {
        std::vector<double> h(2 * K);
        EXPECT(hs_daubechies_filter(K, h.data()) == HS_OK);
        double n2 = 0.0;
        for (double x : h) n2 += x * x;
        EXPECT(std::fabs(n2 - 1.0) < 1e-12);
    }
    EXPECT(hs_daubechies_filter(0, nullptr) != HS_OK);
    // argument checks of hs_create (before any device is touched)
    hs_ctx* ctx = nullptr;
    hs_problem_desc d{};
    d.nx = 30; d.ny = 32; d.L = 2; d.oversamp = 2; d.J = 8; d.levels = 4; d.n_db = 8; d.dtype = HS_F32;
    EXPECT(hs_create(&d, &ctx) == HS_ERR_SHAPE && ctx == nullptr);
    d.nx = 32; d.dtype = 7;
    EXPECT(hs_create(&d, &ctx) == HS_ERR_DTYPE);
    d.dtype = HS_F64; d.gram_mode = 9;
    EXPECT(hs_create(&d, &ctx) != HS_OK);
    EXPECT(hs_create(nullptr, &ctx) == HS_ERR_INVALID_ARG);
    EXPECT(hs_last_error(nullptr) != nullptr);
    for (int s = 0; s >= -9; --s) EXPECT(hs_status_string(s) != nullptr);
    EXPECT(hs_visibility_order(-1, nullptr, nullptr, 0, nullptr, 16, 16, 8, nullptr, nullptr) != HS_OK);
    std::printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}
