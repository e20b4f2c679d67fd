// Host sanitizer run of the C ABI's host code (test infrastructure): parameter
// derivation, workspace layout, argument checks of create and of the
// allocation-free entry point, last-error messages, and the autotune cache
// file (keys, round trip, damaged files).  Nothing here touches a GPU: every
// call either needs no device or fails its host checks first.  Built by
// tests/test_capi_host_sanitizers.py with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <string>

#include "../include/lbm13.h"
#include "../paper_1401_0188_amd/csrc/lbm13_tune_cache.h"

static int failures = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            std::printf("FAIL line %d: %s\n", __LINE__, #c);               \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static lbm13_params defaults() {
    lbm13_params p;
    std::memset(&p, 0, sizeof p);
    p.s_XX = 1.6; p.s_rx = 1.05; p.s_eps = 1.0; p.s_varpi = 1.0; p.s_XXe = 1.5;
    p.Pr = 0.71; p.E0 = -2.0; p.c1 = -3.0; p.k2 = -2.5; p.c_epsE = -2.5;
    p.c_varpi_rho = -6.0; p.c_varpi_E = -0.5; p.rho0 = 1.0; p.collide = 1;
    return p;
}

int main() {
    lbm13_derived d;
    lbm13_params p = defaults();
    CHECK(lbm13_derive(&p, &d) == LBM13_OK && std::fabs(d.cs2 - 1.0) < 1e-15);
    p.c1 = -8.0; p.E0 = 0.0; p.c_epsE = -30.0;  // A = -9
    CHECK(lbm13_derive(&p, &d) == LBM13_EUNSTABLE_PARAMS);
    p = defaults(); p.s_XX = NAN;
    CHECK(lbm13_derive(&p, &d) == LBM13_EUNSTABLE_PARAMS);
    p = defaults(); p.Pr = 0.0;
    CHECK(lbm13_derive(&p, &d) == LBM13_EUNSTABLE_PARAMS);
    p = defaults(); p.c1 = -114404.0 / 51051.0 + 11492.0 * p.c_epsE / 51051.0 - 7854.0 * p.E0 / 51051.0;  // Y ~ 0
    (void)lbm13_derive(&p, &d);  // any status, no undefined behaviour
    CHECK(lbm13_derive(nullptr, &d) != LBM13_OK || true);

    // workspace layout at the edges of the supported sizes
    CHECK(lbm13_workspace_bytes(2, 2, LBM13_FP64) > 0);
    CHECK(lbm13_workspace_bytes(65536, 64, LBM13_FP32_DEV) > 0);
    CHECK(lbm13_workspace_bytes(1, 5, LBM13_FP64) == 0);
    CHECK(lbm13_workspace_bytes(65537, 8, LBM13_FP64) == 0);
    CHECK(lbm13_workspace_bytes(8, 8, 7) == 0);
    int nx[3] = {64, 2, 513}, ny[3] = {64, 7, 3};
    CHECK(lbm13_batch_workspace_bytes(3, nx, ny, LBM13_FP32_DEV) > 0);
    CHECK(lbm13_batch_workspace_bytes(0, nx, ny, LBM13_FP32_DEV) == 0);
    CHECK(lbm13_batch_workspace_bytes(3, nullptr, ny, LBM13_FP32_DEV) == 0);

    // create: argument checks that fail before any device work
    lbm13_ctx* c = nullptr;
    CHECK(lbm13_create(64, 64, LBM13_FP64, nullptr, 1 << 30, nullptr, &c) == LBM13_EINVAL && !c);
    CHECK(lbm13_create(64, 64, LBM13_FP64, reinterpret_cast<void*>(256), 16, nullptr, &c) == LBM13_ENOMEM);
    CHECK(lbm13_create(64, 64, LBM13_FP64, reinterpret_cast<void*>(257), 1 << 30, nullptr, &c) == LBM13_EINVAL);
    CHECK(lbm13_create(64, 64, LBM13_FP64, reinterpret_cast<void*>(256), 1 << 30, nullptr, nullptr) == LBM13_EINVAL);
    CHECK(std::strlen(lbm13_last_error(nullptr)) > 0);
    CHECK(lbm13_step(nullptr, 1) == LBM13_EINVAL && lbm13_destroy(nullptr) == LBM13_EINVAL);

    // allocation-free entry point: rejections on the host
    p = defaults();
    lbm13_side sides[4] = {};
    void* dummy = reinterpret_cast<void*>(256);
    const double* in = static_cast<const double*>(dummy);
    double* out = static_cast<double*>(dummy);
    CHECK(lbm13_advance_noalloc(4096, 4096, LBM13_FP32_DEV, &p, sides, in, out, 3, nullptr) == LBM13_EINVAL);
    CHECK(std::strstr(lbm13_last_error(nullptr), "static scratch") != nullptr);
    CHECK(lbm13_advance_noalloc(64, 64, LBM13_FP64, &p, sides, in, out, -1, nullptr) == LBM13_EINVAL);
    CHECK(lbm13_advance_noalloc(64, 64, LBM13_FP64, nullptr, sides, in, out, 3, nullptr) == LBM13_EINVAL);
    sides[0].kind = LBM13_WALL_ADIABATIC;  // West a wall, East periodic
    CHECK(lbm13_advance_noalloc(64, 64, LBM13_FP64, &p, sides, in, out, 3, nullptr) == LBM13_EINVAL);
    sides[0].kind = 9;
    CHECK(lbm13_advance_noalloc(64, 64, LBM13_FP64, &p, sides, in, out, 3, nullptr) == LBM13_EINVAL);
    sides[0].kind = LBM13_PERIODIC;
    p.s_rx = 2.0;
    CHECK(lbm13_advance_noalloc(64, 64, LBM13_FP64, &p, sides, in, out, 3, nullptr) == LBM13_EUNSTABLE_PARAMS);

    // autotune cache file
    const char* path = "capi_host_tune_cache.json";
    std::remove(path);
    int cfg[6] = {0, 0, 0, 0, 0, 0};
    const std::string k1 = lbm13::tune_key("gfx950:sramecc+:xnack-", 1, 16777216, 1, false);
    const std::string k2 = lbm13::tune_key("gfx950", 0, 7197838, 64, true);
    CHECK(k1 == "gfx950:fp32:n24:d0:periodic");
    CHECK(k2 == "gfx950:fp64:n22:d6:walls");
    CHECK(!lbm13::tune_cache_lookup(path, k1, cfg));
    const int a[6] = {3, 64, 8, 64, 16, 1}, b[6] = {2, 32, 16, 32, 16, 0};
    CHECK(lbm13::tune_cache_store(path, k1, a));
    CHECK(lbm13::tune_cache_store(path, k2, b));
    CHECK(lbm13::tune_cache_lookup(path, k1, cfg) && std::memcmp(cfg, a, sizeof a) == 0);
    CHECK(lbm13::tune_cache_lookup(path, k2, cfg) && std::memcmp(cfg, b, sizeof b) == 0);
    CHECK(lbm13::tune_cache_store(path, k1, b));  // replaces, keeps the other entry
    CHECK(lbm13::tune_cache_lookup(path, k1, cfg) && std::memcmp(cfg, b, sizeof b) == 0);
    CHECK(lbm13::tune_cache_lookup(path, k2, cfg));
    const char* damaged[] = {"", "{", "{\"entries\": {\"x\": [1, 2", "{\"entries\": {\"x\": [1, 2, 3, 4, 5, 6, 7]}}",
                             "{\"entries\": {\"x\": [1, a, 3, 4, 5, 6]}}", "\"entries\"\"entries\": ]]]",
                             "{\"entries\": {\"x\": [99999999999, 1, 1, 1, 1, 1]}}"};
    for (const char* text : damaged) {
        { std::ofstream f(path, std::ios::trunc); f << text; }
        CHECK(!lbm13::tune_cache_lookup(path, "x", cfg));
        CHECK(lbm13::tune_cache_store(path, "x", a));  // rewritten whole
        CHECK(lbm13::tune_cache_lookup(path, "x", cfg) && std::memcmp(cfg, a, sizeof a) == 0);
    }
    std::remove(path);
    CHECK(!lbm13::tune_cache_store("/nonexistent-dir/x/cache.json", k1, a));

    std::printf("%d failure(s)\n", failures);
    return failures ? 1 : 0;
}
