// Standalone use of the C ABI (include/lbm13.h) without PyTorch: a periodic
// shear wave ux = U sin(2 pi y / n) on an n x n FP64 domain, advanced in
// three-step launches, whose amplitude must decay as exp(-nu k^2 t) with the
// shear viscosity nu the library derives from the relaxation rates (sec. 2).
//
// Build (from the repository root, after the library is built):
//   hipcc --offload-arch=gfx950 -Iinclude paper_1401_0188_amd/examples/c_api_example.cpp \
//         -Lpaper_1401_0188_amd -llbm13 -Wl,-rpath,$PWD/paper_1401_0188_amd -o c_api_example
// Exit status 0 when the decay matches within 1 %.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "lbm13.h"

#define CHECK_HIP(x)                                                                   \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));               \
            return 1;                                                                  \
        }                                                                              \
    } while (0)
#define CHECK_LBM(ctx, x)                                                              \
    do {                                                                               \
        int s_ = (x);                                                                  \
        if (s_ != LBM13_OK) {                                                          \
            std::fprintf(stderr, "%s: %d %s\n", #x, s_, ctx ? lbm13_last_error(ctx) : ""); \
            return 1;                                                                  \
        }                                                                              \
    } while (0)

int main() {
    const int n = 256, steps = 3000;
    const double U = 1e-3, pi = 3.14159265358979323846, k = 2 * pi / n;
    const size_t N = (size_t)n * n;

    // host fields: rho = 1, ux = U sin(k y), uy = 0, T = E0
    lbm13_params p = {};
    p.s_XX = 1.6; p.s_rx = 1.05; p.s_eps = 1.0; p.s_varpi = 1.0; p.s_XXe = 1.5;
    p.Pr = 0.71; p.E0 = -2.0; p.c1 = -3.0; p.k2 = -2.5; p.c_epsE = -2.5; p.c_varpi_rho = -6.0; p.c_varpi_E = -0.5;
    p.rho0 = 1.0; p.collide = 1;
    std::vector<double> rho(N, 1.0), ux(N), uy(N, 0.0), T(N, p.E0);
    for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) ux[(size_t)y * n + x] = U * std::sin(k * y);

    // device memory: the workspace and four field buffers, all owned here
    const size_t ws_bytes = lbm13_workspace_bytes(n, n, LBM13_FP64);
    if (ws_bytes == 0) return 1;
    void* ws = nullptr;
    double* d[4] = {nullptr, nullptr, nullptr, nullptr};
    CHECK_HIP(hipMalloc(&ws, ws_bytes));
    for (auto& b : d) CHECK_HIP(hipMalloc(&b, N * sizeof(double)));
    CHECK_HIP(hipMemcpy(d[0], rho.data(), N * sizeof(double), hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d[1], ux.data(), N * sizeof(double), hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d[2], uy.data(), N * sizeof(double), hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d[3], T.data(), N * sizeof(double), hipMemcpyHostToDevice));

    lbm13_ctx* ctx = nullptr;
    CHECK_LBM(ctx, lbm13_create(n, n, LBM13_FP64, ws, ws_bytes, nullptr, &ctx));
    lbm13_side sides[4] = {{LBM13_PERIODIC, 0.0, 0.0}, {LBM13_PERIODIC, 0.0, 0.0},
                           {LBM13_PERIODIC, 0.0, 0.0}, {LBM13_PERIODIC, 0.0, 0.0}};
    lbm13_derived dv;
    CHECK_LBM(ctx, lbm13_set_params(ctx, &p, sides, &dv));
    CHECK_LBM(ctx, lbm13_set_steps_per_launch(ctx, 3));
    CHECK_LBM(ctx, lbm13_init_moments(ctx, d[0], d[1], d[2], d[3]));
    CHECK_LBM(ctx, lbm13_step(ctx, steps));
    CHECK_LBM(ctx, lbm13_moments(ctx, d[0], d[1], d[2], d[3]));
    CHECK_HIP(hipDeviceSynchronize());
    CHECK_HIP(hipMemcpy(ux.data(), d[1], N * sizeof(double), hipMemcpyDeviceToHost));

    // projection of ux on sin(k y), normalised to U at t = 0
    double amp = 0.0;
    for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) amp += ux[(size_t)y * n + x] * std::sin(k * y);
    amp *= 2.0 / (double)N / U;
    const double expect = std::exp(-dv.nu * k * k * steps);
    const double rel = std::fabs(amp / expect - 1.0);
    std::printf("shear amplitude after %d steps: %.8f, exp(-nu k^2 t) = %.8f (nu = %.6f), relative difference %.2e\n",
                steps, amp, expect, dv.nu, rel);

    CHECK_LBM(ctx, lbm13_destroy(ctx));
    for (auto& b : d) CHECK_HIP(hipFree(b));
    CHECK_HIP(hipFree(ws));
    return rel <= 0.01 ? 0 : 2;
}
