/*
 * Host sanitizer run of the oracle (test infrastructure): every side kind, the
 * smallest domains, forces and an energy source, a few steps, then moments,
 * diagnostics and a Fourier projection, all of which must be finite.  Built
 * by tests/test_oracle_asan.py with AddressSanitizer and UndefinedBehavior-
 * Sanitizer, which report any access outside an array or undefined operation.
 */
#include "../oracle/oracle13.c"

#include <stdio.h>

static or13_params defaults(void)
{
    or13_params p;
    memset(&p, 0, sizeof p);
    p.Pr = 0.71; p.E0 = -2.0; p.c1 = -3.0; p.k2 = -2.5; p.c_epsE = -2.5;
    p.c_varpi_rho = -6.0; p.c_varpi_E = -0.5;
    p.s_XX = 1.6; p.s_rx = 1.05; p.s_eps = 1.0; p.s_varpi = 1.0; p.s_XXe = 1.5;
    p.rho0 = 1.0; p.collide = 1;
    return p;
}

static int finite_all(const double *a, long n)
{
    for (long i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

int main(void)
{
    static const int sizes[][2] = {{2, 2}, {2, 7}, {7, 2}, {3, 3}, {16, 12}, {33, 20}};
    /* kinds W, E, S, N; tangential speeds; wall temperatures */
    static const int kinds[][4] = {{0, 0, 0, 0}, {2, 2, 0, 0}, {0, 0, 1, 1}, {2, 2, 1, 1}, {0, 0, 2, 2}};
    static const double ut[][4] = {{0, 0, 0, 0}, {0.01, 0, 0, 0}, {0, 0, 0.02, 0}, {0, 0, 0, -0.01}, {0, 0, 0.01, 0}};
    static const double Tw[][4] = {{0, 0, 0, 0}, {-1.99, -2.01, 0, 0}, {0, 0, 0, 0}, {-1.99, -2.01, 0, 0},
                                   {0, 0, -1.99, -2.01}};
    int fails = 0;
    for (unsigned s = 0; s < sizeof sizes / sizeof sizes[0]; ++s) {
        const int nx = sizes[s][0], ny = sizes[s][1];
        const long n = (long)nx * ny;
        double *rho = malloc(sizeof(double) * n), *ux = malloc(sizeof(double) * n);
        double *uy = malloc(sizeof(double) * n), *T = malloc(sizeof(double) * n);
        double *f = malloc(sizeof(double) * Q * n);
        double *m[4] = {malloc(sizeof(double) * n), malloc(sizeof(double) * n), malloc(sizeof(double) * n),
                        malloc(sizeof(double) * n)};
        for (unsigned c = 0; c < sizeof kinds / sizeof kinds[0]; ++c) {
            or13_params p = defaults();
            or13_sides sd;
            for (int w = 0; w < 4; ++w) {
                sd.kind[w] = kinds[c][w];
                sd.u_t[w] = ut[c][w];
                sd.T_w[w] = Tw[c][w];
            }
            if (c == 0) { p.F0x = 1e-5; p.Q_E = 1e-6; }
            if (c == 3) p.gy = -1e-3;
            for (long i = 0; i < n; ++i) {
                const double x = (double)(i % nx), y = (double)(i / nx);
                rho[i] = 1.0 + 1e-3 * sin(0.7 * x + 0.3 * y);
                ux[i] = 0.01 * cos(0.5 * y);
                uy[i] = 0.005 * sin(0.4 * x);
                T[i] = -2.0 + 1e-3 * cos(0.2 * x + 0.9 * y);
            }
            or13_init(nx, ny, rho, ux, uy, T, &p, f);
            if (or13_run(nx, ny, f, &p, &sd, 20) != 0) { printf("run failed %dx%d case %u\n", nx, ny, c); ++fails; continue; }
            or13_moments(nx, ny, f, &p, m[0], m[1], m[2], m[3]);
            double diag[16], four[8];
            or13_diagnostics(nx, ny, f, &p, &sd, diag);
            or13_fourier(nx, ny, f, &p, 1, 1, four);
            int ok = finite_all(f, Q * n) && finite_all(four, 8);
            for (int k = 0; k < 4; ++k) ok = ok && finite_all(m[k], n);
            ok = ok && finite_all(diag, 4);
            if (!ok) { printf("non-finite result %dx%d case %u\n", nx, ny, c); ++fails; }
        }
        free(rho); free(ux); free(uy); free(T); free(f);
        for (int k = 0; k < 4; ++k) free(m[k]);
    }
    printf("oracle sanitizer run: %d failure(s)\n", fails);
    return fails != 0;
}
