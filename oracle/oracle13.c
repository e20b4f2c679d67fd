/*
 * oracle13.c -- plain FP64 CPU oracle of the single-distribution D2Q13
 * "energy-conserving" lattice Boltzmann time step of Lallemand & Dubois,
 * "Comparison of Simulations of Convective Flows" (Commun. Comput. Phys. 2015).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the HIP library is
 * checked against; it is never part of the product path.  It shares no code,
 * header, table or constant with the library: everything below is written
 * from the paper, in plain loops, in the order the paper states the scheme.
 *
 * Layout: populations f[i][y][x], i = 0..12, dense (index (i*ny + y)*nx + x).
 * State f(t) = pre-collision populations after t steps.
 *
 * Readings of the paper taken here (each one is listed in the design notes):
 *   - q polynomial is x(x^2+y^2-3) (the printed "+3" is not orthogonal), sec. 2.
 *   - moment index range 0..12 (the printed "0..8" covers only D2Q9), sec. 2.
 *   - s_XY = s_XX, s_qy = s_qx, s_ry = s_rx (rates not listed for them), sec. 2.
 *   - body force added to j after relaxation, equilibria from pre-force j,
 *     no work term on E; u = (j + F/2)/rho on read-back, secs. 5 and 8.
 *   - uniform energy source Q added to E after relaxation, equilibria from the
 *     pre-source E, sec. 9.
 *   - walls are half a spacing outside the first/last node; links crossing a
 *     wall reverse their path (bounce-back of the whole velocity); links with a
 *     tangential component use bounce-back, links normal to a temperature wall
 *     use anti-bounce-back, adiabatic walls use bounce-back only, sec. 7,
 *     eq. (d2q13-cl-abb); wall density extrapolated linearly from the first two
 *     fluid layers, E and XX imposed.
 *   - temperature T = E - (13/2)(ux^2+uy^2), sec. 7.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 13

/* Velocity set: eqs (d2q5-vitesses), (d2q9-vitesses), (d2q13-vitesses). */
static const int VX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0};
static const int VY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2};

/* Moment order of eq (d2q13-polynomes). */
enum { M_RHO = 0, M_E, M_EPS, M_VARPI, M_JX, M_JY, M_QX, M_QY, M_RX, M_RY, M_XX, M_XY, M_XXE };

/* side kinds */
enum { OR_PERIODIC = 0, OR_ADIABATIC = 1, OR_DIRICHLET_T = 2 };
/* sides: 0 = West (x = -1/2), 1 = East (x = nx - 1/2), 2 = South (y = -1/2), 3 = North (y = ny - 1/2) */

typedef struct {
    double Pr, E0, c1, k2, c_epsE, c_varpi_rho, c_varpi_E; /* free equilibrium coefficients, sec. 2 */
    double s_XX, s_rx, s_eps, s_varpi, s_XXe;              /* free relaxation rates, sec. 2 */
    double F0x, F0y;                                       /* uniform body force, sec. 8 */
    double gx, gy, rho0;                                   /* buoyancy F = g (rho - rho0), sec. 5 */
    int collide;                                           /* 0: streaming and walls only */
    double Q_E;                                            /* uniform volumic energy source, sec. 9 */
} or13_params;

typedef struct {
    int kind[4];
    double u_t[4]; /* tangential wall velocity */
    double T_w[4]; /* wall temperature (Dirichlet walls) */
} or13_sides;

typedef struct {
    double A, Y, h1, k1, h2, c2, c_eps_rho;
    double sigma_XX, sigma_q, s_q;
    double nu, kappa, cs2, B, kappa_E;
} or13_derived;

/* ------------------------------------------------------------------------ */
/* Moment matrix M_kj = p_k(v_j), eqs (d2q13-moments), (d2q13-polynomes).     */
/* Each polynomial is evaluated exactly in integers after multiplying it by   */
/* its common denominator; the result must divide evenly.                     */

static int exact_div(long num, long den)
{
    if (num % den != 0) {
        fprintf(stderr, "oracle13: moment polynomial is not integer on the lattice\n");
        abort();
    }
    return (int)(num / den);
}

static int poly(int k, int x, int y)
{
    long r = (long)x * x + (long)y * y;
    long xx_yy = (long)x * x - (long)y * y;
    switch (k) {
    case M_RHO: return 1;
    case M_E: return (int)(-28 + 13 * r);
    case M_EPS: return exact_div(280 + r * (-361 + 77 * r), 2);             /* 140 + r(-361/2 + 77r/2) */
    case M_VARPI: return exact_div(-288 + r * (1162 + r * (-819 + 137 * r)), 24); /* -12 + r(581/12 + r(-273/8 + 137r/24)) */
    case M_JX: return x;
    case M_JY: return y;
    case M_QX: return (int)(x * (r - 3));
    case M_QY: return (int)(y * (r - 3));
    case M_RX: return exact_div(x * (202 + r * (-189 + 35 * r)), 12);      /* x(101/6 + r(-63/4 + 35r/12)) */
    case M_RY: return exact_div(y * (202 + r * (-189 + 35 * r)), 12);
    case M_XX: return (int)xx_yy;
    case M_XY: return x * y;
    case M_XXE: return exact_div(xx_yy * (-65 + 17 * r), 12);               /* (x^2-y^2)(-65/12 + 17r/12) */
    }
    abort();
}

static double Mm[Q][Q];  /* M[k][j] */
static double Dk[Q];     /* D_k = sum_j M_kj^2 (the basis is orthogonal) */
static int matrix_ready = 0;

static void build_matrix(void)
{
    if (matrix_ready) return;
    for (int k = 0; k < Q; ++k) {
        double d = 0.0;
        for (int j = 0; j < Q; ++j) {
            Mm[k][j] = (double)poly(k, VX[j], VY[j]);
            d += Mm[k][j] * Mm[k][j];
        }
        Dk[k] = d;
    }
    matrix_ready = 1;
}

void or13_matrix(double *M_out /* 13*13 row-major */, double *D_out /* 13 */)
{
    build_matrix();
    for (int k = 0; k < Q; ++k) {
        for (int j = 0; j < Q; ++j) M_out[k * Q + j] = Mm[k][j];
        D_out[k] = Dk[k];
    }
}

void or13_velocities(int *vx, int *vy)
{
    for (int j = 0; j < Q; ++j) { vx[j] = VX[j]; vy[j] = VY[j]; }
}

/* ------------------------------------------------------------------------ */
/* Parameter constraints, eqs (d2q13-henon), (d2q13-diffusion),              */
/* (d2q13-sigma-qx).  nu, kappa, cs2 and kappa_E are transport coefficients  */
/* of the scheme: cs2 from the first-order system (d2q13-equiv-edp-ordre-1), */
/* kappa = nu / Pr by definition of the Prandtl number, nu from the second-  */
/* order expansion, kappa_E = E-conductivity in steady conduction (j = 0).   */
/* Returns 0, or -1 when a rate leaves (0, 2), A = 13 c1 + 95 + 2 E0 <= 0    */
/* (no positive sound speed or viscosity) or the inputs are degenerate.     */
int or13_derive(const or13_params *p, or13_derived *d)
{
    double c1 = p->c1, E0 = p->E0, k2 = p->k2, ceE = p->c_epsE;
    d->A = 13.0 * c1 + 95.0 + 2.0 * E0;
    d->Y = 114404.0 + 51051.0 * c1 - 11492.0 * ceE + 7854.0 * E0;
    d->sigma_XX = 1.0 / p->s_XX - 0.5;                                   /* (d2q13-henon) */
    d->h1 = 17.0 / 26.0 - c1 / 2.0 - E0 / 13.0;                          /* (d2q13-diffusion) */
    d->k1 = 2.0 / 13.0;
    d->h2 = -(39.0 / 2.0 + 13.0 / 2.0 * c1 + E0) * k2
            - 7.0 / 624.0 * d->A * (874481.0 + 459459.0 * c1 - 103428.0 * ceE + 70686.0 * E0) / d->Y;
    d->sigma_q = -1309.0 / 2.0 * d->sigma_XX * d->A / d->Y;             /* (d2q13-sigma-qx) */
    d->s_q = 1.0 / (d->sigma_q + 0.5);
    d->c_eps_rho = 140.0 + 28.0 * ceE + d->A * d->Y / (22984.0 * p->Pr);
    d->c2 = -65.0 / 24.0 - 21.0 / 8.0 * (c1 + d->h1 + d->k1 * E0) - k2 * E0 - d->h2;
    d->nu = d->sigma_XX * d->A / 104.0;
    d->kappa = d->nu / p->Pr;
    d->cs2 = d->A / 52.0;
    d->B = (39.0 + 13.0 * c1 + 2.0 * E0) / 2.0;
    d->kappa_E = d->kappa * (28.0 + d->B) / 28.0;
    double rates[6] = {p->s_XX, p->s_rx, p->s_eps, p->s_varpi, p->s_XXe, d->s_q};
    for (int i = 0; i < 6; ++i)
        if (!(rates[i] > 0.0 && rates[i] < 2.0)) return -1;
    if (!(d->Y != 0.0) || !(p->Pr > 0.0)) return -1;
    /* A <= 0: the squared sound speed A/52 and the viscosity sigma_XX A/104 are not positive */
    if (!(d->A > 0.0) || !(d->nu > 0.0) || !(d->cs2 > 0.0)) return -1;
    return 0;
}

/* Equilibrium moments, eq (d2q13-moments-equil). */
static void equilibrium(const or13_params *p, const or13_derived *d,
                        double rho, double jx, double jy, double E, double meq[Q])
{
    meq[M_RHO] = rho;
    meq[M_E] = E;
    meq[M_EPS] = d->c_eps_rho * rho + p->c_epsE * E;
    meq[M_VARPI] = p->c_varpi_rho * rho + p->c_varpi_E * E;
    meq[M_JX] = jx;
    meq[M_JY] = jy;
    meq[M_QX] = jx * (p->c1 + d->h1 * rho + d->k1 * E);
    meq[M_QY] = jy * (p->c1 + d->h1 * rho + d->k1 * E);
    meq[M_RX] = jx * (d->c2 + d->h2 * rho + p->k2 * E);
    meq[M_RY] = jy * (d->c2 + d->h2 * rho + p->k2 * E);
    meq[M_XX] = (jx * jx - jy * jy) / rho;
    meq[M_XY] = jx * jy / rho;
    meq[M_XXE] = 0.0;
}

void or13_equilibrium_moments(const or13_params *p, double rho, double jx, double jy, double E, double *meq)
{
    or13_derived d;
    build_matrix();
    or13_derive(p, &d);
    equilibrium(p, &d, rho, jx, jy, E, meq);
}

/* f_j = sum_k M_kj m_k / D_k  (inverse of an orthogonal basis). */
static void moments_to_f(const double m[Q], double f[Q])
{
    for (int j = 0; j < Q; ++j) {
        double s = 0.0;
        for (int k = 0; k < Q; ++k) s += Mm[k][j] * m[k] / Dk[k];
        f[j] = s;
    }
}

static void f_to_moments(const double f[Q], double m[Q])
{
    for (int k = 0; k < Q; ++k) {
        double s = 0.0;
        for (int j = 0; j < Q; ++j) s += Mm[k][j] * f[j];
        m[k] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Initial state f = f^eq(rho, j = rho u, E = T + (13/2)|u|^2).              */
void or13_init(int nx, int ny, const double *rho, const double *ux, const double *uy, const double *T,
               const or13_params *p, double *f)
{
    or13_derived d;
    build_matrix();
    or13_derive(p, &d);
    long n = (long)nx * ny;
    for (long c = 0; c < n; ++c) {
        double m[Q], fl[Q];
        double u2 = ux[c] * ux[c] + uy[c] * uy[c];
        equilibrium(p, &d, rho[c], rho[c] * ux[c], rho[c] * uy[c], T[c] + 6.5 * u2, m);
        moments_to_f(m, fl);
        for (int i = 0; i < Q; ++i) f[i * n + c] = fl[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Collision at every node: m = M f; relax the nine non-conserved moments;   */
/* add the body force to j; f* = M^-1 m*.                                     */
void or13_collide(int nx, int ny, const double *f, const or13_params *p, double *fstar)
{
    or13_derived d;
    build_matrix();
    or13_derive(p, &d);
    long n = (long)nx * ny;
    double s[Q] = {0};
    s[M_EPS] = p->s_eps;
    s[M_VARPI] = p->s_varpi;
    s[M_QX] = d.s_q;
    s[M_QY] = d.s_q;
    s[M_RX] = p->s_rx;
    s[M_RY] = p->s_rx;
    s[M_XX] = p->s_XX;
    s[M_XY] = p->s_XX;
    s[M_XXE] = p->s_XXe;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) {
        double fl[Q], m[Q], meq[Q], ms[Q], fs[Q];
        for (int i = 0; i < Q; ++i) fl[i] = f[i * n + c];
        if (!p->collide) {
            for (int i = 0; i < Q; ++i) fstar[i * n + c] = fl[i];
            continue;
        }
        f_to_moments(fl, m);
        equilibrium(p, &d, m[M_RHO], m[M_JX], m[M_JY], m[M_E], meq);
        for (int k = 0; k < Q; ++k) ms[k] = m[k] - s[k] * (m[k] - meq[k]);
        double Fx = p->F0x + p->gx * (m[M_RHO] - p->rho0);
        double Fy = p->F0y + p->gy * (m[M_RHO] - p->rho0);
        ms[M_JX] = m[M_JX] + Fx;
        ms[M_JY] = m[M_JY] + Fy;
        ms[M_E] = m[M_E] + p->Q_E; /* energy source after relaxation (sec. 9) */
        moments_to_f(ms, fs);
        for (int i = 0; i < Q; ++i) fstar[i * n + c] = fs[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Wall rule helpers, sec. 7 and eq (d2q13-cl-abb).                           */

static double node_rho(const double *f, long n, long c)
{
    double s = 0.0;
    for (int i = 0; i < Q; ++i) s += f[i * n + c];
    return s;
}

static double node_E(const double *f, long n, long c)
{
    double s = 0.0;
    for (int i = 0; i < Q; ++i) s += Mm[M_E][i] * f[i * n + c];
    return s;
}

/* Equilibrium moments of wall `w` on the wall-normal line through node (x, y),
 * from the time-t state f: rho_W = (3 rho_0 - rho_1)/2 (linear extrapolation to
 * the wall half a spacing outside layer 0), j_W = rho_W u_W, E_W = T_W + (13/2)u_W^2
 * for temperature walls or E of layer 0 for adiabatic walls. */
static void wall_equilibrium(int nx, int ny, const double *f, const or13_params *p, const or13_derived *d,
                             const or13_sides *sd, int w, int x, int y, double meq[Q])
{
    long n = (long)nx * ny;
    long c0, c1;
    if (w == 0) { c0 = (long)y * nx + 0; c1 = (long)y * nx + 1; }
    else if (w == 1) { c0 = (long)y * nx + (nx - 1); c1 = (long)y * nx + (nx - 2); }
    else if (w == 2) { c0 = 0L * nx + x; c1 = 1L * nx + x; }
    else { c0 = (long)(ny - 1) * nx + x; c1 = (long)(ny - 2) * nx + x; }
    double rho0 = node_rho(f, n, c0), rho1 = node_rho(f, n, c1);
    double rhoW = 0.5 * (3.0 * rho0 - rho1);
    double ut = sd->u_t[w];
    double jx = (w < 2) ? 0.0 : rhoW * ut;
    double jy = (w < 2) ? rhoW * ut : 0.0;
    double EW = (sd->kind[w] == OR_DIRICHLET_T) ? sd->T_w[w] + 6.5 * ut * ut : node_E(f, n, c0);
    equilibrium(p, d, rhoW, jx, jy, EW, meq);
}

/* ------------------------------------------------------------------------ */
/* Streaming f_i(x, t+1) = f*_i(x - v_i) with periodic wrap, and the wall     */
/* rule for sources beyond a wall.  f is the time-t state (for wall density),  */
/* fstar the post-collision populations, fout receives f(t+1).                 */
void or13_stream(int nx, int ny, const double *f, const double *fstar, const or13_params *p,
                 const or13_sides *sd, double *fout)
{
    or13_derived d;
    build_matrix();
    or13_derive(p, &d);
    long n = (long)nx * ny;
    int xper = (sd->kind[0] == OR_PERIODIC);
    int yper = (sd->kind[2] == OR_PERIODIC);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            long c = (long)y * nx + x;
            for (int i = 0; i < Q; ++i) {
                int sx = x - VX[i], sy = y - VY[i];
                int wall = -1;
                if (xper) sx = ((sx % nx) + nx) % nx;
                else if (sx < 0) wall = 0;
                else if (sx >= nx) wall = 1;
                if (yper) sy = ((sy % ny) + ny) % ny;
                else if (wall < 0 && sy < 0) wall = 2;
                else if (wall < 0 && sy >= ny) wall = 3;
                if (wall < 0) {
                    fout[i * n + c] = fstar[i * n + (long)sy * nx + sx];
                    continue;
                }
                /* path reversal: source node x' reflected through the wall, tangential coordinate kept */
                int px = x, py = y;
                if (wall == 0) px = -1 + VX[i] - x;
                if (wall == 1) px = 2 * nx - 1 + VX[i] - x;
                if (wall == 2) py = -1 + VY[i] - y;
                if (wall == 3) py = 2 * ny - 1 + VY[i] - y;
                int opp = -1;
                for (int j = 0; j < Q; ++j)
                    if (VX[j] == -VX[i] && VY[j] == -VY[i]) opp = j;
                int normal = (wall < 2) ? (VY[i] == 0) : (VX[i] == 0);
                int abb = normal && sd->kind[wall] == OR_DIRICHLET_T;
                double meq[Q];
                wall_equilibrium(nx, ny, f, p, &d, sd, wall, x, y, meq);
                double extra = 0.0;
                for (int k = 0; k < Q; ++k) {
                    int odd = (k == M_JX || k == M_JY || k == M_QX || k == M_QY || k == M_RX || k == M_RY);
                    if (abb ? !odd : odd) extra += 2.0 * Mm[k][i] * meq[k] / Dk[k];
                }
                double src = fstar[opp * n + (long)py * nx + px];
                fout[i * n + c] = (abb ? -src : src) + extra;
            }
        }
    }
}

/* One full step t -> t+1.  fstar_out may be NULL (scratch allocated here). */
int or13_step(int nx, int ny, const double *f, const or13_params *p, const or13_sides *sd,
              double *fout, double *fstar_out)
{
    long n = (long)nx * ny;
    double *fs = fstar_out ? fstar_out : (double *)malloc(sizeof(double) * Q * n);
    if (!fs) return -2;
    or13_collide(nx, ny, f, p, fs);
    or13_stream(nx, ny, f, fs, p, sd, fout);
    if (!fstar_out) free(fs);
    return 0;
}

/* n steps in place on f (ping-pong through a scratch buffer). */
int or13_run(int nx, int ny, double *f, const or13_params *p, const or13_sides *sd, long steps)
{
    long n = (long)nx * ny;
    double *a = f;
    double *b = (double *)malloc(sizeof(double) * Q * n);
    double *fs = (double *)malloc(sizeof(double) * Q * n);
    if (!b || !fs) { free(b); free(fs); return -2; }
    for (long t = 0; t < steps; ++t) {
        or13_collide(nx, ny, a, p, fs);
        or13_stream(nx, ny, a, fs, p, sd, b);
        double *tmp = a; a = b; b = tmp;
    }
    if (a != f) { memcpy(f, a, sizeof(double) * Q * n); b = a; }
    free(b);
    free(fs);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Read-back at time t: rho = sum f, j = sum v f, E = sum M_E f,             */
/* F = F0 + g(rho - rho0), u = (j + F/2)/rho, T = E - (13/2)|u|^2 (sec. 7).  */
void or13_moments(int nx, int ny, const double *f, const or13_params *p,
                  double *rho, double *ux, double *uy, double *T)
{
    build_matrix();
    long n = (long)nx * ny;
    for (long c = 0; c < n; ++c) {
        double fl[Q], m[Q];
        for (int i = 0; i < Q; ++i) fl[i] = f[i * n + c];
        f_to_moments(fl, m);
        double Fx = p->F0x + p->gx * (m[M_RHO] - p->rho0);
        double Fy = p->F0y + p->gy * (m[M_RHO] - p->rho0);
        double u = (m[M_JX] + 0.5 * Fx) / m[M_RHO];
        double v = (m[M_JY] + 0.5 * Fy) / m[M_RHO];
        rho[c] = m[M_RHO];
        ux[c] = u;
        uy[c] = v;
        T[c] = m[M_E] - 6.5 * (u * u + v * v);
    }
}

/* ------------------------------------------------------------------------ */
/* Diagnostics of the time-t state (all FP64):                                */
/*  out[0..3]  sum rho, sum jx, sum jy, sum E  (pre-collision)                */
/*  out[4]     net x-flux of E through the interior faces x+1/2, 1 <= x <= nx-3, */
/*             minus B times the mass flux through the same faces, summed over */
/*             faces and rows (exact face-crossing count of the post-collision  */
/*             populations; faces a reflected speed-2 link can reach are left  */
/*             out).  With a periodic x axis every face counts.                */
/*  out[5]     mean Nusselt number over the cavity, Table 1:                   */
/*             out[4] / (faces * ny) * nx / (kappa_E (T_W - T_E))              */
/*  out[6]     max |u|                                                         */
/*  out[7]     max |u(x) + u(xbar)|, xbar the point reflected through the     */
/*             domain centre (Fig. 14)                                         */
/*  out[8]     out[7] / out[6]                                                 */
/*  out[9]     number of non-finite populations                                */
/*  out[10]    min rho                                                         */
/* Why J_E - B j: linearised about rest, the equilibrium E flux is B j and the  */
/* E-perturbation flux carries the factor (28 + B)/28 both in advection and in   */
/* conduction, so (J_E - B j) / ((28+B)/28) = u dE - kappa dE/dx, the heat flux  */
/* whose wall-normal mean defines the Nusselt number.                          */
void or13_diagnostics(int nx, int ny, const double *f, const or13_params *p, const or13_sides *sd,
                      double *out)
{
    or13_derived d;
    build_matrix();
    or13_derive(p, &d);
    long n = (long)nx * ny;
    double *rho = malloc(sizeof(double) * n), *ux = malloc(sizeof(double) * n);
    double *uy = malloc(sizeof(double) * n), *T = malloc(sizeof(double) * n);
    double *fs = malloc(sizeof(double) * Q * n);
    or13_moments(nx, ny, f, p, rho, ux, uy, T);
    or13_collide(nx, ny, f, p, fs);
    int xper = (sd->kind[0] == OR_PERIODIC);
    int flo = xper ? 0 : 1, fhi = xper ? nx - 1 : nx - 3; /* counted faces x+1/2, flo <= x <= fhi */
    double srho = 0, sjx = 0, sjy = 0, sE = 0, sJ = 0, umax = 0, asym = 0, nonfin = 0, rmin = INFINITY;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long c = (long)y * nx + x;
            double fl[Q], m[Q];
            for (int i = 0; i < Q; ++i) {
                fl[i] = f[i * n + c];
                if (!isfinite(fl[i])) nonfin += 1.0;
            }
            f_to_moments(fl, m);
            srho += m[M_RHO];
            sjx += m[M_JX];
            sjy += m[M_JY];
            sE += m[M_E];
            for (int i = 0; i < Q; ++i) {
                /* faces crossed by the link leaving (x, y) with velocity v_i */
                int cnt = 0;
                if (VX[i] > 0) {
                    for (int xf = x; xf < x + VX[i]; ++xf)
                        if (xper || (xf >= flo && xf <= fhi)) cnt += 1;
                } else if (VX[i] < 0) {
                    for (int xf = x + VX[i]; xf < x; ++xf)
                        if (xper || (xf >= flo && xf <= fhi)) cnt -= 1;
                }
                sJ += (Mm[M_E][i] - d.B) * cnt * fs[i * n + c];
            }
            double um = sqrt(ux[c] * ux[c] + uy[c] * uy[c]);
            if (um > umax) umax = um;
            if (rho[c] < rmin) rmin = rho[c];
        }
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long c = (long)y * nx + x, cb = (long)(ny - 1 - y) * nx + (nx - 1 - x);
            double ax = ux[c] + ux[cb], ay = uy[c] + uy[cb];
            double a = sqrt(ax * ax + ay * ay);
            if (a > asym) asym = a;
        }
    /* Energy exchanged with each wall in the next step (sec. 7 walls): an
       incoming link (x, i) whose source x - v_i lies beyond wall w brings
       M_E,i f_i(x, t+1); an outgoing link (x, j) whose target x + v_j lies
       beyond w takes M_E,j f*_j(x, t).  A link beyond an x wall and a y wall
       counts for the x wall, as in the streaming. */
    double *fn = malloc(sizeof(double) * Q * n);
    or13_stream(nx, ny, f, fs, p, sd, fn);
    int yper = (sd->kind[2] == OR_PERIODIC);
    double wflux[4] = {0.0, 0.0, 0.0, 0.0}, wmass[4] = {0.0, 0.0, 0.0, 0.0};
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long c = (long)y * nx + x;
            for (int i = 0; i < Q; ++i) {
                for (int dir = -1; dir <= 1; dir += 2) {
                    int sx = x + dir * VX[i], sy = y + dir * VY[i], w = -1;
                    if (!xper && sx < 0) w = 0;
                    else if (!xper && sx >= nx) w = 1;
                    else if (!yper && sy < 0) w = 2;
                    else if (!yper && sy >= ny) w = 3;
                    if (w < 0) continue;
                    double v = dir < 0 ? fn[i * n + c] : -fs[i * n + c];  /* incoming, outgoing */
                    wflux[w] += Mm[M_E][i] * v;
                    wmass[w] += v;
                }
            }
        }
    free(fn);
    double dT = sd->T_w[0] - sd->T_w[1];
    int faces = xper ? nx : (fhi - flo + 1);
    out[0] = srho;
    out[1] = sjx;
    out[2] = sjy;
    out[3] = sE;
    out[4] = sJ;
    out[5] = (dT != 0.0 && faces > 0) ? sJ / ((double)faces * ny) * nx / (d.kappa_E * dT) : 0.0;
    out[6] = umax;
    out[7] = asym;
    out[8] = umax > 0 ? asym / umax : 0.0;
    out[9] = nonfin;
    out[10] = rmin;
    /* wall Nusselt numbers: energy per step through the West (in) and East (out)
       walls per unit wall length, less B times the mass exchanged (the advected
       equilibrium part, as in the face flux), over the conduction flux kappa_E dT / nx */
    double wscale = (!xper && dT != 0.0) ? (double)nx / (d.kappa_E * dT) / ny : 0.0;
    out[11] = (wflux[0] - d.B * wmass[0]) * wscale;
    out[12] = -(wflux[1] - d.B * wmass[1]) * wscale;
    out[13] = wflux[0] + wflux[1] + wflux[2] + wflux[3];
    out[14] = wmass[0] + wmass[1] + wmass[2] + wmass[3];
    free(rho); free(ux); free(uy); free(T); free(fs);
}

/* Fourier projection of rho, u_x, u_y and E (sec. 6 aggregates):
   out[2q] + i out[2q+1] = sum_{x,y} q(x, y) exp(-2 pi i (kx x / nx + ky y / ny)). */
void or13_fourier(int nx, int ny, const double *f, const or13_params *p, int kx, int ky, double *out)
{
    build_matrix();
    long n = (long)nx * ny;
    double *rho = malloc(sizeof(double) * n), *ux = malloc(sizeof(double) * n);
    double *uy = malloc(sizeof(double) * n), *T = malloc(sizeof(double) * n);
    or13_moments(nx, ny, f, p, rho, ux, uy, T);
    for (int k = 0; k < 8; ++k) out[k] = 0.0;
    const double pi = 3.14159265358979323846;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long c = (long)y * nx + x;
            double fl[Q], m[Q];
            for (int i = 0; i < Q; ++i) fl[i] = f[i * n + c];
            f_to_moments(fl, m);
            double th = 2.0 * pi * ((double)kx * x / nx + (double)ky * y / ny);
            double cr = cos(th), ci = -sin(th);
            double q[4] = {rho[c], ux[c], uy[c], m[M_E]};
            for (int k = 0; k < 4; ++k) {
                out[2 * k] += q[k] * cr;
                out[2 * k + 1] += q[k] * ci;
            }
        }
    free(rho); free(ux); free(uy); free(T);
}

int or13_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the OpenMP loops from now on (n > 0); each node's update is
 * independent, so results do not depend on it. */
void or13_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
