/*
 * lbm13.h -- C ABI of the MI355X (gfx950) D2Q13 "energy-conserving" lattice
 * Boltzmann step of Lallemand & Dubois, "Comparison of Simulations of Convective
 * Flows" (Commun. Comput. Phys. 2015).
 *
 * One time step (sec. 2, sec. 7): at every node the 13 populations are mapped
 * to the 13 orthogonal moments of eq (d2q13-polynomes); rho, E, jx, jy are
 * conserved; the nine other moments relax toward the equilibria of eq
 * (d2q13-moments-equil) with the rates of eqs (d2q13-henon), (d2q13-diffusion),
 * (d2q13-sigma-qx); the body force (secs. 5, 8) is added to j and the uniform
 * energy source (sec. 9) to E; the inverse
 * transform gives the post-collision populations, which move along the 13
 * velocities (eq d2q13-vitesses, reach 1 and 2).  Links that leave the domain
 * through a wall come back by bounce-back (links with a tangential component,
 * and every link at an adiabatic wall) or anti-bounce-back (links normal to a
 * temperature wall), eq (d2q13-cl-abb).
 *
 * Conventions shared by every call:
 *  - Every function returns an int status (LBM13_OK or a negative code); no
 *    exception, abort or exit crosses the ABI.  lbm13_last_error() gives a
 *    message for the last failing call on a context.
 *  - Device memory is owned by the caller: lbm13_create() adopts a device
 *    workspace of lbm13_workspace_bytes() bytes and never frees it.  Field
 *    arguments marked "device" are device pointers, row-major [y][x] with x
 *    fastest, nx*ny doubles each, unless stated otherwise.
 *  - Work is enqueued on the caller's HIP stream (hipStream_t passed as void*;
 *    NULL = the null stream) and is asynchronous unless a call says it
 *    synchronises.
 *  - A context is not thread-safe; distinct contexts are independent.
 *  - Grid: node (x, y), 0 <= x < nx, 0 <= y < ny, nx, ny >= 2.  A non-periodic
 *    side is a straight wall half a spacing outside the first/last node.
 *  - State: the library keeps the post-collision populations f*(t) of the
 *    current step, stored as deviations from the rest populations
 *    f^eq(rho = 1, j = 0, E = E0) in FP64 or FP32 (precision chosen at create).
 */
#ifndef LBM13_H
#define LBM13_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LBM13_OK 0
#define LBM13_EINVAL (-1)           /* bad argument, size or pointer */
#define LBM13_ENOMEM (-2)           /* workspace smaller than lbm13_workspace_bytes() */
#define LBM13_EDEVICE (-3)          /* a HIP runtime call or kernel launch failed */
#define LBM13_EUNSTABLE_PARAMS (-4) /* a relaxation rate (given or derived) outside (0, 2), or degenerate constants */
#define LBM13_ENONFINITE (-5)       /* diagnostics found a non-finite population or rho <= 0 */
#define LBM13_ESTATE (-6)           /* call out of order (e.g. step before set_params / init) */

/* storage and arithmetic precision of the populations */
#define LBM13_FP64 0      /* FP64 storage and collision */
#define LBM13_FP32_DEV 1  /* FP32 deviations from rest, FP32 collision, FP64 reductions */

/* side kinds; sides are indexed 0 = West (x = -1/2), 1 = East (x = nx - 1/2),
 * 2 = South (y = -1/2), 3 = North (y = ny - 1/2).  Opposite sides are both
 * periodic or both walls. */
#define LBM13_PERIODIC 0
#define LBM13_WALL_ADIABATIC 1   /* bounce-back on every link: no mass or energy flux (sec. 9, Table 1 cavity) */
#define LBM13_WALL_DIRICHLET_T 2 /* bounce-back on tangential links, anti-bounce-back on normal links (sec. 7) */

/* One side of the domain.  u_tangential: wall velocity along the wall (along y
 * for West/East, along x for South/North).  T_wall: imposed temperature
 * T = E - (13/2)|u|^2 (sec. 7), used by LBM13_WALL_DIRICHLET_T sides. */
typedef struct {
    int kind;
    double u_tangential;
    double T_wall;
} lbm13_side;

/* Free parameters of the scheme, as listed after eq (d2q13-sigma-qx): the
 * Prandtl number, E0 (energy of the rest state at rho = 1), c1, k2, c_epsE,
 * c_varpi_rho, c_varpi_E and the relaxation rates s_XX (also used for XY),
 * s_rx (also ry), s_eps, s_varpi, s_XXe.  Forces: F = F0 + g (rho - rho0) is
 * added to j after relaxation (F0: sec. 8 pressure gradient; g: sec. 5
 * buoyancy).  collide = 0 skips the collision (streaming and walls only).
 * Q_E: uniform volumic energy source added to E after relaxation (sec. 9). */
typedef struct {
    double s_XX, s_rx, s_eps, s_varpi, s_XXe;
    double Pr, E0, c1, k2, c_epsE, c_varpi_rho, c_varpi_E;
    double F0[2];
    double g[2];
    double rho0;
    int collide;
    double Q_E;
} lbm13_params;

/* Coefficients derived from lbm13_params by the constraints of eqs
 * (d2q13-diffusion), (d2q13-sigma-qx), and transport coefficients of the
 * scheme: nu (shear viscosity), kappa = nu/Pr (thermal diffusivity), cs2
 * (squared sound speed, from eq d2q13-equiv-edp-ordre-1), B (equilibrium
 * E-flux per unit momentum), kappa_E = kappa (28 + B)/28 (E-conductivity). */
typedef struct {
    double A, Y, h1, k1, h2, c2, c_eps_rho;
    double sigma_XX, sigma_q, s_q;
    double nu, kappa, cs2, B, kappa_E;
} lbm13_derived;

typedef struct lbm13_ctx lbm13_ctx;

/* Host-only: derive the constrained coefficients (eqs d2q13-henon,
 * d2q13-diffusion, d2q13-sigma-qx).  Returns LBM13_EUNSTABLE_PARAMS when a rate
 * (given or the derived s_q) leaves (0, 2), Pr <= 0, or A = 13 c1 + 95 + 2 E0
 * <= 0 (then cs2 = A/52 and nu = sigma_XX A/104 are not positive); `out` is
 * filled in either case.  No device access.  lbm13_set_params applies the same
 * checks. */
int lbm13_derive(const lbm13_params *p, lbm13_derived *out);

/* Bytes of device workspace a single domain nx x ny in `precision` needs
 * (both population buffers, parameter block, tile table, reduction partials).
 * Returns 0 for invalid sizes.  Host-only. */
size_t lbm13_workspace_bytes(int nx, int ny, int precision);

/* Create a context on the current HIP device.  `workspace` is a device
 * allocation of at least lbm13_workspace_bytes(nx, ny, precision) bytes, 256-
 * byte aligned, owned by the caller and kept alive until lbm13_destroy().
 * `stream` is the hipStream_t every call enqueues on.  *out receives the
 * context (NULL on failure).  Errors: EINVAL (sizes, NULL), ENOMEM (too small). */
int lbm13_create(int nx, int ny, int precision, void *workspace, size_t workspace_bytes, void *stream,
                 lbm13_ctx **out);

/* Set the scheme's parameters and the four sides (W, E, S, N).  Derives the
 * constrained coefficients on the host in FP64 and uploads them (async copy
 * of a host staging block that the context owns).  `derived` may be NULL.
 * Errors: EINVAL (inconsistent periodicity), EUNSTABLE_PARAMS. */
int lbm13_set_params(lbm13_ctx *ctx, const lbm13_params *p, const lbm13_side sides[4], lbm13_derived *derived);

/* Initial state from macroscopic fields (device pointers, nx*ny doubles):
 * populations f(0) = f^eq(rho, j = rho u, E = T + (13/2)|u|^2) (sec. 7 relation
 * between T and E), then one collision, so the kept state is f*(0).  Resets the
 * step counter.  Requires set_params. */
int lbm13_init_moments(lbm13_ctx *ctx, const double *rho, const double *ux, const double *uy, const double *T);

/* Enqueue n >= 0 time steps (stream, walls, collide) on the stream. Async. */
int lbm13_step(lbm13_ctx *ctx, long long n);

/* Macroscopic fields of the current state f(t) (device pointers, nx*ny doubles
 * each; any of them may be NULL): rho = sum f, u = (j + F/2)/rho with
 * F = F0 + g(rho - rho0), T = E - (13/2)|u|^2 (sec. 7).  Async. */
int lbm13_moments(lbm13_ctx *ctx, double *rho, double *ux, double *uy, double *T);

/* FP64 diagnostics of the current state, written to the host array out[16]
 * (synchronises the stream):
 *  [0] sum rho  [1] sum jx  [2] sum jy  [3] sum E      (state f(t))
 *  [4] heat flux: sum over interior faces x+1/2 (1 <= x <= nx-3; every face if
 *      x is periodic) and rows of the face-crossing flux of (M_E - B) carried
 *      by f*(t)
 *  [5] mean Nusselt number, Table 1: [4]/(faces*ny) * nx / (kappa_E (T_W - T_E))
 *      (0 when T_W == T_E)
 *  [6] max |u|  [7] max |u(x) + u(xbar)| with xbar the node reflected through
 *      the domain centre (Fig. 14)  [8] [7]/[6]
 *  [9] count of non-finite stored values  [10] min rho
 *  walls (sec. 7), for the exchange of the next step: an incoming link whose
 *  source lies beyond a wall brings its bounce-back / anti-bounce-back value,
 *  an outgoing link whose target lies beyond it takes f*; a link beyond an x
 *  and a y wall counts for the x wall:
 *  [11] Nu at the West wall: (energy - B mass) taken in per step, per unit
 *       wall length, times nx / (kappa_E (T_W - T_E))  [12] the same given out
 *       at the East wall (0 when x is periodic or T_W == T_E)
 *  [13] energy taken in through all walls per step (sum E(t+1) - sum E(t)
 *       - Q_E nx ny)  [14] mass taken in (sum rho(t+1) - sum rho(t); nonzero
 *       where anti-bounce-back links let mass through)  [15] reserved (0).
 * Returns LBM13_ENONFINITE (with out filled) when [9] > 0 or [10] <= 0. */
int lbm13_diagnostics(lbm13_ctx *ctx, double out[16]);

/* Fourier projection of the current state (sec. 6 aggregates), written to the
 * host array out[8] (synchronises): out[2q] + i out[2q+1] =
 * sum_{x,y} q(x, y) exp(-2 pi i (kx x / nx + ky y / ny)) for q = rho, u_x,
 * u_y, E (u and E as in lbm13_moments; E = T + (13/2)|u|^2).  Any integers
 * kx, ky.  FP64 accumulation in a fixed order. */
int lbm13_fourier(lbm13_ctx *ctx, int kx, int ky, double out[8]);

/* Copy the kept post-collision populations f*(t) as absolute FP64 values into
 * the device array dst[13][ny][nx] (dense), or load them from src (same
 * layout; the step counter is kept).  Async. */
int lbm13_get_state(lbm13_ctx *ctx, double *dst);
int lbm13_set_state(lbm13_ctx *ctx, const double *src);

/* Raw checkpoint of the kept state in the device buffer dst of dst_bytes >=
 * lbm13_state_bytes() bytes: a 256-byte header (magic "LBM13CK", format
 * version, precision, nx, ny, steps taken, payload bytes) followed by 13*ny*nx
 * values of the storage precision (8 bytes for LBM13_FP64, 4 for
 * LBM13_FP32_DEV), the stored deviations from the rest populations, dense
 * [13][ny][nx].  lbm13_save is async; EINVAL when dst is NULL or too small,
 * ESTATE before any state exists.  lbm13_load(ctx, src, src_bytes) requires
 * src_bytes == lbm13_state_bytes(), reads the header back (synchronises the
 * stream) and returns EINVAL, changing nothing, unless it names this context's
 * nx, ny and precision; it then restores the populations bit-exactly and the
 * step counter, so a run resumed from a checkpoint equals the uninterrupted
 * run.  src must be a device pointer. */
size_t lbm13_state_bytes(const lbm13_ctx *ctx);
int lbm13_save(lbm13_ctx *ctx, void *dst, size_t dst_bytes);
int lbm13_load(lbm13_ctx *ctx, const void *src, size_t src_bytes);

/* Number of steps taken since the last lbm13_init_moments() (which resets it). */
long long lbm13_steps_done(const lbm13_ctx *ctx);

/* Tile shape of the step kernel: tile_x in {32, 64} nodes along x, tile_y in
 * {4, 8, 16} rows (tile_x * tile_y >= 256).  Rebuilds the tile table.  EINVAL
 * for unsupported shapes. */
int lbm13_set_tile(lbm13_ctx *ctx, int tile_x, int tile_y);

/* Time every supported launch configuration (single-step tile shapes,
 * two-steps-per-launch tile shapes with and without the interior kernel,
 * three-steps-per-launch tile shapes) for
 * `steps` steps on the current state
 * (the state is advanced, so save it first if needed) and keep the fastest.
 * Writes the chosen kernel's tile shape to tile_x/tile_y when not NULL (see
 * lbm13_launch_config for the whole choice).  Synchronises. */
int lbm13_autotune(lbm13_ctx *ctx, int steps, int *tile_x, int *tile_y);

/* lbm13_autotune through a cache file (host path; created if missing): the
 * launch configuration tuned earlier for the same device architecture,
 * precision and size class (floor(log2) of the node count and of the domain
 * count, walls present or not) is applied without timing, else the autotuner
 * runs and its choice is stored.  The file is JSON, {"version": 1, "entries":
 * {key: [the six integers of lbm13_launch_config]}}; damaged content or an
 * entry this build does not support is ignored and tuned again.  *from_cache
 * (may be NULL) tells which happened.  A cache that cannot be written leaves
 * the tuned configuration in place, returns LBM13_OK and says so in
 * lbm13_last_error.  Synchronises when it tunes. */
int lbm13_autotune_cached(lbm13_ctx *ctx, int steps, const char *cache_path, int *from_cache);

/* Current launch configuration: cfg = {steps per launch, single-step tile_x,
 * tile_y, two- and three-step tile_x, tile_y, interior-kernel mode 0, 1 or 2
 * (lbm13_set_interior_kernel)}.
 * Host-only. */
int lbm13_launch_config(const lbm13_ctx *ctx, int cfg[6]);

/* Capture k steps (k even, 2..4096) into a HIP graph that lbm13_step() then
 * replays for every full block of k steps; k = 0 switches graphs off. */
int lbm13_use_graph(lbm13_ctx *ctx, int k);

/* Time steps advanced per kernel launch: 1, 2 (each workgroup advances its
 * tile and a two-node halo by one step into LDS, then the tile by a second
 * step; same arithmetic per node, so results equal two single steps, with
 * about half the HBM traffic per step) or 3 (tile + 4-node halo, then tile +
 * 2-node halo, then the tile: a third of the HBM traffic per step; any sides
 * and walls, wall states of the intermediate steps from the levels kept in
 * LDS; tiles far from walls and ragged edges run a kernel that keeps only the
 * windows the next level reads, the others also keep the slots the wall
 * fix-ups read for reflected populations;
 * the two-step tile must be a three-step shape: FP32 (64, 16), (32, 32),
 * (64, 8), (32, 16), (32, 8); FP64 (64, 8), (32, 16), (32, 8); lbm13_step returns
 * EINVAL otherwise).  A remainder of lbm13_step(n) is done by shorter
 * launches.  EINVAL for other values. */
int lbm13_set_steps_per_launch(lbm13_ctx *ctx, int k);

/* Tile of the two- and three-steps-per-launch kernels: (64, 16), (64, 12),
 * (64, 8), (64, 4), (32, 32), (32, 16), (32, 8) or (32, 4) nodes, both
 * precisions (three steps take the subset listed above).
 * Tiles whose region (tile + 2-node halo) and its sources lie inside the domain
 * away from walls and wraps run a kernel that keeps only 13 x tile values in
 * LDS; the others keep the region (up to 141 KB, FP64 64 x 16).
 * Defaults: (32, 32) FP32, (32, 16) FP64.  EINVAL otherwise. */
int lbm13_set_fused_tile(lbm13_ctx *ctx, int tile_x, int tile_y);

/* Two- and three-step launches: 1 (default) runs the tiles whose region lies
 * inside the domain away from walls (and, for two steps, wraps) on a separate
 * kernel that keeps only the windows the next level reads in LDS,
 * concurrently with the general kernel on the other tiles; 0 runs every tile
 * on the general kernel (fewer, better balanced workgroups for batches of
 * small domains); 2 runs, for three steps, both kinds of tile in one launch,
 * in the tile table's spatial order, each on its path (neighbouring tiles
 * then share their halo reads; two steps take 2 as 1).  Two steps: identical
 * results; three steps: identical with collisions off, equal to rounding with
 * them on (the kernels contract the same arithmetic differently).  EINVAL
 * otherwise. */
int lbm13_set_interior_kernel(lbm13_ctx *ctx, int on);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): advance one
 * nx x ny domain by n >= 0 steps without a context or workspace.  f_in: device
 * array [13][ny][nx] of the absolute FP64 post-collision populations f*(t), as
 * lbm13_get_state writes them; f_out (device, same layout, may equal f_in)
 * receives f*(t + n).  p, sides: as lbm13_set_params (host memory, read during
 * the call).  The result is bit-identical to lbm13_create + lbm13_set_params
 * + lbm13_set_state(f_in) + lbm13_step(n) + lbm13_get_state(f_out) with the
 * default tiles, three steps per launch and the interior-tile kernel off (the
 * same kernels).  Every other buffer (working-precision populations, tile
 * tables, parameter block, wall side arrays) lives in one static device array
 * of LBM13_NOALLOC_SCRATCH_BYTES (64 MiB) per device, which each device that
 * runs the call holds until the process ends: the call allocates no device or
 * pinned memory, creates no stream or event, does not synchronise and enqueues
 * only kernels on `stream` (hipStream_t, NULL = the null stream), so it can be
 * captured.  The array keeps the last call's contents and is shared by every
 * call on the device: calls that overlap on one device (other streams, other
 * threads) race and must be serialised by the caller.  Errors (the message in
 * lbm13_last_error(NULL)): EINVAL for NULL pointers, n < 0, bad sizes or sides,
 * or a domain whose buffers exceed the array (the limit is
 * lbm13_workspace_bytes(nx, ny, precision) <= LBM13_NOALLOC_SCRATCH_BYTES:
 * squares up to 768^2 in FP32_DEV and 556^2 in FP64), all before any device
 * work; EUNSTABLE_PARAMS as lbm13_derive; EDEVICE.  Async. */
#define LBM13_NOALLOC_SCRATCH_BYTES (64u << 20)
int lbm13_advance_noalloc(int nx, int ny, int precision, const lbm13_params *p, const lbm13_side sides[4],
                          const double *f_in, double *f_out, long long n, void *stream);

/* Destroy the context: waits for the work queued on its stream (graph
 * replays included), then frees its host objects, graphs, auxiliary streams and
 * events; never the workspace, which the caller may free once this returns. */
int lbm13_destroy(lbm13_ctx *ctx);

/* Message of the last failing call on ctx ("" if none).  With ctx NULL: the
 * message of the last failed lbm13_create / lbm13_batch_create on the calling
 * thread that got past argument checks, else a static message. */
const char *lbm13_last_error(const lbm13_ctx *ctx);

/* ------------------------------------------------------------------------ */
/* Batched form: `count` independent domains of uneven sizes, each with its own
 * parameters and sides, advanced by one launch per step over a single tile
 * table (optionally replayed as one HIP graph of k steps).  Same conventions
 * and semantics as the single-domain calls, with a domain index i. */
typedef struct lbm13_batch lbm13_batch;

size_t lbm13_batch_workspace_bytes(int count, const int *nx, const int *ny, int precision);
int lbm13_batch_create(int count, const int *nx, const int *ny, int precision, void *workspace,
                       size_t workspace_bytes, void *stream, lbm13_batch **out);
int lbm13_batch_set_params(lbm13_batch *b, int i, const lbm13_params *p, const lbm13_side sides[4],
                           lbm13_derived *derived);
int lbm13_batch_init_moments(lbm13_batch *b, int i, const double *rho, const double *ux, const double *uy,
                             const double *T);
int lbm13_batch_step(lbm13_batch *b, long long n);
int lbm13_batch_moments(lbm13_batch *b, int i, double *rho, double *ux, double *uy, double *T);
/* out[16*count]: the 16 diagnostics of lbm13_diagnostics() per domain; syncs. */
int lbm13_batch_diagnostics(lbm13_batch *b, double *out);
int lbm13_batch_get_state(lbm13_batch *b, int i, double *dst);
int lbm13_batch_set_state(lbm13_batch *b, int i, const double *src);
/* Checkpoints of domain i, as lbm13_save / lbm13_load; lbm13_batch_load keeps
 * the batch's step counter (shared by every domain). */
size_t lbm13_batch_state_bytes(const lbm13_batch *b, int i);
int lbm13_batch_save(lbm13_batch *b, int i, void *dst, size_t dst_bytes);
int lbm13_batch_load(lbm13_batch *b, int i, const void *src, size_t src_bytes);
int lbm13_batch_set_tile(lbm13_batch *b, int tile_x, int tile_y);
int lbm13_batch_autotune(lbm13_batch *b, int steps, int *tile_x, int *tile_y);
int lbm13_batch_autotune_cached(lbm13_batch *b, int steps, const char *cache_path, int *from_cache);
int lbm13_batch_use_graph(lbm13_batch *b, int k);
int lbm13_batch_set_steps_per_launch(lbm13_batch *b, int k);
int lbm13_batch_set_fused_tile(lbm13_batch *b, int tile_x, int tile_y);
int lbm13_batch_fourier(lbm13_batch *b, int i, int kx, int ky, double out[8]);
int lbm13_batch_set_interior_kernel(lbm13_batch *b, int on);
int lbm13_batch_launch_config(const lbm13_batch *b, int cfg[6]);
long long lbm13_batch_nodes(const lbm13_batch *b);
int lbm13_batch_destroy(lbm13_batch *b);
const char *lbm13_batch_last_error(const lbm13_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LBM13_H */
