// lbm13_capi.cpp -- C ABI of the D2Q13 step (declared in include/lbm13.h).
//
// Host side: derivation of the constrained coefficients (sec. 2, eqs
// d2q13-henon, d2q13-diffusion, d2q13-sigma-qx), the workspace layout, the
// tile tables, HIP graph capture and the tile autotuner.  Every step of the
// method runs in the kernels of lbm13_kernels.hip; nothing here touches
// populations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm13.h"
#include "lbm13_device.h"
#include "lbm13_tune_cache.h"

#ifndef LBM13_PLANE_PAD
#define LBM13_PLANE_PAD 256  // elements added to each velocity plane (breaks power-of-two plane strides)
#endif

namespace lbm13 {
template <typename R>
hipError_t launch_step(int, int, const R*, R*, const Dom<R>*, const Tile*, int, const Tile*, int, R*, int,
                       hipStream_t);
template <typename R>
hipError_t launch_side_fill(const R*, const Dom<R>*, const WallLine*, int, R*, int, int, hipStream_t);
template <typename R>
hipError_t launch_step2(int, int, const R*, R*, const Dom<R>*, const Tile*, int, int, R*, int, hipStream_t);
template <typename R>
hipError_t launch_diag(int, int, const R*, const Dom<R>*, int, const Tile*, int, double*, R*, int, double*,
                       hipStream_t);
template <typename R>
hipError_t launch_fourier(int, int, const R*, const Dom<R>*, int, int, const Tile*, int, int, double*, double*,
                          hipStream_t);
template <typename R>
hipError_t launch_step3(int, int, const R*, R*, const Dom<R>*, const Tile*, int, int, R*, int, bool, hipStream_t,
                        bool);
template <typename R>
hipError_t launch_init(int, int, R*, const Dom<R>*, int, const double*, const double*, const double*, const double*,
                       const double*, hipStream_t);
template <typename R>
hipError_t launch_moments(int, int, const R*, const Dom<R>*, int, double*, double*, double*, double*, hipStream_t);
template <typename R>
hipError_t launch_get_state(int, int, const R*, const Dom<R>*, int, double*, hipStream_t);
template <typename R>
hipError_t launch_set_state(int, int, R*, const Dom<R>*, int, const double*, hipStream_t);
hipError_t launch_ckpt_header(const CkptHeader&, void*, hipStream_t);
hipError_t launch_upload(const void*, size_t, void*, hipStream_t);
hipError_t noalloc_scratch(void**);
}  // namespace lbm13

using lbm13::Dom;
using lbm13::Tile;
using lbm13::WallLine;

namespace {

constexpr size_t kAlign = 256;
constexpr int kCoef = 16;  // doubles of init coefficients per domain
const int kShapes[][2] = {{64, 4}, {64, 8}, {64, 16}, {32, 8}, {32, 16}};
// fused (two steps per launch) tile shapes, as compiled in the kernels
const int kFusedShapes[][2] = {{64, 16}, {64, 12}, {64, 8}, {64, 4}, {32, 32}, {32, 16}, {32, 8}, {32, 4}};

// three steps per launch: compiled tile shapes per precision (FP64 first)
const int kStep3Shapes[2][5][2] = {{{64, 8}, {32, 16}, {32, 8}, {0, 0}, {0, 0}},
                                   {{64, 16}, {32, 32}, {64, 8}, {32, 16}, {32, 8}}};

// Width, in tiles, of the column bands the three-step tile table is ordered in
// (measured on the 4096^2 wave: 16 for every FP32 tile against 4, 8 and 32;
// 32 for FP64 against 8 and 16).
constexpr int kBandTiles[2] = {32, 16};  // FP64, FP32

bool step3_shape(int precision, int tw, int th) {
    for (auto& f : kStep3Shapes[precision == LBM13_FP64 ? 0 : 1])
        if (f[0] == tw && f[1] == th) return true;
    return false;
}

// whether the region of a two-step tile fits the LDS of one workgroup
bool fused_fits(int precision, int tw, int th) {
    const int es = precision == LBM13_FP64 ? 8 : 4;
    return 13 * (tw + 4) * (th + 4) * es + 6 * (tw + th + 8) * es <= 163840;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool valid_shape(int tx, int ty) {
    for (auto& s : kShapes)
        if (s[0] == tx && s[1] == ty) return true;
    return false;
}

struct Layout {
    size_t doms, coef, tiles_all, tiles_run, tiles_fused, tiles_fused3, part, diag, lines, wall, bufA, bufB, total;
    size_t buf_bytes;
    int tmax, tfmax;
    long long nlines_max;
    std::vector<long long> off;   // per-domain element offset of the populations
    std::vector<long long> woff;  // per-domain element offset of the wall-layer side array
    std::vector<int> pitch, plane;
};

// Deterministic workspace layout for `count` domains.
bool make_layout(int count, const int* nx, const int* ny, int precision, Layout& L) {
    if (count <= 0 || !nx || !ny || (precision != LBM13_FP64 && precision != LBM13_FP32_DEV)) return false;
    const size_t es = precision == LBM13_FP64 ? 8 : 4;
    const size_t dom_size = precision == LBM13_FP64 ? sizeof(Dom<double>) : sizeof(Dom<float>);
    L.off.resize(count);
    L.woff.resize(count);
    L.pitch.resize(count);
    L.plane.resize(count);
    long long tmax = 0, tfmax = 0, lines = 0;
    size_t elems = 0;
    for (int d = 0; d < count; ++d) {
        if (nx[d] < 2 || ny[d] < 2 || nx[d] > (1 << 16) || ny[d] > (1 << 16)) return false;
        const int pitch = (int)align_up((size_t)nx[d], 64);
        const size_t plane = align_up((size_t)pitch * ny[d], 64) + LBM13_PLANE_PAD;
        if (plane * 13 >= (size_t)INT32_MAX) return false;
        L.pitch[d] = pitch;
        L.plane[d] = (int)plane;
        L.off[d] = (long long)elems;
        elems += align_up(13 * plane, kAlign / es);
        L.woff[d] = 8 * lines;  // 2 buffers x 2 (nx + ny) lines x 4 values
        lines += 2LL * (nx[d] + ny[d]);
        long long t = 0;
        for (auto& s : kShapes)
            t = std::max(t, (long long)((nx[d] + s[0] - 1) / s[0]) * ((ny[d] + s[1] - 1) / s[1]));
        tmax += t;
        long long tf = 0;
        for (auto& f : kFusedShapes)
            tf = std::max(tf, (long long)((nx[d] + f[0] - 1) / f[0]) * ((ny[d] + f[1] - 1) / f[1]));
        tfmax += tf;
    }
    if (tmax >= INT32_MAX / 2 || tfmax >= INT32_MAX / 2) return false;
    L.tmax = (int)tmax;
    L.tfmax = (int)tfmax;
    size_t p = 0;
    L.doms = p;      p = align_up(p + dom_size * count, kAlign);
    L.coef = p;      p = align_up(p + sizeof(double) * kCoef * count, kAlign);
    L.tiles_all = p; p = align_up(p + sizeof(Tile) * tmax, kAlign);
    L.tiles_run = p; p = align_up(p + sizeof(Tile) * tmax, kAlign);
    L.tiles_fused = p; p = align_up(p + sizeof(Tile) * tfmax, kAlign);
    L.tiles_fused3 = p; p = align_up(p + sizeof(Tile) * tfmax, kAlign);
    L.part = p;      p = align_up(p + sizeof(double) * lbm13::kDiagPartials * tmax, kAlign);
    L.diag = p;      p = align_up(p + sizeof(double) * lbm13::kDiagOut * count, kAlign);
    L.nlines_max = lines;
    L.lines = p;     p = align_up(p + sizeof(WallLine) * lines, kAlign);
    L.wall = p;      p = align_up(p + es * 8 * lines, kAlign);
    L.buf_bytes = elems * es;
    L.bufA = p;      p = align_up(p + L.buf_bytes, kAlign);
    L.bufB = p;      p = align_up(p + L.buf_bytes, kAlign);
    L.total = p;
    return true;
}

// Constraints of sec. 2: eqs (d2q13-henon), (d2q13-diffusion), (d2q13-sigma-qx).
// Transport coefficients: cs2 from the first-order system (d2q13-equiv-edp-ordre-1),
// nu = sigma_XX (13 c1 + 95 + 2 E0)/104 from the second-order expansion of the XY
// moment, kappa = nu / Pr, B = (39 + 13 c1 + 2 E0)/2 the equilibrium E flux per
// unit momentum, kappa_E = kappa (28 + B)/28.
int derive(const lbm13_params* p, lbm13_derived* d) {
    const double c1 = p->c1, E0 = p->E0, k2 = p->k2, ceE = p->c_epsE;
    const double A = 13.0 * c1 + 95.0 + 2.0 * E0;
    const double Y = 114404.0 + 51051.0 * c1 - 11492.0 * ceE + 7854.0 * E0;
    d->A = A;
    d->Y = Y;
    d->sigma_XX = 1.0 / p->s_XX - 0.5;
    d->h1 = 17.0 / 26.0 - 0.5 * c1 - E0 / 13.0;
    d->k1 = 2.0 / 13.0;
    d->h2 = -(19.5 + 6.5 * c1 + E0) * k2 - (7.0 / 624.0) * A * (874481.0 + 459459.0 * c1 - 103428.0 * ceE + 70686.0 * E0) / Y;
    d->sigma_q = -654.5 * d->sigma_XX * A / Y;
    d->s_q = 1.0 / (d->sigma_q + 0.5);
    d->c_eps_rho = 140.0 + 28.0 * ceE + A * Y / (22984.0 * p->Pr);
    d->c2 = -65.0 / 24.0 - 2.625 * (c1 + d->h1 + d->k1 * E0) - k2 * E0 - d->h2;
    d->nu = d->sigma_XX * A / 104.0;
    d->kappa = d->nu / p->Pr;
    d->cs2 = A / 52.0;
    d->B = 0.5 * (39.0 + 13.0 * c1 + 2.0 * E0);
    d->kappa_E = d->kappa * (28.0 + d->B) / 28.0;
    const double rates[6] = {p->s_XX, p->s_rx, p->s_eps, p->s_varpi, p->s_XXe, d->s_q};
    for (double r : rates)
        if (!(r > 0.0 && r < 2.0)) return LBM13_EUNSTABLE_PARAMS;
    if (!(p->Pr > 0.0) || !(Y != 0.0) || !std::isfinite(d->c_eps_rho) || !std::isfinite(d->h2))
        return LBM13_EUNSTABLE_PARAMS;
    // A = 13 c1 + 95 + 2 E0 <= 0 makes cs2 = A/52 and nu = sigma_XX A/104 non-positive: no
    // sound and no viscosity, whatever the rates.
    if (!(A > 0.0) || !(d->nu > 0.0) || !(d->cs2 > 0.0)) return LBM13_EUNSTABLE_PARAMS;
    return LBM13_OK;
}

// Rest populations f^eq(1, 0, E0) by |v|^2 class (0, 1, 2, 4): the inverse of
// the orthogonal basis applied to (rho, E, eps, varpi) = (1, E0, eps_eq, varpi_eq).
void rest_populations(const lbm13_params* p, const lbm13_derived* d, double out[4]) {
    const double eps = d->c_eps_rho + p->c_epsE * p->E0;
    const double vp = p->c_varpi_rho + p->c_varpi_E * p->E0;
    const double ME[4] = {-28, -15, -2, 24}, Me[4] = {140, -2, -67, 34}, Mv[4] = {-12, 8, -6, 1};
    for (int c = 0; c < 4; ++c)
        out[c] = 1.0 / 13.0 + ME[c] * p->E0 / 4004.0 + Me[c] * eps / 42196.0 + Mv[c] * vp / 548.0;
}

}  // namespace

struct lbm13_batch {
    int count = 0, precision = 0;
    std::vector<int> nx, ny;
    Layout L;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    // two-step launches run the edge-tile kernel on `aux`, forked from and
    // joined back to the launch stream, concurrently with the interior kernel
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::vector<unsigned char> dom_host;  // staging of the Dom array
    std::vector<double> coef_host;
    std::vector<int> sides_kind;          // 4 per domain
    std::vector<char> has_params, has_state;
    std::vector<Tile> all, run, fused, fused3;
    bool step3_ok = false;                // three-step launches possible (see rebuild)
    std::vector<WallLine> lines;
    int spl = 1;                          // time steps per launch (1, 2 or 3)
    int ftw = 64, fth = 12;               // fused tile shape
    int nbulk = 0, nedge = 0;
    int nfint = 0, nfedge = 0;            // interior / edge tiles of the fused table
    int n3int = 0, n3edge = 0;            // interior / edge tiles of the three-step table
    bool sourced = true;                  // some domain has a body force or an energy source
    int split = 1;                        // 1: interior tiles run the compact-LDS kernel beside; 2: in one launch (three steps)
    int tile_x = 64, tile_y = 8;
    int cur = 0;                          // buffer holding the current state
    char* bufp[2] = {nullptr, nullptr};   // the two population buffers
    bool noalloc = false;                 // workspace is the static scratch: uploads by kernel arguments, no syncs
    long long steps = 0;
    int graph_k = 0;
    int graph_flip = 0;                   // 1 when a captured graph has an odd number of launches
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    std::string err;
};

struct lbm13_ctx {
    lbm13_batch* b = nullptr;
};

// Message of the last failed create on this thread (no context exists to hold it).
static thread_local std::string g_create_err;

namespace {

int fail(lbm13_batch* b, int code, const std::string& msg) {
    if (b) b->err = msg;
    return code;
}

int hip_fail(lbm13_batch* b, hipError_t e, const char* where) {
    return fail(b, LBM13_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

size_t dom_size(const lbm13_batch* b) {
    return b->precision == LBM13_FP64 ? sizeof(Dom<double>) : sizeof(Dom<float>);
}

template <typename R>
Dom<R>* dom_host(lbm13_batch* b, int d) {
    return reinterpret_cast<Dom<R>*>(b->dom_host.data()) + d;
}

template <typename R>
R* buf(lbm13_batch* b, int which) {
    return reinterpret_cast<R*>(b->bufp[which]);
}

// Host data to the workspace at byte offset `off`: an async copy (the host
// data must live until it runs: the callers keep it in the batch and
// synchronise), or, for the allocation-free path, kernel launches that carry
// the data as arguments (nothing to keep, capture-safe).
hipError_t upload(lbm13_batch* b, size_t off, const void* host, size_t bytes) {
    if (bytes == 0) return hipSuccess;
    if (b->noalloc) return lbm13::launch_upload(host, bytes, b->ws + off, b->stream);
    return hipMemcpyAsync(b->ws + off, host, bytes, hipMemcpyHostToDevice, b->stream);
}

template <typename R>
const Dom<R>* doms_dev(lbm13_batch* b) {
    return reinterpret_cast<const Dom<R>*>(b->ws + b->L.doms);
}

void drop_graphs(lbm13_batch* b) {
    for (int p = 0; p < 2; ++p) {
        if (b->gexec[p]) (void)hipGraphExecDestroy(b->gexec[p]);
        if (b->graph[p]) (void)hipGraphDestroy(b->graph[p]);
        b->gexec[p] = nullptr;
        b->graph[p] = nullptr;
    }
}

bool near_wall_tile(const lbm13_batch* b, int d, int x0, int y0) {
    const int* k = &b->sides_kind[4 * d];
    const int x1 = std::min(x0 + b->tile_x, b->nx[d]) - 1, y1 = std::min(y0 + b->tile_y, b->ny[d]) - 1;
    if (k[0] != LBM13_PERIODIC && (x0 < 2 || x1 >= b->nx[d] - 2)) return true;
    if (k[2] != LBM13_PERIODIC && (y0 < 2 || y1 >= b->ny[d] - 2)) return true;
    return false;
}

template <typename R>
void set_tile_ranges(lbm13_batch* b) {
    for (int d = 0; d < b->count; ++d) {
        dom_host<R>(b, d)->tile0 = 0;
        dom_host<R>(b, d)->ntiles = 0;
    }
    int t = 0;
    for (int d = 0; d < b->count; ++d) {
        dom_host<R>(b, d)->tile0 = t;
        const int n = ((b->nx[d] + b->tile_x - 1) / b->tile_x) * ((b->ny[d] + b->tile_y - 1) / b->tile_y);
        dom_host<R>(b, d)->ntiles = n;
        t += n;
    }
}

// Whether some domain with parameters has a body force or an energy source
// (the three-step window kernel drops those terms otherwise).
template <typename R>
bool any_sources(lbm13_batch* b) {
    for (int d = 0; d < b->count; ++d) {
        if (!b->has_params[d]) continue;
        const Dom<R>* D = dom_host<R>(b, d);
        if (D->F0x_d != 0.0 || D->F0y_d != 0.0 || D->gx_d != 0.0 || D->gy_d != 0.0 || D->QE_d != 0.0) return true;
    }
    return false;
}

// Rebuild the tile tables for the current tile shape and sides; uploads the
// tables and the Dom array and synchronises (not a hot path).
int rebuild(lbm13_batch* b) {
    b->all.clear();
    std::vector<Tile> bulk, edge;
    for (int d = 0; d < b->count; ++d)
        for (int y0 = 0; y0 < b->ny[d]; y0 += b->tile_y)
            for (int x0 = 0; x0 < b->nx[d]; x0 += b->tile_x) {
                const bool e = near_wall_tile(b, d, x0, y0);
                Tile t{d, x0, y0, e ? 1 : 0};
                b->all.push_back(t);
                (e ? edge : bulk).push_back(t);
            }
    if ((int)b->all.size() > b->L.tmax) return fail(b, LBM13_EINVAL, "tile table overflow");
    b->run = bulk;
    b->run.insert(b->run.end(), edge.begin(), edge.end());
    b->fused.clear();
    std::vector<Tile> fedge;
    const long long es = b->precision == LBM13_FP64 ? 8 : 4;
    for (int d = 0; d < b->count; ++d) {
        // interior tiles address the 13 planes with 32-bit byte offsets
        const bool small = (13LL * b->L.plane[d] + 2LL * b->L.pitch[d] + 2) * es <= (long long)INT32_MAX;
        for (int y0 = 0; y0 < b->ny[d]; y0 += b->fth)
            for (int x0 = 0; x0 < b->nx[d]; x0 += b->ftw) {
                // flag 2: interior tile (region plus its gather reach inside the
                // domain and at least two nodes from every wall, no wrap); with the
                // interior kernel off it runs the general kernel's fast path
                const bool in = small && x0 >= 4 && x0 + b->ftw + 4 <= b->nx[d] && y0 >= 4 &&
                                y0 + b->fth + 4 <= b->ny[d];
                if (in && b->split) b->fused.push_back(Tile{d, x0, y0, 2});
                else fedge.push_back(Tile{d, x0, y0, in ? 2 : 0});
            }
    }
    b->nfint = (int)b->fused.size();
    b->nfedge = (int)fedge.size();
    b->fused.insert(b->fused.end(), fedge.begin(), fedge.end());
    if ((int)b->fused.size() > b->L.tfmax) return fail(b, LBM13_EINVAL, "fused tile table overflow");
    // Three steps per launch (a three-step tile shape).  Interior tiles run
    // step3_kernel: whole tiles whose region and its reach (six nodes around the
    // tile) stay at least two nodes from every wall, on a periodic axis a side
    // of at least the tile + 12 (the region and its reach wrap at most once),
    // planes within 32-bit byte offsets; flag 2, plus 4 where the region wraps.
    // The other tiles, and every tile with the interior kernel off, run
    // step3_wall_kernel.
    b->fused3.clear();
    b->step3_ok = step3_shape(b->precision, b->ftw, b->fth);
    std::vector<Tile> f3edge;
    for (int d = 0; d < b->count && b->step3_ok; ++d) {
        const int* k = &b->sides_kind[4 * d];
        const int nx = b->nx[d], ny = b->ny[d], tw = b->ftw, th = b->fth;
        const bool small = (13LL * b->L.plane[d] + 2LL * b->L.pitch[d] + 2) * es <= (long long)INT32_MAX;
        // column bands of kBandTiles tiles: the XCDs take contiguous runs of the
        // table, so a run covers few columns and many rows, and the halo rows a
        // tile shares with the tiles above and below are read while still in L2
        const int bw = tw * kBandTiles[b->precision == LBM13_FP64 ? 0 : 1];
        for (int bx = 0; bx < nx; bx += bw)
            for (int y0 = 0; y0 < ny; y0 += th)
                for (int x0 = bx; x0 < std::min(nx, bx + bw); x0 += tw) {
                    const bool xin = x0 >= 6 && x0 + tw + 6 <= nx, yin = y0 >= 6 && y0 + th + 6 <= ny;
                    const bool xok = x0 + tw <= nx && (k[0] == LBM13_PERIODIC ? nx >= tw + 12 : xin);
                    const bool yok = y0 + th <= ny && (k[2] == LBM13_PERIODIC ? ny >= th + 12 : yin);
                    const bool interior = b->split && small && xok && yok;
                    const Tile tl{d, x0, y0, interior ? (xin && yin ? 2 : 2 | 4) : 0};
                    if (interior || b->split == 2)  // with one launch the table keeps the spatial order
                        b->fused3.push_back(tl);
                    else
                        f3edge.push_back(tl);
                }
    }
    if (b->split == 2) {  // every tile in fused3, in order; n3int counts the interior ones
        int nin = 0;
        for (const Tile& tl : b->fused3) nin += (tl.flags & 2) ? 1 : 0;
        b->n3int = nin;
        b->n3edge = (int)b->fused3.size() - nin;
    } else {
        b->n3int = (int)b->fused3.size();
        b->n3edge = (int)f3edge.size();
        b->fused3.insert(b->fused3.end(), f3edge.begin(), f3edge.end());
    }
    if ((int)b->fused3.size() > b->L.tfmax) return fail(b, LBM13_EINVAL, "three-step tile table overflow");
    b->lines.clear();
    for (int d = 0; d < b->count; ++d) {
        const int* k = &b->sides_kind[4 * d];
        const int nx = b->nx[d], ny = b->ny[d];
        if (k[0] != LBM13_PERIODIC)
            for (int y = 0; y < ny; ++y) {
                b->lines.push_back(WallLine{d, 0, y, y});
                b->lines.push_back(WallLine{d, 1, y, ny + y});
            }
        if (k[2] != LBM13_PERIODIC)
            for (int x = 0; x < nx; ++x) {
                b->lines.push_back(WallLine{d, 2, x, 2 * ny + x});
                b->lines.push_back(WallLine{d, 3, x, 2 * ny + nx + x});
            }
    }
    if ((long long)b->lines.size() > b->L.nlines_max) return fail(b, LBM13_EINVAL, "wall line table overflow");
    b->nbulk = (int)bulk.size();
    b->nedge = (int)edge.size();
    b->sourced = b->precision == LBM13_FP64 ? any_sources<double>(b) : any_sources<float>(b);
    if (b->precision == LBM13_FP64) set_tile_ranges<double>(b);
    else set_tile_ranges<float>(b);
    hipError_t e;
    e = upload(b, b->L.tiles_all, b->all.data(), sizeof(Tile) * b->all.size());
    if (e != hipSuccess) return hip_fail(b, e, "upload tile table");
    e = upload(b, b->L.tiles_run, b->run.data(), sizeof(Tile) * b->run.size());
    if (e != hipSuccess) return hip_fail(b, e, "upload tile table");
    e = upload(b, b->L.tiles_fused, b->fused.data(), sizeof(Tile) * b->fused.size());
    if (e != hipSuccess) return hip_fail(b, e, "upload fused tile table");
    e = upload(b, b->L.tiles_fused3, b->fused3.data(), sizeof(Tile) * b->fused3.size());
    if (e != hipSuccess) return hip_fail(b, e, "upload three-step tile table");
    e = upload(b, b->L.lines, b->lines.data(), sizeof(WallLine) * b->lines.size());
    if (e != hipSuccess) return hip_fail(b, e, "upload wall lines");
    e = upload(b, b->L.doms, b->dom_host.data(), b->dom_host.size());
    if (e != hipSuccess) return hip_fail(b, e, "upload domain table");
    if (!b->noalloc) {  // the async copies read the host tables: keep them until done
        e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return hip_fail(b, e, "synchronise");
    }
    drop_graphs(b);
    return LBM13_OK;
}

template <typename R>
void fill_dom(lbm13_batch* b, int d, const lbm13_params* p, const lbm13_side* sides, const lbm13_derived* dv) {
    Dom<R>* D = dom_host<R>(b, d);
    const int tile0 = D->tile0, ntiles = D->ntiles;
    std::memset(D, 0, sizeof(Dom<R>));
    D->tile0 = tile0;
    D->ntiles = ntiles;
    D->off = b->L.off[d];
    D->woff = b->L.woff[d];
    D->plane = b->L.plane[d];
    D->pitch = b->L.pitch[d];
    D->nx = b->nx[d];
    D->ny = b->ny[d];
    D->xper = sides[0].kind == LBM13_PERIODIC;
    D->yper = sides[2].kind == LBM13_PERIODIC;
    for (int w = 0; w < 4; ++w) D->kind[w] = sides[w].kind;
    D->collide = p->collide ? 1 : 0;
    const double a1 = p->c1 + dv->h1 + dv->k1 * p->E0;
    const double a2 = dv->c2 + dv->h2 + p->k2 * p->E0;
    D->c_er = R(dv->c_eps_rho);
    D->c_eE = R(p->c_epsE);
    D->c_vr = R(p->c_varpi_rho);
    D->c_vE = R(p->c_varpi_E);
    D->a1 = R(a1);
    D->h1 = R(dv->h1);
    D->k1 = R(dv->k1);
    D->a2 = R(a2);
    D->h2 = R(dv->h2);
    D->k2 = R(p->k2);
    const double F0x = p->F0[0] + p->g[0] * (1.0 - p->rho0), F0y = p->F0[1] + p->g[1] * (1.0 - p->rho0);
    D->F0x_d = F0x;
    D->F0y_d = F0y;
    D->gx_d = p->g[0];
    D->gy_d = p->g[1];
    const double ke = p->s_eps / 42196.0, kv = p->s_varpi / 548.0;
    {
        // rows of M over the classes (rest, |v|^2 = 1, 2, 4) for E, eps, varpi
        // (the rho row is 1 on every class)
        const double Er[4] = {-28, -15, -2, 24}, er[4] = {140, -2, -67, 34}, vr[4] = {-12, 8, -6, 1};
        for (int j = 0; j < 4; ++j) {
            D->aeps[j] = R(ke * (er[j] - dv->c_eps_rho - p->c_epsE * Er[j]));
            D->avp[j] = R(kv * (vr[j] - p->c_varpi_rho - p->c_varpi_E * Er[j]));
            D->eQ[j] = R(-Er[j] * p->Q_E / 4004.0);
        }
    }
    D->kX = R(p->s_XX / 68.0);
    D->kY = R(p->s_XX / 4.0);
    D->kXe = R(p->s_XXe / 68.0);
    D->kq = R(dv->s_q / 20.0);
    D->kr = R(p->s_rx / 70.0);
    {
        // update patterns of an axis' odd populations from the relaxations
        // kq (q - q^eq) and kr (r - r^eq): speed-1 -2, 4; speed-2 2, 1;
        // diagonal -1, -3 (rows of M^T D^-1 over q and r)
        const double kq = dv->s_q / 20.0, kr = p->s_rx / 70.0;
        const double w[6] = {-2.0 * kq, 4.0 * kr, 2.0 * kq, kr, -kq, -3.0 * kr};
        for (int k = 0; k < 6; ++k) D->ow[k] = R(w[k]);
    }
    D->fjx = R(-F0x / 14.0);
    D->fjy = R(-F0y / 14.0);
    D->gjx = R(-p->g[0] / 14.0);
    D->gjy = R(-p->g[1] / 14.0);
    D->QE = R(p->Q_E);
    D->QE_d = p->Q_E;
    for (int w = 0; w < 4; ++w) {
        const double u = sides[w].u_tangential;
        D->wall_u[w] = R(u);
        D->wall_dE[w] = R(sides[w].kind == LBM13_WALL_DIRICHLET_T ? sides[w].T_wall + 6.5 * u * u - p->E0 : 0.0);
    }
    D->E0 = p->E0;
    rest_populations(p, dv, D->frest);
    D->B = dv->B;
    const double dT = sides[0].T_wall - sides[1].T_wall;
    D->nu_scale = dT != 0.0 ? (double)b->nx[d] / (dv->kappa_E * dT) : 0.0;
    double* c = &b->coef_host[(size_t)kCoef * d];
    const double cc[10] = {dv->c_eps_rho, p->c_epsE, p->c_varpi_rho, p->c_varpi_E, a1, dv->h1, dv->k1,
                           a2, dv->h2, p->k2};
    for (int k = 0; k < 10; ++k) c[k] = cc[k];
}

bool check_index(lbm13_batch* b, int i) { return b && i >= 0 && i < b->count; }

template <typename R>
hipError_t launch_one_step(lbm13_batch* b, int from, hipStream_t s) {
    const Tile* run = reinterpret_cast<const Tile*>(b->ws + b->L.tiles_run);
    R* side = reinterpret_cast<R*>(b->ws + b->L.wall);
    return lbm13::launch_step<R>(b->tile_x, b->tile_y, buf<R>(b, from), buf<R>(b, 1 - from), doms_dev<R>(b), run,
                                 b->nbulk, run + b->nbulk, b->nedge, side, from, s);
}

// Streams and events of the concurrent two-step launch (created once, at the
// first two-step launch or capture, never while a capture is open).
hipError_t ensure_aux(lbm13_batch* b) {
    hipError_t e = hipSuccess;
    if (!b->aux) e = hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking);
    if (e == hipSuccess && !b->ev_fork) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess && !b->ev_join) e = hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming);
    return e;
}

// Two time steps: the interior tiles on stream s and, concurrently, the edge
// tiles on the auxiliary stream (fork and join through events, which a graph
// capture records as two parallel branches).  Both kernels read the same
// state and write disjoint nodes; only edge tiles write wall-layer values.
template <typename R>
hipError_t launch_two_steps(lbm13_batch* b, int from, hipStream_t s) {
    const Tile* tiles = reinterpret_cast<const Tile*>(b->ws + b->L.tiles_fused);
    R* side = reinterpret_cast<R*>(b->ws + b->L.wall);
    const R* src = buf<R>(b, from);
    R* dst = buf<R>(b, 1 - from);
    if (b->nfint == 0 || b->nfedge == 0 || !b->aux)
        return lbm13::launch_step2<R>(b->ftw, b->fth, src, dst, doms_dev<R>(b), tiles, b->nfint, b->nfedge, side,
                                      from, s);
    hipError_t e = hipEventRecord(b->ev_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->aux, b->ev_fork, 0);
    if (e == hipSuccess)
        e = lbm13::launch_step2<R>(b->ftw, b->fth, src, dst, doms_dev<R>(b), tiles + b->nfint, 0, b->nfedge, side,
                                   from, b->aux);
    if (e == hipSuccess) e = hipEventRecord(b->ev_join, b->aux);
    if (e == hipSuccess)
        e = lbm13::launch_step2<R>(b->ftw, b->fth, src, dst, doms_dev<R>(b), tiles, b->nfint, 0, side, from, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, b->ev_join, 0);
    return e;
}

// Three time steps: interior tiles on stream s and the other tiles concurrently
// on the auxiliary stream, as for two steps.
template <typename R>
hipError_t launch_three_steps(lbm13_batch* b, int from, hipStream_t s) {
    const Tile* tiles = reinterpret_cast<const Tile*>(b->ws + b->L.tiles_fused3);
    R* side = reinterpret_cast<R*>(b->ws + b->L.wall);
    const R* src = buf<R>(b, from);
    R* dst = buf<R>(b, 1 - from);
    if (b->split == 2 && b->n3int > 0 && b->n3edge > 0)  // both kinds of tile, in order, in one launch
        return lbm13::launch_step3<R>(b->ftw, b->fth, src, dst, doms_dev<R>(b), tiles, b->n3int, b->n3edge, side,
                                      from, b->sourced, s, true);
    if (b->split == 2)  // one kind only: its own kernel (the table holds just those tiles)
        return lbm13::launch_step3<R>(b->ftw, b->fth, src, dst, doms_dev<R>(b), tiles, b->n3int, b->n3edge, side,
                                      from, b->sourced, s, false);
    if (b->n3int == 0 || b->n3edge == 0 || !b->aux)
        return lbm13::launch_step3<R>(b->ftw, b->fth, src, dst, doms_dev<R>(b), tiles, b->n3int, b->n3edge, side,
                                      from, b->sourced, s, false);
    hipError_t e = hipEventRecord(b->ev_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->aux, b->ev_fork, 0);
    if (e == hipSuccess)
        e = lbm13::launch_step3<R>(b->ftw, b->fth, src, dst, doms_dev<R>(b), tiles + b->n3int, 0, b->n3edge, side,
                                   from, b->sourced, b->aux, false);
    if (e == hipSuccess) e = hipEventRecord(b->ev_join, b->aux);
    if (e == hipSuccess)
        e = lbm13::launch_step3<R>(b->ftw, b->fth, src, dst, doms_dev<R>(b), tiles, b->n3int, 0, side, from,
                                   b->sourced, s, false);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, b->ev_join, 0);
    return e;
}

// Enqueue n steps as launches of spl steps (then 2 and 1 for the remainder),
// swapping the buffers once per launch; `launches` counts them.
template <typename R>
hipError_t enqueue_steps(lbm13_batch* b, long long n, int& from, hipStream_t s, long long& launches) {
    while (n > 0) {
        const int k = (b->spl == 3 && n >= 3) ? 3 : (b->spl >= 2 && n >= 2) ? 2 : 1;
        const hipError_t e = k == 3 ? launch_three_steps<R>(b, from, s)
                             : k == 2 ? launch_two_steps<R>(b, from, s)
                                      : launch_one_step<R>(b, from, s);
        if (e != hipSuccess) return e;
        from = 1 - from;
        n -= k;
        ++launches;
    }
    return hipSuccess;
}

// Wall-layer side values of the kept state (after init, set_state, load).
template <typename R>
hipError_t fill_side(lbm13_batch* b, int only_dom) {
    const WallLine* lines = reinterpret_cast<const WallLine*>(b->ws + b->L.lines);
    R* side = reinterpret_cast<R*>(b->ws + b->L.wall);
    return lbm13::launch_side_fill<R>(buf<R>(b, b->cur), doms_dev<R>(b), lines, (int)b->lines.size(), side, b->cur,
                                      only_dom, b->stream);
}

// only_dom = -1: every domain.
hipError_t fill_side_any(lbm13_batch* b, int only_dom) {
    return b->precision == LBM13_FP64 ? fill_side<double>(b, only_dom) : fill_side<float>(b, only_dom);
}

template <typename R>
int capture_graph(lbm13_batch* b, int parity) {
    hipError_t e;
    if (!b->capture_stream) {
        e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(b, e, "create capture stream");
    }
    if (b->spl >= 2 && (e = ensure_aux(b)) != hipSuccess) return hip_fail(b, e, "create auxiliary stream");
    e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(b, e, "begin capture");
    int from = parity;
    long long launches = 0;
    const hipError_t le = enqueue_steps<R>(b, b->graph_k, from, b->capture_stream, launches);
    b->graph_flip = (int)(launches & 1);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->capture_stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(b, le, "launch during capture");
    }
    if (e != hipSuccess) return hip_fail(b, e, "end capture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(b, e, "instantiate graph");
    }
    b->graph[parity] = g;
    b->gexec[parity] = x;
    return LBM13_OK;
}

template <typename R>
int step_impl(lbm13_batch* b, long long n) {
    if (b->spl == 3 && !b->step3_ok)
        return fail(b, LBM13_EINVAL, "three steps per launch need a three-step tile shape (FP32: 64x16, 32x32, "
                                     "64x8, 32x16, 32x8; FP64: 64x8, 32x16, 32x8)");
    while (b->graph_k > 0 && n >= b->graph_k) {
        if (!b->gexec[b->cur]) {
            int st = capture_graph<R>(b, b->cur);
            if (st) return st;
        }
        hipError_t e = hipGraphLaunch(b->gexec[b->cur], b->stream);
        if (e != hipSuccess) return hip_fail(b, e, "graph launch");
        // each launch in the graph swaps the buffers once
        if (b->graph_flip) b->cur = 1 - b->cur;
        n -= b->graph_k;
        b->steps += b->graph_k;
    }
    if (b->spl >= 2 && n >= 2 && b->split) {  // with the interior kernel off every launch is one kernel
        hipError_t e = ensure_aux(b);
        if (e != hipSuccess) return hip_fail(b, e, "create auxiliary stream");
    }
    int from = b->cur;
    long long launches = 0;
    const hipError_t e = enqueue_steps<R>(b, n, from, b->stream, launches);
    if (e != hipSuccess) return hip_fail(b, e, "step launch");
    b->cur = from;
    b->steps += n;
    return LBM13_OK;
}

int ready(lbm13_batch* b) {
    if (!b) return LBM13_EINVAL;
    for (int d = 0; d < b->count; ++d) {
        if (!b->has_params[d]) return fail(b, LBM13_ESTATE, "domain " + std::to_string(d) + " has no parameters");
        if (!b->has_state[d]) return fail(b, LBM13_ESTATE, "domain " + std::to_string(d) + " has no initial state");
    }
    return LBM13_OK;
}

template <typename R>
int autotune_impl(lbm13_batch* b, int steps, int* tx, int* ty) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(b, LBM13_EDEVICE, "event create");
    const int keep_k = b->graph_k;
    b->graph_k = 0;
    steps = (steps + 5) / 6 * 6;  // a multiple of 6 keeps two- and three-step launches whole
    struct Cand {
        int spl, w, h, split;
    };
    std::vector<Cand> cands;
    for (auto& s : kShapes) cands.push_back(Cand{1, s[0], s[1], b->split});
    for (auto& f : kFusedShapes)
        if (fused_fits(b->precision, f[0], f[1]))
            for (int sp = 1; sp >= 0; --sp) cands.push_back(Cand{2, f[0], f[1], sp});
    for (auto& f : kStep3Shapes[b->precision == LBM13_FP64 ? 0 : 1])
        if (f[0] > 0)
            for (int sp = 2; sp >= 0; --sp) cands.push_back(Cand{3, f[0], f[1], sp});
    float best = 1e30f;
    Cand pick{b->spl, b->spl >= 2 ? b->ftw : b->tile_x, b->spl >= 2 ? b->fth : b->tile_y, b->split};
    int st = LBM13_OK;
    for (const Cand& c : cands) {
        b->spl = c.spl;
        b->split = c.split;
        if (c.spl == 1) {
            b->tile_x = c.w;
            b->tile_y = c.h;
        } else {
            b->ftw = c.w;
            b->fth = c.h;
        }
        if ((st = rebuild(b))) break;
        if (c.spl == 3 && !b->step3_ok) continue;  // not a three-step shape
        if (c.spl == 3 && c.split == 2 && (b->n3int == 0 || b->n3edge == 0)) continue;  // the same launch as 1
        if ((st = step_impl<R>(b, 6))) break;
        (void)hipEventRecord(e0, b->stream);
        if ((st = step_impl<R>(b, steps))) break;
        (void)hipEventRecord(e1, b->stream);
        if (hipEventSynchronize(e1) != hipSuccess) {
            st = fail(b, LBM13_EDEVICE, "event sync");
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
            best = ms;
            pick = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->spl = pick.spl;
    b->split = pick.split;
    if (pick.spl == 1) {
        b->tile_x = pick.w;
        b->tile_y = pick.h;
    } else {
        b->ftw = pick.w;
        b->fth = pick.h;
    }
    int st2 = rebuild(b);
    b->graph_k = keep_k;
    if (st) return st;
    if (st2) return st2;
    if (tx) *tx = pick.w;
    if (ty) *ty = pick.h;
    return LBM13_OK;
}

}  // namespace

// =========================================================================== batch API

namespace {

// The allocation-free step: a batch of one domain whose workspace is the
// static device scratch (tables uploaded as kernel arguments, no
// synchronisation), state in from f_in, n steps of the context path with
// three steps per launch and the interior kernel off, state out to f_out.
template <typename R>
int advance_noalloc_impl(lbm13_batch& b, const lbm13_params* p, const lbm13_side sides[4],
                                const lbm13_derived& dv, const double* f_in, double* f_out, long long n) {
    fill_dom<R>(&b, 0, p, sides, &dv);
    b.has_params[0] = 1;
    int st = rebuild(&b);
    if (st) return st;
    hipError_t e = lbm13::launch_set_state<R>(b.nx[0], b.ny[0], buf<R>(&b, b.cur), doms_dev<R>(&b), 0, f_in, b.stream);
    if (e != hipSuccess) return hip_fail(&b, e, "set_state launch");
    e = fill_side<R>(&b, 0);
    if (e != hipSuccess) return hip_fail(&b, e, "side fill launch");
    b.has_state[0] = 1;
    st = step_impl<R>(&b, n);
    if (st) return st;
    e = lbm13::launch_get_state<R>(b.nx[0], b.ny[0], buf<R>(&b, b.cur), doms_dev<R>(&b), 0, f_out, b.stream);
    if (e != hipSuccess) return hip_fail(&b, e, "get_state launch");
    return LBM13_OK;
}

int noalloc_fail(int code, const std::string& msg) {
    g_create_err = "lbm13_advance_noalloc: " + msg;
    return code;
}

}  // namespace

extern "C" {

int lbm13_derive(const lbm13_params* p, lbm13_derived* out) {
    if (!p || !out) return LBM13_EINVAL;
    return derive(p, out);
}

size_t lbm13_batch_workspace_bytes(int count, const int* nx, const int* ny, int precision) {
    Layout L;
    if (!make_layout(count, nx, ny, precision, L)) return 0;
    return L.total;
}

int lbm13_batch_create(int count, const int* nx, const int* ny, int precision, void* workspace,
                       size_t workspace_bytes, void* stream, lbm13_batch** out) {
    if (!out) return LBM13_EINVAL;
    *out = nullptr;
    Layout L;
    if (!make_layout(count, nx, ny, precision, L) || !workspace) return LBM13_EINVAL;
    if (workspace_bytes < L.total) return LBM13_ENOMEM;
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return LBM13_EINVAL;
    lbm13_batch* b = new (std::nothrow) lbm13_batch;
    if (!b) return LBM13_ENOMEM;
    b->count = count;
    b->precision = precision;
    b->nx.assign(nx, nx + count);
    b->ny.assign(ny, ny + count);
    b->L = L;
    b->ws = static_cast<char*>(workspace);
    b->bufp[0] = b->ws + L.bufA;
    b->bufp[1] = b->ws + L.bufB;
    b->stream = static_cast<hipStream_t>(stream);
    b->dom_host.assign(dom_size(b) * count, 0);
    b->coef_host.assign((size_t)kCoef * count, 0.0);
    b->sides_kind.assign(4 * count, LBM13_PERIODIC);
    b->has_params.assign(count, 0);
    b->has_state.assign(count, 0);
    b->ftw = precision == LBM13_FP64 ? lbm13::Fused<double>::TW : lbm13::Fused<float>::TW;
    b->fth = precision == LBM13_FP64 ? lbm13::Fused<double>::TH : lbm13::Fused<float>::TH;
    int st = rebuild(b);
    if (st) {
        g_create_err = b->err;
        delete b;
        return st;
    }
    *out = b;
    return LBM13_OK;
}

int lbm13_batch_set_params(lbm13_batch* b, int i, const lbm13_params* p, const lbm13_side sides[4],
                           lbm13_derived* derived) {
    if (!check_index(b, i) || !p || !sides) return b ? fail(b, LBM13_EINVAL, "bad argument") : LBM13_EINVAL;
    for (int w = 0; w < 4; ++w)
        if (sides[w].kind < LBM13_PERIODIC || sides[w].kind > LBM13_WALL_DIRICHLET_T)
            return fail(b, LBM13_EINVAL, "unknown side kind");
    if ((sides[0].kind == LBM13_PERIODIC) != (sides[1].kind == LBM13_PERIODIC) ||
        (sides[2].kind == LBM13_PERIODIC) != (sides[3].kind == LBM13_PERIODIC))
        return fail(b, LBM13_EINVAL, "opposite sides must both be periodic or both walls");
    lbm13_derived dv;
    int st = derive(p, &dv);
    if (derived) *derived = dv;
    if (st) return fail(b, st, "relaxation rate outside (0, 2) or degenerate constants");
    for (int w = 0; w < 4; ++w) b->sides_kind[4 * i + w] = sides[w].kind;
    if (b->precision == LBM13_FP64) fill_dom<double>(b, i, p, sides, &dv);
    else fill_dom<float>(b, i, p, sides, &dv);
    hipError_t e = upload(b, b->L.coef + sizeof(double) * kCoef * i, &b->coef_host[(size_t)kCoef * i],
                          sizeof(double) * kCoef);
    if (e != hipSuccess) return hip_fail(b, e, "upload coefficients");
    b->has_params[i] = 1;
    st = rebuild(b);
    if (st) return st;
    bool any_state = false;
    for (char h : b->has_state) any_state = any_state || h;
    if (any_state) {
        e = fill_side_any(b, -1);  // walls may have changed under a kept state
        if (e != hipSuccess) return hip_fail(b, e, "side fill launch");
    }
    return LBM13_OK;
}

int lbm13_batch_init_moments(lbm13_batch* b, int i, const double* rho, const double* ux, const double* uy,
                             const double* T) {
    if (!check_index(b, i) || !rho || !ux || !uy || !T) return b ? fail(b, LBM13_EINVAL, "bad argument") : LBM13_EINVAL;
    if (!b->has_params[i]) return fail(b, LBM13_ESTATE, "set_params first");
    const double* coef = reinterpret_cast<const double*>(b->ws + b->L.coef) + (size_t)kCoef * i;
    hipError_t e;
    if (b->precision == LBM13_FP64)
        e = lbm13::launch_init<double>(b->nx[i], b->ny[i], buf<double>(b, b->cur), doms_dev<double>(b), i, rho, ux, uy,
                                       T, coef, b->stream);
    else
        e = lbm13::launch_init<float>(b->nx[i], b->ny[i], buf<float>(b, b->cur), doms_dev<float>(b), i, rho, ux, uy, T,
                                      coef, b->stream);
    if (e != hipSuccess) return hip_fail(b, e, "init launch");
    e = fill_side_any(b, i);
    if (e != hipSuccess) return hip_fail(b, e, "side fill launch");
    b->has_state[i] = 1;
    b->steps = 0;
    return LBM13_OK;
}

int lbm13_batch_step(lbm13_batch* b, long long n) {
    if (!b || n < 0) return b ? fail(b, LBM13_EINVAL, "negative step count") : LBM13_EINVAL;
    int st = ready(b);
    if (st) return st;
    return b->precision == LBM13_FP64 ? step_impl<double>(b, n) : step_impl<float>(b, n);
}

int lbm13_batch_moments(lbm13_batch* b, int i, double* rho, double* ux, double* uy, double* T) {
    if (!check_index(b, i)) return b ? fail(b, LBM13_EINVAL, "bad domain index") : LBM13_EINVAL;
    if (!b->has_state[i]) return fail(b, LBM13_ESTATE, "no state");
    hipError_t e;
    if (b->precision == LBM13_FP64)
        e = lbm13::launch_moments<double>(b->nx[i], b->ny[i], buf<double>(b, b->cur), doms_dev<double>(b), i, rho, ux,
                                          uy, T, b->stream);
    else
        e = lbm13::launch_moments<float>(b->nx[i], b->ny[i], buf<float>(b, b->cur), doms_dev<float>(b), i, rho, ux, uy,
                                         T, b->stream);
    return e == hipSuccess ? LBM13_OK : hip_fail(b, e, "moments launch");
}

int lbm13_batch_diagnostics(lbm13_batch* b, double* out) {
    if (!b || !out) return b ? fail(b, LBM13_EINVAL, "bad argument") : LBM13_EINVAL;
    int st = ready(b);
    if (st) return st;
    const Tile* all = reinterpret_cast<const Tile*>(b->ws + b->L.tiles_all);
    double* part = reinterpret_cast<double*>(b->ws + b->L.part);
    double* dout = reinterpret_cast<double*>(b->ws + b->L.diag);
    hipError_t e;
    if (b->precision == LBM13_FP64)
        e = lbm13::launch_diag<double>(b->tile_x, b->tile_y, buf<double>(b, b->cur), doms_dev<double>(b), b->count, all,
                                       (int)b->all.size(), part, reinterpret_cast<double*>(b->ws + b->L.wall),
                                       b->cur, dout, b->stream);
    else
        e = lbm13::launch_diag<float>(b->tile_x, b->tile_y, buf<float>(b, b->cur), doms_dev<float>(b), b->count, all,
                                      (int)b->all.size(), part, reinterpret_cast<float*>(b->ws + b->L.wall), b->cur,
                                      dout, b->stream);
    if (e != hipSuccess) return hip_fail(b, e, "diagnostics launch");
    e = hipMemcpyAsync(out, dout, sizeof(double) * lbm13::kDiagOut * b->count, hipMemcpyDeviceToHost, b->stream);
    if (e != hipSuccess) return hip_fail(b, e, "diagnostics copy");
    e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(b, e, "diagnostics sync");
    for (int d = 0; d < b->count; ++d)
        if (out[lbm13::kDiagOut * d + 9] > 0 || !(out[lbm13::kDiagOut * d + 10] > 0))
            return fail(b, LBM13_ENONFINITE, "non-finite population or rho <= 0 in domain " + std::to_string(d));
    return LBM13_OK;
}

int lbm13_batch_fourier(lbm13_batch* b, int i, int kx, int ky, double* out) {
    if (!check_index(b, i) || !out) return b ? fail(b, LBM13_EINVAL, "bad argument") : LBM13_EINVAL;
    if (!b->has_state[i]) return fail(b, LBM13_ESTATE, "no state");
    if (!b->has_params[i]) return fail(b, LBM13_ESTATE, "no parameters");
    const Tile* all = reinterpret_cast<const Tile*>(b->ws + b->L.tiles_all);
    double* part = reinterpret_cast<double*>(b->ws + b->L.part);
    double* dout = reinterpret_cast<double*>(b->ws + b->L.diag);  // first 8 values, transient
    const int ntiles = ((b->nx[i] + b->tile_x - 1) / b->tile_x) * ((b->ny[i] + b->tile_y - 1) / b->tile_y);
    hipError_t e;
    if (b->precision == LBM13_FP64)
        e = lbm13::launch_fourier<double>(b->tile_x, b->tile_y, buf<double>(b, b->cur), doms_dev<double>(b), i, ntiles,
                                          all, kx, ky, part, dout, b->stream);
    else
        e = lbm13::launch_fourier<float>(b->tile_x, b->tile_y, buf<float>(b, b->cur), doms_dev<float>(b), i, ntiles,
                                         all, kx, ky, part, dout, b->stream);
    if (e != hipSuccess) return hip_fail(b, e, "fourier launch");
    e = hipMemcpyAsync(out, dout, sizeof(double) * 8, hipMemcpyDeviceToHost, b->stream);
    if (e != hipSuccess) return hip_fail(b, e, "fourier copy");
    e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(b, e, "fourier sync");
    return LBM13_OK;
}

int lbm13_batch_get_state(lbm13_batch* b, int i, double* dst) {
    if (!check_index(b, i) || !dst) return b ? fail(b, LBM13_EINVAL, "bad argument") : LBM13_EINVAL;
    if (!b->has_state[i]) return fail(b, LBM13_ESTATE, "no state");
    if (!b->has_params[i]) return fail(b, LBM13_ESTATE, "no parameters");
    hipError_t e;
    if (b->precision == LBM13_FP64)
        e = lbm13::launch_get_state<double>(b->nx[i], b->ny[i], buf<double>(b, b->cur), doms_dev<double>(b), i, dst,
                                            b->stream);
    else
        e = lbm13::launch_get_state<float>(b->nx[i], b->ny[i], buf<float>(b, b->cur), doms_dev<float>(b), i, dst,
                                           b->stream);
    return e == hipSuccess ? LBM13_OK : hip_fail(b, e, "get_state launch");
}

int lbm13_batch_set_state(lbm13_batch* b, int i, const double* src) {
    if (!check_index(b, i) || !src) return b ? fail(b, LBM13_EINVAL, "bad argument") : LBM13_EINVAL;
    if (!b->has_params[i]) return fail(b, LBM13_ESTATE, "set_params first");
    hipError_t e;
    if (b->precision == LBM13_FP64)
        e = lbm13::launch_set_state<double>(b->nx[i], b->ny[i], buf<double>(b, b->cur), doms_dev<double>(b), i, src,
                                            b->stream);
    else
        e = lbm13::launch_set_state<float>(b->nx[i], b->ny[i], buf<float>(b, b->cur), doms_dev<float>(b), i, src,
                                           b->stream);
    if (e != hipSuccess) return hip_fail(b, e, "set_state launch");
    e = fill_side_any(b, i);
    if (e != hipSuccess) return hip_fail(b, e, "side fill launch");
    b->has_state[i] = 1;
    return LBM13_OK;
}

static size_t payload_bytes(const lbm13_batch* b, int i) {
    return (size_t)13 * b->nx[i] * b->ny[i] * (b->precision == LBM13_FP64 ? 8 : 4);
}

size_t lbm13_batch_state_bytes(const lbm13_batch* b, int i) {
    if (!b || i < 0 || i >= b->count) return 0;
    return lbm13::kCkptHeaderBytes + payload_bytes(b, i);
}

// Raw copies between the padded planes and a dense [13][ny][nx] array.
static int raw_copy(lbm13_batch* b, int i, void* dense, const void* dense_src) {
    const size_t es = b->precision == LBM13_FP64 ? 8 : 4;
    char* plane0 = b->bufp[b->cur] + es * (size_t)b->L.off[i];
    const size_t row = es * b->nx[i], pitch = es * b->L.pitch[i], plane = es * (size_t)b->L.plane[i];
    const size_t dplane = row * b->ny[i];
    for (int q = 0; q < 13; ++q) {
        hipError_t e;
        if (dense)
            e = hipMemcpy2DAsync(static_cast<char*>(dense) + q * dplane, row, plane0 + q * plane, pitch, row,
                                 b->ny[i], hipMemcpyDeviceToDevice, b->stream);
        else
            e = hipMemcpy2DAsync(plane0 + q * plane, pitch, static_cast<const char*>(dense_src) + q * dplane, row,
                                 row, b->ny[i], hipMemcpyDeviceToDevice, b->stream);
        if (e != hipSuccess) return hip_fail(b, e, "raw state copy");
    }
    return LBM13_OK;
}

int lbm13_batch_save(lbm13_batch* b, int i, void* dst, size_t dst_bytes) {
    if (!check_index(b, i) || !dst) return b ? fail(b, LBM13_EINVAL, "bad argument") : LBM13_EINVAL;
    if (dst_bytes < lbm13_batch_state_bytes(b, i)) return fail(b, LBM13_EINVAL, "checkpoint buffer too small");
    if (!b->has_state[i]) return fail(b, LBM13_ESTATE, "no state");
    lbm13::CkptHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, "LBM13CK", 8);
    h.version = lbm13::kCkptVersion;
    h.precision = b->precision;
    h.nx = b->nx[i];
    h.ny = b->ny[i];
    h.steps = b->steps;
    h.payload = payload_bytes(b, i);
    hipError_t e = lbm13::launch_ckpt_header(h, dst, b->stream);
    if (e != hipSuccess) return hip_fail(b, e, "checkpoint header");
    return raw_copy(b, i, static_cast<char*>(dst) + lbm13::kCkptHeaderBytes, nullptr);
}

// Reads the checkpoint's header back (synchronising the stream) and accepts it
// only for this domain's size and precision; restores the populations and,
// when restore_steps, the step counter.
static int load_impl(lbm13_batch* b, int i, const void* src, size_t src_bytes, bool restore_steps) {
    if (!check_index(b, i) || !src) return b ? fail(b, LBM13_EINVAL, "bad argument") : LBM13_EINVAL;
    if (src_bytes != lbm13_batch_state_bytes(b, i))
        return fail(b, LBM13_EINVAL, "checkpoint size does not match this domain");
    if (!b->has_params[i]) return fail(b, LBM13_ESTATE, "set_params first");
    lbm13::CkptHeader h;
    hipError_t e = hipMemcpyAsync(&h, src, sizeof h, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(b, e, "checkpoint header read");
    if (std::memcmp(h.magic, "LBM13CK", 8) != 0 || h.version != lbm13::kCkptVersion)
        return fail(b, LBM13_EINVAL, "not a checkpoint of this library");
    if (h.precision != b->precision || h.nx != b->nx[i] || h.ny != b->ny[i] || h.payload != payload_bytes(b, i))
        return fail(b, LBM13_EINVAL, "checkpoint of another domain size or precision");
    int st = raw_copy(b, i, nullptr, static_cast<const char*>(src) + lbm13::kCkptHeaderBytes);
    if (st != LBM13_OK) return st;
    e = fill_side_any(b, i);
    if (e != hipSuccess) return hip_fail(b, e, "side fill launch");
    b->has_state[i] = 1;
    if (restore_steps) b->steps = h.steps;
    return LBM13_OK;
}

int lbm13_batch_load(lbm13_batch* b, int i, const void* src, size_t src_bytes) {
    return load_impl(b, i, src, src_bytes, false);
}

int lbm13_batch_set_tile(lbm13_batch* b, int tile_x, int tile_y) {
    if (!b) return LBM13_EINVAL;
    if (!valid_shape(tile_x, tile_y)) return fail(b, LBM13_EINVAL, "unsupported tile shape");
    b->tile_x = tile_x;
    b->tile_y = tile_y;
    return rebuild(b);
}

int lbm13_batch_autotune(lbm13_batch* b, int steps, int* tile_x, int* tile_y) {
    if (!b || steps <= 0) return b ? fail(b, LBM13_EINVAL, "steps must be positive") : LBM13_EINVAL;
    int st = ready(b);
    if (st) return st;
    return b->precision == LBM13_FP64 ? autotune_impl<double>(b, steps, tile_x, tile_y)
                                      : autotune_impl<float>(b, steps, tile_x, tile_y);
}

int lbm13_batch_autotune_cached(lbm13_batch* b, int steps, const char* cache_path, int* from_cache) {
    if (from_cache) *from_cache = 0;
    if (!b || steps <= 0 || !cache_path) return b ? fail(b, LBM13_EINVAL, "bad argument") : LBM13_EINVAL;
    int st = ready(b);
    if (st) return st;
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(b, e, "device properties");
    bool walls = false;
    for (int k : b->sides_kind) walls = walls || k != LBM13_PERIODIC;
    const std::string key = lbm13::tune_key(prop.gcnArchName, b->precision, lbm13_batch_nodes(b), b->count, walls);
    int cfg[6];
    if (lbm13::tune_cache_lookup(cache_path, key, cfg)) {
        // accept only a configuration this build supports for this precision
        bool ok = cfg[0] >= 1 && cfg[0] <= 3 && valid_shape(cfg[1], cfg[2]) && cfg[5] >= 0 && cfg[5] <= 2;
        bool fused = false;
        for (auto& f : kFusedShapes) fused = fused || (f[0] == cfg[3] && f[1] == cfg[4]);
        ok = ok && fused && fused_fits(b->precision, cfg[3], cfg[4]);
        if (ok && cfg[0] == 3) ok = step3_shape(b->precision, cfg[3], cfg[4]);
        if (ok) {
            b->spl = cfg[0];
            b->tile_x = cfg[1];
            b->tile_y = cfg[2];
            b->ftw = cfg[3];
            b->fth = cfg[4];
            b->split = cfg[5];
            st = rebuild(b);
            if (st) return st;
            if (from_cache) *from_cache = 1;
            return LBM13_OK;
        }
    }
    st = lbm13_batch_autotune(b, steps, nullptr, nullptr);
    if (st) return st;
    (void)lbm13_batch_launch_config(b, cfg);
    if (!lbm13::tune_cache_store(cache_path, key, cfg)) b->err = "autotuned; the cache file could not be written";
    return LBM13_OK;
}

int lbm13_batch_use_graph(lbm13_batch* b, int k) {
    if (!b) return LBM13_EINVAL;
    if (k != 0 && (k < 2 || k > 4096 || (k & 1))) return fail(b, LBM13_EINVAL, "graph length must be even, 2..4096");
    drop_graphs(b);
    b->graph_k = k;
    return LBM13_OK;
}

int lbm13_batch_set_fused_tile(lbm13_batch* b, int tile_x, int tile_y) {
    if (!b) return LBM13_EINVAL;
    bool ok = false;
    for (auto& f : kFusedShapes) ok = ok || (f[0] == tile_x && f[1] == tile_y);
    if (!ok || !fused_fits(b->precision, tile_x, tile_y))
        return fail(b, LBM13_EINVAL, "unsupported two-step tile shape for this precision");
    b->ftw = tile_x;
    b->fth = tile_y;
    return rebuild(b);
}

int lbm13_batch_set_steps_per_launch(lbm13_batch* b, int k) {
    if (!b) return LBM13_EINVAL;
    if (k != 1 && k != 2 && k != 3) return fail(b, LBM13_EINVAL, "steps per launch must be 1, 2 or 3");
    drop_graphs(b);
    b->spl = k;
    return LBM13_OK;
}

int lbm13_batch_set_interior_kernel(lbm13_batch* b, int on) {
    if (!b) return LBM13_EINVAL;
    if (on < 0 || on > 2) return fail(b, LBM13_EINVAL, "interior kernel switch must be 0, 1 or 2");
    b->split = on;
    return rebuild(b);
}

int lbm13_batch_launch_config(const lbm13_batch* b, int cfg[6]) {
    if (!b || !cfg) return LBM13_EINVAL;
    cfg[0] = b->spl;
    cfg[1] = b->tile_x;
    cfg[2] = b->tile_y;
    cfg[3] = b->ftw;
    cfg[4] = b->fth;
    cfg[5] = b->split;
    return LBM13_OK;
}

long long lbm13_batch_nodes(const lbm13_batch* b) {
    if (!b) return 0;
    long long n = 0;
    for (int d = 0; d < b->count; ++d) n += (long long)b->nx[d] * b->ny[d];
    return n;
}

int lbm13_batch_destroy(lbm13_batch* b) {
    if (!b) return LBM13_EINVAL;
    // queued launches and graph replays still use the graphs, streams, events
    // and workspace: let them finish first
    (void)hipStreamSynchronize(b->stream);
    if (b->aux) (void)hipStreamSynchronize(b->aux);
    drop_graphs(b);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    if (b->aux) (void)hipStreamDestroy(b->aux);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    delete b;
    return LBM13_OK;
}

const char* lbm13_batch_last_error(const lbm13_batch* b) {
    if (b) return b->err.c_str();
    return g_create_err.empty() ? "null batch" : g_create_err.c_str();
}

// =========================================================================== single-domain API

size_t lbm13_workspace_bytes(int nx, int ny, int precision) {
    return lbm13_batch_workspace_bytes(1, &nx, &ny, precision);
}

int lbm13_create(int nx, int ny, int precision, void* workspace, size_t workspace_bytes, void* stream,
                 lbm13_ctx** out) {
    if (!out) return LBM13_EINVAL;
    *out = nullptr;
    lbm13_ctx* c = new (std::nothrow) lbm13_ctx;
    if (!c) return LBM13_ENOMEM;
    int st = lbm13_batch_create(1, &nx, &ny, precision, workspace, workspace_bytes, stream, &c->b);
    if (st) {
        delete c;
        return st;
    }
    *out = c;
    return LBM13_OK;
}

int lbm13_set_params(lbm13_ctx* c, const lbm13_params* p, const lbm13_side sides[4], lbm13_derived* derived) {
    return c ? lbm13_batch_set_params(c->b, 0, p, sides, derived) : LBM13_EINVAL;
}

int lbm13_init_moments(lbm13_ctx* c, const double* rho, const double* ux, const double* uy, const double* T) {
    return c ? lbm13_batch_init_moments(c->b, 0, rho, ux, uy, T) : LBM13_EINVAL;
}

int lbm13_step(lbm13_ctx* c, long long n) { return c ? lbm13_batch_step(c->b, n) : LBM13_EINVAL; }

int lbm13_moments(lbm13_ctx* c, double* rho, double* ux, double* uy, double* T) {
    return c ? lbm13_batch_moments(c->b, 0, rho, ux, uy, T) : LBM13_EINVAL;
}

int lbm13_diagnostics(lbm13_ctx* c, double out[16]) { return c ? lbm13_batch_diagnostics(c->b, out) : LBM13_EINVAL; }

int lbm13_fourier(lbm13_ctx* c, int kx, int ky, double out[8]) {
    return c ? lbm13_batch_fourier(c->b, 0, kx, ky, out) : LBM13_EINVAL;
}

int lbm13_get_state(lbm13_ctx* c, double* dst) { return c ? lbm13_batch_get_state(c->b, 0, dst) : LBM13_EINVAL; }

int lbm13_set_state(lbm13_ctx* c, const double* src) {
    return c ? lbm13_batch_set_state(c->b, 0, src) : LBM13_EINVAL;
}

long long lbm13_steps_done(const lbm13_ctx* c) { return c && c->b ? c->b->steps : 0; }

size_t lbm13_state_bytes(const lbm13_ctx* c) { return c ? lbm13_batch_state_bytes(c->b, 0) : 0; }

int lbm13_save(lbm13_ctx* c, void* dst, size_t dst_bytes) {
    return c ? lbm13_batch_save(c->b, 0, dst, dst_bytes) : LBM13_EINVAL;
}

int lbm13_load(lbm13_ctx* c, const void* src, size_t src_bytes) {
    return c ? load_impl(c->b, 0, src, src_bytes, true) : LBM13_EINVAL;
}

int lbm13_set_tile(lbm13_ctx* c, int tile_x, int tile_y) {
    return c ? lbm13_batch_set_tile(c->b, tile_x, tile_y) : LBM13_EINVAL;
}

int lbm13_autotune(lbm13_ctx* c, int steps, int* tile_x, int* tile_y) {
    return c ? lbm13_batch_autotune(c->b, steps, tile_x, tile_y) : LBM13_EINVAL;
}

int lbm13_autotune_cached(lbm13_ctx* c, int steps, const char* cache_path, int* from_cache) {
    return c ? lbm13_batch_autotune_cached(c->b, steps, cache_path, from_cache) : LBM13_EINVAL;
}

int lbm13_use_graph(lbm13_ctx* c, int k) { return c ? lbm13_batch_use_graph(c->b, k) : LBM13_EINVAL; }

int lbm13_launch_config(const lbm13_ctx* c, int cfg[6]) { return c ? lbm13_batch_launch_config(c->b, cfg) : LBM13_EINVAL; }

int lbm13_set_interior_kernel(lbm13_ctx* c, int on) {
    return c ? lbm13_batch_set_interior_kernel(c->b, on) : LBM13_EINVAL;
}

int lbm13_set_fused_tile(lbm13_ctx* c, int tile_x, int tile_y) {
    return c ? lbm13_batch_set_fused_tile(c->b, tile_x, tile_y) : LBM13_EINVAL;
}

int lbm13_set_steps_per_launch(lbm13_ctx* c, int k) {
    return c ? lbm13_batch_set_steps_per_launch(c->b, k) : LBM13_EINVAL;
}

int lbm13_destroy(lbm13_ctx* c) {
    if (!c) return LBM13_EINVAL;
    int st = lbm13_batch_destroy(c->b);
    delete c;
    return st;
}

int lbm13_advance_noalloc(int nx, int ny, int precision, const lbm13_params* p, const lbm13_side sides[4],
                          const double* f_in, double* f_out, long long n, void* stream) {
    if (!p || !sides || !f_in || !f_out || n < 0) return noalloc_fail(LBM13_EINVAL, "bad argument");
    Layout L;
    if (!make_layout(1, &nx, &ny, precision, L)) return noalloc_fail(LBM13_EINVAL, "invalid size or precision");
    if (L.total > lbm13::kNoallocScratchBytes)
        return noalloc_fail(LBM13_EINVAL, "a " + std::to_string(nx) + " x " + std::to_string(ny) + " domain needs " +
                                              std::to_string(L.total) + " bytes; the static scratch holds " +
                                              std::to_string(lbm13::kNoallocScratchBytes));
    for (int w = 0; w < 4; ++w)
        if (sides[w].kind < LBM13_PERIODIC || sides[w].kind > LBM13_WALL_DIRICHLET_T)
            return noalloc_fail(LBM13_EINVAL, "unknown side kind");
    if ((sides[0].kind == LBM13_PERIODIC) != (sides[1].kind == LBM13_PERIODIC) ||
        (sides[2].kind == LBM13_PERIODIC) != (sides[3].kind == LBM13_PERIODIC))
        return noalloc_fail(LBM13_EINVAL, "opposite sides must both be periodic or both walls");
    lbm13_derived dv;
    if (derive(p, &dv) != LBM13_OK)
        return noalloc_fail(LBM13_EUNSTABLE_PARAMS, "relaxation rate outside (0, 2) or degenerate constants");
    void* sp = nullptr;
    hipError_t e = lbm13::noalloc_scratch(&sp);
    if (e != hipSuccess) return noalloc_fail(LBM13_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    lbm13_batch b;
    b.count = 1;
    b.precision = precision;
    b.nx.assign(1, nx);
    b.ny.assign(1, ny);
    b.L = L;
    b.ws = static_cast<char*>(sp);
    b.bufp[0] = b.ws + L.bufA;
    b.bufp[1] = b.ws + L.bufB;
    b.noalloc = true;
    b.stream = static_cast<hipStream_t>(stream);
    b.dom_host.assign(dom_size(&b), 0);
    b.coef_host.assign(kCoef, 0.0);
    b.sides_kind.assign(4, LBM13_PERIODIC);
    for (int w = 0; w < 4; ++w) b.sides_kind[w] = sides[w].kind;
    b.has_params.assign(1, 0);
    b.has_state.assign(1, 0);
    b.ftw = precision == LBM13_FP64 ? lbm13::Fused<double>::TW : lbm13::Fused<float>::TW;
    b.fth = precision == LBM13_FP64 ? lbm13::Fused<double>::TH : lbm13::Fused<float>::TH;
    b.split = 0;
    b.spl = 3;
    const int st = precision == LBM13_FP64 ? advance_noalloc_impl<double>(b, p, sides, dv, f_in, f_out, n)
                                           : advance_noalloc_impl<float>(b, p, sides, dv, f_in, f_out, n);
    if (st) return noalloc_fail(st, b.err);
    return LBM13_OK;
}

const char* lbm13_last_error(const lbm13_ctx* c) {
    if (c) return lbm13_batch_last_error(c->b);
    return g_create_err.empty() ? "null context" : g_create_err.c_str();
}

}  // extern "C"
