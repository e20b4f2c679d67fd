// lbm13_kernels.hip -- HIP kernels of the D2Q13 energy-conserving lattice
// Boltzmann step for CDNA4 (gfx950).
//
// Scheme: Lallemand & Dubois, "Comparison of Simulations of Convective Flows",
// sec. 2 (velocities, moments, equilibria, constraints), secs. 5 and 8 (body
// forces), sec. 7 (mixed bounce-back / anti-bounce-back walls, temperature).
//
// The step is a pull: each node gathers the 13 post-collision populations of
// the previous step from x - v_i (reach 1 and 2), substitutes wall links,
// collides in registers and writes its 13 new post-collision values with
// coalesced non-temporal stores.  One wavefront covers 64 (or 2 x 32)
// consecutive nodes of a row, so every population plane is read and written
// as contiguous 256/512-byte segments; the +-1/+-2 shifted reads of
// neighbouring wavefronts share cache lines in L2.  The two- and three-step
// kernels advance a tile and a halo of two nodes per extra step, keeping the
// intermediate states in LDS, so HBM is read and written once per launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "lbm13_device.h"

namespace lbm13 {

// Velocity set (eq d2q13-vitesses) and the moment matrix of eq (d2q13-polynomes)
// with the q polynomial read as x(x^2 + y^2 - 3), rows rho, E, eps, varpi, jx,
// jy, qx, qy, rx, ry, XX, XY, XXe.  Used by the wall path and the diagnostics;
// the bulk collision below uses the same matrix in pair-symmetric form.
__constant__ int c_vx[13] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0};
__constant__ int c_vy[13] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2};
__constant__ int c_cls[13] = {0, 1, 1, 1, 1, 2, 2, 2, 2, 3, 3, 3, 3};  // |v|^2 class
__constant__ float c_M[13][13] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-28, -15, -15, -15, -15, -2, -2, -2, -2, 24, 24, 24, 24},
    {140, -2, -2, -2, -2, -67, -67, -67, -67, 34, 34, 34, 34},
    {-12, 8, 8, 8, 8, -6, -6, -6, -6, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0},
    {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2},
    {0, -2, 0, 2, 0, -1, 1, 1, -1, 2, 0, -2, 0},
    {0, 0, -2, 0, 2, -1, -1, 1, 1, 0, 2, 0, -2},
    {0, 4, 0, -4, 0, -3, 3, 3, -3, 1, 0, -1, 0},
    {0, 0, 4, 0, -4, -3, -3, 3, 3, 0, 1, 0, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0, 4, -4, 4, -4},
    {0, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, -4, 4, -4, 4, 0, 0, 0, 0, 1, -1, 1, -1}};
__constant__ float c_D[13] = {13, 4004, 42196, 548, 14, 14, 20, 20, 70, 70, 68, 4, 68};

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// 1 / x from the hardware reciprocal: FP32 within 1 ulp; FP64 refined by two
// Newton steps e = 1 - x y, y <- y + y e (each squares the relative error).
__device__ __forceinline__ float reciprocal(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double reciprocal(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(y, e, y);
}

// ---------------------------------------------------------------------------
// Collision of one node, in place on the deviations g (sec. 2):
//   m = M g; Delta_k = s_k (m_k - m_k^eq) on the nine non-conserved moments;
//   j* = j + F (secs. 5, 8); E* = E + Q_E (sec. 9); g* = g - M^T D^-1 Delta.
// Pairs (i, opposite of i) give sums s (even moments) and differences d (odd
// moments); the inverse splits the same way.  Sourced = false drops the body
// force and energy-source terms, for launches whose domains have neither.
template <typename R, bool Sourced = true>
__device__ __forceinline__ void collide(R g[13], const Dom<R>& D) {
    const R s13 = g[1] + g[3], d13 = g[1] - g[3];
    const R s24 = g[2] + g[4], d24 = g[2] - g[4];
    const R s57 = g[5] + g[7], d57 = g[5] - g[7];
    const R s68 = g[6] + g[8], d68 = g[6] - g[8];
    const R s9 = g[9] + g[11], d9 = g[9] - g[11];
    const R s10 = g[10] + g[12], d10 = g[10] - g[12];
    const R S1 = s13 + s24, S2 = s57 + s68, S3 = s9 + s10;
    const R rho = g[0] + S1 + S2 + S3;  // rho - 1
    const R E = R(-28) * g[0] - R(15) * S1 - R(2) * S2 + R(24) * S3;  // E - E0
    const R A1 = s13 - s24, A3 = s9 - s10;
    const R XX = A1 + R(4) * A3;
    const R XY = s57 - s68;
    const R XXe = R(-4) * A1 + A3;
    const R p = d57 - d68, m = d57 + d68;  // diagonal pair differences along x and along y
    const R jx = (d13 + p) + R(2) * d9;
    const R jy = (d24 + m) + R(2) * d10;

    const R inv_rho = reciprocal(R(1) + rho);
    // Delta_k / D_k for the anisotropic even moments
    const R aXX = D.kX * (XX - (jx * jx - jy * jy) * inv_rho);
    const R aXY = D.kY * (XY - jx * jy * inv_rho);
    const R aXXe = D.kXe * XXe;

    // odd moments: non-equilibrium parts of q and r per axis (q^eq, r^eq = j
    // times affine functions of rho and E), mapped onto the three update
    // patterns of the axis (speed-1 link, speed-2 link, diagonal) by weights
    // that fold s_q, s_r and the norms: D.ow = (-2, 4; 2, 1; -1, -3) x (kq, kr)
    const R fq = D.a1 + D.h1 * rho + D.k1 * E;
    const R fr = D.a2 + D.h2 * rho + D.k2 * E;
    const R nqx = (R(2) * (d9 - d13) - p) - jx * fq, nrx = (R(4) * d13 + d9 - R(3) * p) - jx * fr;
    const R nqy = (R(2) * (d10 - d24) - m) - jy * fq, nry = (R(4) * d24 + d10 - R(3) * m) - jy * fr;
    R o1 = D.ow[0] * nqx + D.ow[1] * nrx;
    R o9 = D.ow[2] * nqx + D.ow[3] * nrx;
    R odx = D.ow[4] * nqx + D.ow[5] * nrx;
    R o2 = D.ow[0] * nqy + D.ow[1] * nry;
    R o10 = D.ow[2] * nqy + D.ow[3] * nry;
    R ody = D.ow[4] * nqy + D.ow[5] * nry;

    // isotropic even part: eps and varpi relaxed (each a linear form of the
    // class sums), mapped back by the integer rows of M so that the update
    // keeps sum g and the E moment exactly
    const R aeps = D.aeps[0] * g[0] + D.aeps[1] * S1 + D.aeps[2] * S2 + D.aeps[3] * S3;
    const R avp = D.avp[0] * g[0] + D.avp[1] * S1 + D.avp[2] * S2 + D.avp[3] * S3;
    R e0 = R(140) * aeps - R(12) * avp;
    R ec1 = R(-2) * aeps + R(8) * avp;
    R ec5 = R(-67) * aeps - R(6) * avp;
    R ec9 = R(34) * aeps + avp;
    if constexpr (Sourced) {
        // the energy source enters as Delta_E = -Q_E (sec. 9), the force as
        // Delta_j = -F (secs. 5, 8)
        e0 += D.eQ[0];
        ec1 += D.eQ[1];
        ec5 += D.eQ[2];
        ec9 += D.eQ[3];
        const R bjx = D.fjx + D.gjx * rho, bjy = D.fjy + D.gjy * rho;
        o1 += bjx;
        o2 += bjy;
        o9 += R(2) * bjx;
        o10 += R(2) * bjy;
        odx += bjx;
        ody += bjy;
    }
    const R o5 = odx + ody, o6 = ody - odx;
    const R t1 = aXX - R(4) * aXXe, t9 = R(4) * aXX + aXXe;
    const R e1 = ec1 + t1;
    const R e2 = ec1 - t1;
    const R e5 = ec5 + aXY;
    const R e6 = ec5 - aXY;
    const R e9 = ec9 + t9;
    const R e10 = ec9 - t9;

    g[0] -= e0;
    g[1] -= e1 + o1;
    g[3] -= e1 - o1;
    g[2] -= e2 + o2;
    g[4] -= e2 - o2;
    g[5] -= e5 + o5;
    g[7] -= e5 - o5;
    g[6] -= e6 + o6;
    g[8] -= e6 - o6;
    g[9] -= e9 + o9;
    g[11] -= e9 - o9;
    g[10] -= e10 + o10;
    g[12] -= e10 - o10;
}

// ---------------------------------------------------------------------------
// Gather for a node whose 13 sources are all inside the domain or across a
// periodic side.
template <typename R>
__device__ __forceinline__ void gather_bulk(const R* __restrict__ b, const Dom<R>& D, int x, int y, R g[13]) {
    const int P = D.pitch, S = D.plane;
    int xm1 = x - 1, xm2 = x - 2, xp1 = x + 1, xp2 = x + 2;
    int ym1 = y - 1, ym2 = y - 2, yp1 = y + 1, yp2 = y + 2;
    if (D.xper) {
        xm1 = wrap(xm1, D.nx); xm2 = wrap(xm2, D.nx); xp1 = wrap(xp1, D.nx); xp2 = wrap(xp2, D.nx);
    }
    if (D.yper) {
        ym1 = wrap(ym1, D.ny); ym2 = wrap(ym2, D.ny); yp1 = wrap(yp1, D.ny); yp2 = wrap(yp2, D.ny);
    }
    const int r0 = y * P, rm1 = ym1 * P, rm2 = ym2 * P, rp1 = yp1 * P, rp2 = yp2 * P;
    g[0] = b[r0 + x];
    g[1] = b[1 * S + r0 + xm1];
    g[2] = b[2 * S + rm1 + x];
    g[3] = b[3 * S + r0 + xp1];
    g[4] = b[4 * S + rp1 + x];
    g[5] = b[5 * S + rm1 + xm1];
    g[6] = b[6 * S + rm1 + xp1];
    g[7] = b[7 * S + rp1 + xp1];
    g[8] = b[8 * S + rp1 + xm1];
    g[9] = b[9 * S + r0 + xm2];
    g[10] = b[10 * S + rm2 + x];
    g[11] = b[11 * S + r0 + xp2];
    g[12] = b[12 * S + rp2 + x];
}

// Deviation moments rho' and E' of one stored node.
template <typename R>
__device__ __forceinline__ void node_rho_E(const R* __restrict__ b, const Dom<R>& D, int c, R& rho, R& E) {
    R r = R(0), e = R(0);
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        const R v = b[i * D.plane + c];
        r += v;
        e += R(c_M[1][i]) * v;
    }
    rho = r;
    E = e;
}

// Side array of the wall layers: for every position along every wall, rho' and
// E' of the first fluid layer and rho' of the second, for the state kept in
// buffer `buf` (the step kernel writes them for the state it produces).
template <typename R>
__device__ __forceinline__ R* side_line(R* side, const Dom<R>& D, int buf, int line) {
    return side + D.woff + (long long)buf * (2 * (D.nx + D.ny)) * 4 + line * 4;
}

// Fill the side array from a stored state (after init, set_state or load).
template <typename R>
__global__ __launch_bounds__(256) void side_fill_kernel(const R* __restrict__ src, const Dom<R>* __restrict__ doms,
                                                        const WallLine* __restrict__ lines, int nlines,
                                                        R* __restrict__ side, int buf, int only_dom) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlines) return;
    const WallLine wl = lines[l];
    if (only_dom >= 0 && wl.dom != only_dom) return;
    const Dom<R>& D = doms[wl.dom];
    const R* __restrict__ b = src + D.off;
    const int w = wl.w, pos = wl.pos;
    int c0, c1;
    if (w == 0) { c0 = pos * D.pitch; c1 = c0 + 1; }
    else if (w == 1) { c0 = pos * D.pitch + D.nx - 1; c1 = c0 - 1; }
    else if (w == 2) { c0 = pos; c1 = D.pitch + pos; }
    else { c0 = (D.ny - 1) * D.pitch + pos; c1 = c0 - D.pitch; }
    R r0, e0, r1, e1;
    node_rho_E(b, D, c0, r0, e0);
    node_rho_E(b, D, c1, r1, e1);
    R* o = side_line(side, D, buf, wl.line);
    o[0] = r0;
    o[1] = e0 - D.QE;  // E(t): the kept post-collision state carries E(t) + Q_E
    o[2] = r1;
    o[3] = R(0);
}

// Compile-time copy of the moment matrix for the wall fix-ups (same rows as c_M).
constexpr int kM[13][13] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-28, -15, -15, -15, -15, -2, -2, -2, -2, 24, 24, 24, 24},
    {140, -2, -2, -2, -2, -67, -67, -67, -67, 34, 34, 34, 34},
    {-12, 8, 8, 8, 8, -6, -6, -6, -6, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0},
    {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2},
    {0, -2, 0, 2, 0, -1, 1, 1, -1, 2, 0, -2, 0},
    {0, 0, -2, 0, 2, -1, -1, 1, 1, 0, 2, 0, -2},
    {0, 4, 0, -4, 0, -3, 3, 3, -3, 1, 0, -1, 0},
    {0, 0, 4, 0, -4, -3, -3, 3, 3, 0, 1, 0, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0, 4, -4, 4, -4},
    {0, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, -4, 4, -4, 4, 0, 0, 0, 0, 1, -1, 1, -1}};
constexpr int kVX[13] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0};
constexpr int kVY[13] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2};
constexpr int kOPP[13] = {0, 3, 4, 1, 2, 7, 8, 5, 6, 11, 12, 9, 10};

// Equilibrium moments of a wall state, pre-divided by the norms D_k, as
// deviations from rest (eq d2q13-moments-equil; sec. 7: rho_W = (3 rho_0 -
// rho_1)/2 from the first two fluid layers at time t, j_W = rho_W u_W along the
// wall, E_W imposed on a temperature wall or E of the first layer on an
// adiabatic wall).  even: rho, E, eps, varpi, XX, XY; odd: jx, jy, qx, qy, rx, ry.
template <typename R>
struct WallState {
    R even[6], odd[6];
};

template <typename R>
__device__ __forceinline__ WallState<R> wall_state(const Dom<R>& D, int w, R rho0, R E0l, R rho1) {
    WallState<R> ws;
    const R rho = R(1.5) * rho0 - R(0.5) * rho1;
    const R E = (D.kind[w] == kDirichletT) ? D.wall_dE[w] : E0l;
    const R u = D.wall_u[w];
    const R rhoW = R(1) + rho;
    const R jt = rhoW * u;
    const R jx = (w < 2) ? R(0) : jt;
    const R jy = (w < 2) ? jt : R(0);
    const R inv = (u != R(0)) ? R(1) / rhoW : R(0);
    ws.even[0] = rho * R(1.0 / 13.0);
    ws.even[1] = E * R(1.0 / 4004.0);
    ws.even[2] = (D.c_er * rho + D.c_eE * E) * R(1.0 / 42196.0);
    ws.even[3] = (D.c_vr * rho + D.c_vE * E) * R(1.0 / 548.0);
    ws.even[4] = (jx * jx - jy * jy) * inv * R(1.0 / 68.0);
    ws.even[5] = jx * jy * inv * R(0.25);
    const R fq = D.a1 + D.h1 * rho + D.k1 * E;
    const R fr = D.a2 + D.h2 * rho + D.k2 * E;
    ws.odd[0] = jx * R(1.0 / 14.0);
    ws.odd[1] = jy * R(1.0 / 14.0);
    ws.odd[2] = jx * fq * R(0.05);
    ws.odd[3] = jy * fq * R(0.05);
    ws.odd[4] = jx * fr * R(1.0 / 70.0);
    ws.odd[5] = jy * fr * R(1.0 / 70.0);
    return ws;
}

// Term added to the reflected population of link I (eq d2q13-cl-abb):
//   bounce-back:      2 sum_{k odd}  M_kI m_k(W) / D_k
//   anti-bounce-back: 2 sum_{k even} M_kI m_k(W) / D_k
// f^rest is even in v, so its odd part vanishes and its even part cancels
// against the reflected rest population: deviations need no other correction.
template <int I, typename R>
__device__ __forceinline__ R wall_term(const WallState<R>& ws, bool abb) {
    if (abb)
        return R(2) * (R(kM[0][I]) * ws.even[0] + R(kM[1][I]) * ws.even[1] + R(kM[2][I]) * ws.even[2] +
                       R(kM[3][I]) * ws.even[3] + R(kM[10][I]) * ws.even[4] + R(kM[11][I]) * ws.even[5]);
    return R(2) * (R(kM[4][I]) * ws.odd[0] + R(kM[5][I]) * ws.odd[1] + R(kM[6][I]) * ws.odd[2] +
                   R(kM[7][I]) * ws.odd[3] + R(kM[8][I]) * ws.odd[4] + R(kM[9][I]) * ws.odd[5]);
}

// Population sources for the gathers.  Coordinates passed to cx/cy are a
// node's coordinate minus a velocity; cx/cy return an in-bounds coordinate:
// wrapped on a periodic axis, clamped on a walled axis (a clamped link is
// always replaced by a wall fix-up).
//   GlobalSrc: the stored state in HBM (domain coordinates).
//   LdsSrc: a tile's region in LDS, RH rows of pitch RW per population,
//   indexed by unwrapped domain coordinates relative to the region's origin.
template <typename R>
struct GlobalSrc {
    const R* __restrict__ b;
    int S, P, nx, ny, xper, yper;
    __device__ __forceinline__ int cx(int X) const { return xper ? wrap(X, nx) : min(max(X, 0), nx - 1); }
    __device__ __forceinline__ int cy(int Y) const { return yper ? wrap(Y, ny) : min(max(Y, 0), ny - 1); }
    __device__ __forceinline__ R get(int i, int X, int Y) const { return b[i * S + Y * P + X]; }
};

template <typename R, int RW, int RH>
struct LdsSrc {
    const R* l;
    int ox, oy, nx, ny, xper, yper;
    __device__ __forceinline__ int cx(int X) const { return xper ? X : min(max(X, 0), nx - 1); }
    __device__ __forceinline__ int cy(int Y) const { return yper ? Y : min(max(Y, 0), ny - 1); }
    __device__ __forceinline__ R get(int i, int X, int Y) const { return l[(i * RH + (Y - oy)) * RW + (X - ox)]; }
};

// Side values (rho' and E' of the first wall layer, rho' of the second) of the
// line at position pos of wall w: from the global side array, or from the
// copy a fused launch keeps in LDS for its region.
template <typename R>
struct GlobalSide {
    R* side;
    int buf;
    __device__ __forceinline__ void get(const Dom<R>& D, int w, int pos, R& r0, R& e0, R& r1) const {
        const int line = w == 0 ? pos : w == 1 ? D.ny + pos : w == 2 ? 2 * D.ny + pos : 2 * D.ny + D.nx + pos;
        const R* p = side_line(side, D, buf, line);
        r0 = p[0];
        e0 = p[1];
        r1 = p[2];
    }
};

template <typename R, int RW, int RH>
struct LdsSide {
    const R* xs;  // [2][RH][3]: West, East walls by region row
    const R* ys;  // [2][RW][3]: South, North walls by region column
    int ox, oy;
    __device__ __forceinline__ void get(const Dom<R>& D, int w, int pos, R& r0, R& e0, R& r1) const {
        const R* p = w < 2 ? xs + (w * RH + (pos - oy)) * 3 : ys + ((w - 2) * RW + (pos - ox)) * 3;
        r0 = p[0];
        e0 = p[1];
        r1 = p[2];
    }
};

// Replace link I, whose source lies beyond wall w, by its reversed path from x'
// (tangential coordinate kept, normal coordinate reflected through the wall).
template <int I, typename R, typename Src>
__device__ __forceinline__ void fix_link(const Src& A, const Dom<R>& D, int w, int x, int y,
                                         const WallState<R>& ws, R g[13]) {
    int px = x, py = y;
    if (w == 0) px = -1 + kVX[I] - x;
    else if (w == 1) px = 2 * D.nx - 1 + kVX[I] - x;
    else if (w == 2) py = -1 + kVY[I] - y;
    else py = 2 * D.ny - 1 + kVY[I] - y;
    const R src = A.get(kOPP[I], px, py);
    const bool normal = (w < 2) ? (kVY[I] == 0) : (kVX[I] == 0);
    const bool abb = normal && D.kind[w] == kDirichletT;
    g[I] = (abb ? -src : src) + wall_term<I>(ws, abb);
}

template <typename R, typename Src, typename Side>
__device__ __forceinline__ void wall_fixups(const Src& A, const Side& SD, const Dom<R>& D, int x, int y, R g[13]);

// Gather for a node within two nodes of a wall: every link is first read with
// in-bounds coordinates, then the links whose source lies beyond a wall are
// replaced (wall_fixups).
template <typename R, typename Src, typename Side>
__device__ __forceinline__ void gather_wall(const Src& A, const Side& SD, const Dom<R>& D, int x, int y, R g[13]) {
    const int xm1 = A.cx(x - 1), xm2 = A.cx(x - 2), xp1 = A.cx(x + 1), xp2 = A.cx(x + 2);
    const int ym1 = A.cy(y - 1), ym2 = A.cy(y - 2), yp1 = A.cy(y + 1), yp2 = A.cy(y + 2);
    g[0] = A.get(0, x, y);
    g[1] = A.get(1, xm1, y);
    g[2] = A.get(2, x, ym1);
    g[3] = A.get(3, xp1, y);
    g[4] = A.get(4, x, yp1);
    g[5] = A.get(5, xm1, ym1);
    g[6] = A.get(6, xp1, ym1);
    g[7] = A.get(7, xp1, yp1);
    g[8] = A.get(8, xm1, yp1);
    g[9] = A.get(9, xm2, y);
    g[10] = A.get(10, x, ym2);
    g[11] = A.get(11, xp2, y);
    g[12] = A.get(12, x, yp2);
    wall_fixups(A, SD, D, x, y, g);
}

// The wall fix-ups of a gather: the links whose source lies beyond a wall
// replaced (bounce-back for links with a tangential component and for every
// link at an adiabatic wall, anti-bounce-back for links normal to a temperature
// wall; sec. 7).  y walls are applied first and x walls last, so a diagonal
// source beyond two walls takes the West/East wall.  Every other link is left
// as gathered.
template <typename R, typename Src, typename Side>
__device__ __forceinline__ void wall_fixups(const Src& A, const Side& SD, const Dom<R>& D, int x, int y, R g[13]) {
    R r0, e0, r1;
    if (!D.yper && y < 2) {  // South wall: links with v_y > 0
        SD.get(D, 2, x, r0, e0, r1);
        const WallState<R> ws = wall_state(D, 2, r0, e0, r1);
        if (y == 0) { fix_link<2>(A, D, 2, x, y, ws, g); fix_link<5>(A, D, 2, x, y, ws, g); fix_link<6>(A, D, 2, x, y, ws, g); }
        fix_link<10>(A, D, 2, x, y, ws, g);
    }
    if (!D.yper && y >= D.ny - 2) {  // North wall: links with v_y < 0
        SD.get(D, 3, x, r0, e0, r1);
        const WallState<R> ws = wall_state(D, 3, r0, e0, r1);
        if (y == D.ny - 1) { fix_link<4>(A, D, 3, x, y, ws, g); fix_link<7>(A, D, 3, x, y, ws, g); fix_link<8>(A, D, 3, x, y, ws, g); }
        fix_link<12>(A, D, 3, x, y, ws, g);
    }
    if (!D.xper && x < 2) {  // West wall: links with v_x > 0
        SD.get(D, 0, y, r0, e0, r1);
        const WallState<R> ws = wall_state(D, 0, r0, e0, r1);
        if (x == 0) { fix_link<1>(A, D, 0, x, y, ws, g); fix_link<5>(A, D, 0, x, y, ws, g); fix_link<8>(A, D, 0, x, y, ws, g); }
        fix_link<9>(A, D, 0, x, y, ws, g);
    }
    if (!D.xper && x >= D.nx - 2) {  // East wall: links with v_x < 0
        SD.get(D, 1, y, r0, e0, r1);
        const WallState<R> ws = wall_state(D, 1, r0, e0, r1);
        if (x == D.nx - 1) { fix_link<3>(A, D, 1, x, y, ws, g); fix_link<6>(A, D, 1, x, y, ws, g); fix_link<7>(A, D, 1, x, y, ws, g); }
        fix_link<11>(A, D, 1, x, y, ws, g);
    }
}

// After collision, a node in the first or second layer of a wall records its
// rho' (and E' for the first layer, without this step's energy source) for the
// next step's wall states.
template <typename R>
__device__ __forceinline__ void record_wall_layers(R* __restrict__ side, const Dom<R>& D, int buf, int x, int y,
                                                   const R g[13]) {
    const bool xw = !D.xper && (x < 2 || x >= D.nx - 2);
    const bool yw = !D.yper && (y < 2 || y >= D.ny - 2);
    if (!xw && !yw) return;
    R rho = R(0), E = -D.QE;
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        rho += g[i];
        E += R(c_M[1][i]) * g[i];
    }
    if (xw) {
        if (x == 0) { R* p = side_line(side, D, buf, y); p[0] = rho; p[1] = E; }
        if (x == 1) side_line(side, D, buf, y)[2] = rho;
        if (x == D.nx - 1) { R* p = side_line(side, D, buf, D.ny + y); p[0] = rho; p[1] = E; }
        if (x == D.nx - 2) side_line(side, D, buf, D.ny + y)[2] = rho;
    }
    if (yw) {
        if (y == 0) { R* p = side_line(side, D, buf, 2 * D.ny + x); p[0] = rho; p[1] = E; }
        if (y == 1) side_line(side, D, buf, 2 * D.ny + x)[2] = rho;
        if (y == D.ny - 1) { R* p = side_line(side, D, buf, 2 * D.ny + D.nx + x); p[0] = rho; p[1] = E; }
        if (y == D.ny - 2) side_line(side, D, buf, 2 * D.ny + D.nx + x)[2] = rho;
    }
}

// A multi-step launch keeps, for the wall lines its region crosses, rho' and E'
// (without the energy source) of the first wall layer and rho' of the second,
// as its collided nodes give them: xs[2][RH][3] for the West and East walls by
// region row, ys[2][RW][3] for the South and North walls by region column.
template <typename R, int RW, int RH>
__device__ __forceinline__ void record_region_layers(R* xs, R* ys, const Dom<R>& D, int X, int Y, int lx, int ly,
                                                     const R g[13]) {
    const bool xw = !D.xper && (X < 2 || X >= D.nx - 2);
    const bool yw = !D.yper && (Y < 2 || Y >= D.ny - 2);
    if (!xw && !yw) return;
    R rho = R(0), E = -D.QE;
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        rho += g[i];
        E += R(c_M[1][i]) * g[i];
    }
    if (xw) {
        if (X == 0) { xs[(0 * RH + ly) * 3 + 0] = rho; xs[(0 * RH + ly) * 3 + 1] = E; }
        if (X == 1) xs[(0 * RH + ly) * 3 + 2] = rho;
        if (X == D.nx - 1) { xs[(1 * RH + ly) * 3 + 0] = rho; xs[(1 * RH + ly) * 3 + 1] = E; }
        if (X == D.nx - 2) xs[(1 * RH + ly) * 3 + 2] = rho;
    }
    if (yw) {
        if (Y == 0) { ys[(0 * RW + lx) * 3 + 0] = rho; ys[(0 * RW + lx) * 3 + 1] = E; }
        if (Y == 1) ys[(0 * RW + lx) * 3 + 2] = rho;
        if (Y == D.ny - 1) { ys[(1 * RW + lx) * 3 + 0] = rho; ys[(1 * RW + lx) * 3 + 1] = E; }
        if (Y == D.ny - 2) ys[(1 * RW + lx) * 3 + 2] = rho;
    }
}

// XCD-aware block order: the hardware deals consecutive workgroups round-robin
// to the 8 XCDs; this remap gives each XCD a contiguous run of tiles so the
// shifted reads of neighbouring tiles hit the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, local = b >> 3;
    return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

template <typename R>
__device__ __forceinline__ void store_node(R* __restrict__ b, int S, int c, const R g[13]) {
#pragma unroll
    for (int i = 0; i < 13; ++i) __builtin_nontemporal_store(g[i], &b[i * S + c]);
}

// One step over a list of tiles.  TX nodes per row, 256/TX rows per pass, RPT
// passes per tile.  WALLS = false: every node is bulk (tiles at least two nodes
// from any wall); WALLS = true: per-node choice between bulk and wall gather.
template <typename R, int TX, int RPT, bool WALLS>
__global__ __launch_bounds__(256) void step_kernel(const R* __restrict__ src, R* __restrict__ dst,
                                                   const Dom<R>* __restrict__ doms,
                                                   const Tile* __restrict__ tiles, int ntiles,
                                                   R* __restrict__ side, int from) {
    constexpr int TYB = 256 / TX;
    const int t = xcd_tile(blockIdx.x, ntiles);
    const Tile tl = tiles[t];
    const Dom<R>& D = doms[tl.dom];
    const R* __restrict__ a = src + D.off;
    R* __restrict__ o = dst + D.off;
    const int x = tl.x0 + threadIdx.x;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int y = tl.y0 + threadIdx.y + r * TYB;
        if (x >= D.nx || y >= D.ny) continue;
        R g[13];
        // In tiles that touch a wall every node takes the clamped gather with
        // per-wall fix-ups (identical to the bulk gather away from walls), so a
        // wavefront never runs both gathers.
        if (WALLS) {
            const GlobalSrc<R> A{a, D.plane, D.pitch, D.nx, D.ny, D.xper, D.yper};
            gather_wall(A, GlobalSide<R>{side, from}, D, x, y, g);
        } else {
            gather_bulk(a, D, x, y, g);
        }
        if (D.collide) collide(g, D);
        store_node(o, D.plane, y * D.pitch + x, g);
        if (WALLS) record_wall_layers(side, D, 1 - from, x, y, g);
    }
}

// ---------------------------------------------------------------------------
// Two steps per launch.  A workgroup owns a TW x TH tile.  Phase 1 advances
// the tile and a two-node halo around it (the reach of the 13 velocities) from
// t to t + 1, gathering from HBM, and keeps the post-collision result in LDS;
// phase 2 advances the tile from t + 1 to t + 2 gathering from LDS and writes
// HBM once.  Each node's arithmetic is the single-step kernel's, so the result
// equals two single steps; HBM traffic per step is about halved (the halo is
// re-read from L2 by neighbouring tiles), for (TW+4)(TH+4)/(TW TH) times the
// phase-1 collision work.  Wall-layer densities of step t + 1 are kept in LDS
// for phase 2's wall states; phase 2 reads every node's sources with the plain
// stencil and then replaces the links from beyond a wall (wall_fixups).
// Waves per SIMD that a workgroup of nt threads with lds_bytes of LDS allows
// (160 KB of LDS and at most 8 waves per SIMD on a CU of 4 SIMDs); the
// multi-step kernels ask the compiler for the registers of that occupancy.
constexpr int lds_waves_per_eu(int lds_bytes, int nt) {
    const int w = (163840 / lds_bytes) * nt / 256;
    return w < 1 ? 1 : (w > 8 ? 8 : w);
}

__device__ __forceinline__ int pmod(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Raw buffer access: a descriptor (uniform base address, byte range) plus a
// 32-bit per-lane byte offset and a uniform byte offset, so a gather of 13
// planes costs no per-lane address arithmetic.  Out-of-range loads return 0 and
// out-of-range stores are dropped.  The descriptor's fourth word selects the
// 32-bit data format of untyped CDNA buffer accesses.
constexpr int kBufferWord3 = 0x00020000;

template <typename R>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const R* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<R*>(base), (short)0, (int)bytes, kBufferWord3);
}

template <typename R>
__device__ __forceinline__ R buffer_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ float buffer_load<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double buffer_load<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// Non-temporal store (cache policy bit 1).
template <typename R>
__device__ __forceinline__ void buffer_store_nt(R v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ void buffer_store_nt<float>(float v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                                       unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 2);
}
template <>
__device__ __forceinline__ void buffer_store_nt<double>(double v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                                        unsigned soff) {
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 2);
}

template <typename R, int TW, int TH, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(
    sizeof(R) == 4 ? lds_waves_per_eu((13 * (TW + 4) * (TH + 4) + 6 * (TW + TH + 8)) * (int)sizeof(R), NT) : 1)))
void step2_kernel(const R* __restrict__ src, R* __restrict__ dst,
                                                   const Dom<R>* __restrict__ doms,
                                                   const Tile* __restrict__ tiles, int ntiles,
                                                   R* __restrict__ side, int from) {
    constexpr int RW = TW + 4, RH = TH + 4, NI = (RW * RH + NT - 1) / NT;
    __shared__ R lds[13 * RH * RW];
    __shared__ R xs[2 * RH * 3];
    __shared__ R ys[2 * RW * 3];
    const int t = xcd_tile(blockIdx.x, ntiles);
    const Tile tl = tiles[t];
    const Dom<R>& D = doms[tl.dom];
    const R* __restrict__ a = src + D.off;
    R* __restrict__ o = dst + D.off;
    const int ox = tl.x0 - 2, oy = tl.y0 - 2;
    const int tid = threadIdx.x;

    if (tl.flags & 2) {
        // Interior tile (when the interior kernel is not used): gathers through
        // one buffer descriptor as in step2_interior_kernel, the whole region in
        // LDS, no wall, wrap or bounds logic.
        constexpr int es = (int)sizeof(R);
        const int P = D.pitch, S = D.plane;
        const __amdgpu_buffer_rsrc_t in = buffer_rsrc(a - (2 * P + 2), (unsigned)((13 * S + 2 * P + 2) * es));
        R h[NI][13];
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int r = min(tid + k * NT, RW * RH - 1);
            const unsigned c = (unsigned)(((oy + r / RW) * P + ox + r % RW) * es);
#pragma unroll
            for (int i = 0; i < 13; ++i)
                h[k][i] = buffer_load<R>(in, c, (unsigned)((i * S + (2 - kVY[i]) * P + 2 - kVX[i]) * es));
        }
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int r = tid + k * NT;
            if (r < RW * RH) {
                if (D.collide) collide(h[k], D);
#pragma unroll
                for (int i = 0; i < 13; ++i) lds[i * RH * RW + r] = h[k][i];
            }
        }
        __syncthreads();
        const __amdgpu_buffer_rsrc_t out = buffer_rsrc(o, (unsigned)(13 * S * es));
        for (int r = tid; r < TW * TH; r += NT) {
            const int lx = r % TW + 2, ly = r / TW + 2;
            const unsigned c = (unsigned)(((oy + ly) * P + ox + lx) * es);
            R q[13];
#pragma unroll
            for (int i = 0; i < 13; ++i) q[i] = lds[(i * RH + ly - kVY[i]) * RW + lx - kVX[i]];
            if (D.collide) collide(q, D);
#pragma unroll
            for (int i = 0; i < 13; ++i) buffer_store_nt<R>(q[i], out, c, (unsigned)(i * S * es));
        }
        return;
    }

    // Phase 1: all gathers of a thread's region nodes are issued before the
    // first collision.  Region nodes beyond a wall (or past the region's end)
    // gather from a clamped in-domain node and store nothing.
    const GlobalSrc<R> G{a, D.plane, D.pitch, D.nx, D.ny, D.xper, D.yper};
    const GlobalSide<R> GS{side, from};
    const bool region_walls = (!D.xper && (ox < 2 || ox + RW > D.nx - 2)) || (!D.yper && (oy < 2 || oy + RH > D.ny - 2));
    const bool tile_walls = (!D.xper && (tl.x0 < 2 || tl.x0 + TW > D.nx - 2)) ||
                            (!D.yper && (tl.y0 < 2 || tl.y0 + TH > D.ny - 2));
    R g[NI][13];
    int Xs[NI], Ys[NI];
    bool valid[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int r = min(tid + k * NT, RW * RH - 1);
        int X = ox + r % RW, Y = oy + r / RW;
        bool v = tid + k * NT < RW * RH;
        // a region wraps at most once around an axis at least as long as itself
        if (D.xper) X = D.nx >= RW ? wrap(X, D.nx) : pmod(X, D.nx);
        else { v = v && X >= 0 && X < D.nx; X = min(max(X, 0), D.nx - 1); }
        if (D.yper) Y = D.ny >= RH ? wrap(Y, D.ny) : pmod(Y, D.ny);
        else { v = v && Y >= 0 && Y < D.ny; Y = min(max(Y, 0), D.ny - 1); }
        Xs[k] = X;
        Ys[k] = Y;
        valid[k] = v;
        // a region that reaches a wall gathers every node with the wall gather
        // (the bulk result away from the wall), so no wavefront runs both
        if (region_walls) gather_wall(G, GS, D, X, Y, g[k]);
        else gather_bulk(a, D, X, Y, g[k]);
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        if (!valid[k]) continue;
        const int r = tid + k * NT, lx = r % RW, ly = r / RW;
        const int X = Xs[k], Y = Ys[k];
        if (D.collide) collide(g[k], D);
#pragma unroll
        for (int i = 0; i < 13; ++i) lds[(i * RH + ly) * RW + lx] = g[k][i];
        record_region_layers<R, RW, RH>(xs, ys, D, X, Y, lx, ly, g[k]);
    }
    __syncthreads();

    const LdsSrc<R, RW, RH> L{lds, ox, oy, D.nx, D.ny, D.xper, D.yper};
    const LdsSide<R, RW, RH> LS{xs, ys, ox, oy};
    for (int r = tid; r < TW * TH; r += NT) {
        const int lx = r % TW + 2, ly = r / TW + 2;
        const int X = ox + lx, Y = oy + ly;
        if (X >= D.nx || Y >= D.ny) continue;
        R g[13];
        const bool near = (!D.xper && (X < 2 || X >= D.nx - 2)) || (!D.yper && (Y < 2 || Y >= D.ny - 2));
#pragma unroll
        for (int i = 0; i < 13; ++i) g[i] = lds[(i * RH + ly - kVY[i]) * RW + lx - kVX[i]];
        if (tile_walls) wall_fixups(L, LS, D, X, Y, g);
        if (D.collide) collide(g, D);
        store_node(o, D.plane, Y * D.pitch + X, g);
        if (near) record_wall_layers(side, D, 1 - from, X, Y, g);
    }
}

// ---------------------------------------------------------------------------
// Two steps per launch on interior tiles (tile flag 2: the tile, its two-node
// halo and every source of their gathers lie inside the domain, at least two
// nodes from any wall, with no wrap).  Phase 2 reads population i of the
// intermediate state only over the tile shifted back by v_i, so LDS keeps
// TW x TH values per population instead of the whole (TW + 4)(TH + 4) region
// and more workgroups share a CU.  Same per-node arithmetic as step2_kernel.
template <int I>
struct Slot {  // LDS slot of population I: velocity 10, (0, 2), takes slot 0
    static constexpr int value = (I + 3) % 13;
};

template <typename R, int TW, int TH, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(
    sizeof(R) == 4 ? lds_waves_per_eu((2 + 13 * TW * TH) * (int)sizeof(R), NT) : 1)))
void step2_interior_kernel(const R* __restrict__ src, R* __restrict__ dst,
                                                           const Dom<R>* __restrict__ doms,
                                                           const Tile* __restrict__ tiles, int ntiles) {
    constexpr int RW = TW + 4, RH = TH + 4, N = TW * TH;
    constexpr int NI = (RW * RH + NT - 1) / NT;
    // population i of region node (lx, ly) sits at kLead + slot(i) N + (ly - 2 + vy_i) TW + lx - 2 + vx_i;
    // kLead keeps that index non-negative for the population in slot 0
    constexpr int kLead = 2;
    __shared__ R lds[kLead + 13 * N];
    const int t = xcd_tile(blockIdx.x, ntiles);
    const Tile tl = tiles[t];
    const Dom<R>& D = doms[tl.dom];
    const R* __restrict__ a = src + D.off;
    R* __restrict__ o = dst + D.off;
    const int P = D.pitch, S = D.plane;
    const int tid = threadIdx.x;

    // Phase 1: every region node a thread owns is requested before the first
    // collision, so the memory latencies overlap (a thread past the region's
    // end re-reads its last node and stores nothing).  The 13 planes are read
    // through one descriptor based two rows and two columns before plane 0, so
    // every per-velocity offset is non-negative (interior tiles exist only in
    // domains whose planes span less than 2^31 bytes).
    constexpr int es = (int)sizeof(R);
    const __amdgpu_buffer_rsrc_t in = buffer_rsrc(a - (2 * P + 2), (unsigned)((13 * S + 2 * P + 2) * es));
    R g[NI][13];
    int lxs[NI], lys[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int r = min(tid + k * NT, RW * RH - 1);
        lxs[k] = r % RW;
        lys[k] = r / RW;
        const unsigned c = (unsigned)(((tl.y0 - 2 + lys[k]) * P + tl.x0 - 2 + lxs[k]) * es);
#pragma unroll
        for (int i = 0; i < 13; ++i)
            g[k][i] = buffer_load<R>(in, c, (unsigned)((i * S + (2 - kVY[i]) * P + 2 - kVX[i]) * es));
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        if (tid + k * NT < RW * RH) {
            if (D.collide) collide(g[k], D);
            const int lx = lxs[k], ly = lys[k], base = ly * TW + lx;
#define LBM13_WINDOW_STORE(I)                                                                              \
    if ((unsigned)(lx - 2 + kVX[I]) < (unsigned)TW && (unsigned)(ly - 2 + kVY[I]) < (unsigned)TH)          \
        lds[base + (kLead + Slot<I>::value * N + (kVY[I] - 2) * TW + kVX[I] - 2)] = g[k][I];
            LBM13_WINDOW_STORE(0) LBM13_WINDOW_STORE(1) LBM13_WINDOW_STORE(2) LBM13_WINDOW_STORE(3)
            LBM13_WINDOW_STORE(4) LBM13_WINDOW_STORE(5) LBM13_WINDOW_STORE(6) LBM13_WINDOW_STORE(7)
            LBM13_WINDOW_STORE(8) LBM13_WINDOW_STORE(9) LBM13_WINDOW_STORE(10) LBM13_WINDOW_STORE(11)
            LBM13_WINDOW_STORE(12)
#undef LBM13_WINDOW_STORE
        }
    }
    __syncthreads();

    // Phase 2: tile node r reads every population at index r of its slot.
    const __amdgpu_buffer_rsrc_t out = buffer_rsrc(o, (unsigned)(13 * S * es));
    for (int r = tid; r < N; r += NT) {
        const int tx = r % TW, ty = r / TW;
        const unsigned c = (unsigned)(((tl.y0 + ty) * P + tl.x0 + tx) * es);
        R h[13];
        h[0] = lds[kLead + Slot<0>::value * N + r];
        h[1] = lds[kLead + Slot<1>::value * N + r];
        h[2] = lds[kLead + Slot<2>::value * N + r];
        h[3] = lds[kLead + Slot<3>::value * N + r];
        h[4] = lds[kLead + Slot<4>::value * N + r];
        h[5] = lds[kLead + Slot<5>::value * N + r];
        h[6] = lds[kLead + Slot<6>::value * N + r];
        h[7] = lds[kLead + Slot<7>::value * N + r];
        h[8] = lds[kLead + Slot<8>::value * N + r];
        h[9] = lds[kLead + Slot<9>::value * N + r];
        h[10] = lds[kLead + Slot<10>::value * N + r];
        h[11] = lds[kLead + Slot<11>::value * N + r];
        h[12] = lds[kLead + Slot<12>::value * N + r];
        if (D.collide) collide(h, D);
#pragma unroll
        for (int i = 0; i < 13; ++i) buffer_store_nt<R>(h[i], out, c, (unsigned)(i * S * es));
    }
}

// ---------------------------------------------------------------------------
// Three steps per launch on a domain periodic on both axes, whole tiles (flag
// 2; with flag 4 the region wraps around the sides).  Phase 1 advances the
// tile and a four-node halo from HBM and keeps population i only over the
// window phase 2 reads (the tile and a two-node halo, shifted by -v_i); phase
// 2 advances the tile and its two-node halo from LDS into registers, then,
// after a barrier, keeps population i over the window phase 3 reads (the tile
// shifted by -v_i) in the same LDS; phase 3 advances the tile and writes HBM.
// Each node's arithmetic is the single-step kernel's.  Node slots past a
// region's end collide nothing, so whole waves with no node in a slot skip it
// (their phase-1 loads stay: they re-read the region's last node).  Tiles of
// up to 1024 (FP32) or 512 (FP64) nodes take one thread per node, with the
// registers of the occupancy the LDS allows (FP32 64x16: two 1024-thread
// workgroups, eight waves per SIMD; FP64 32x16: two 512-thread workgroups).
// Sourced = false: no domain of the launch has a body force or energy source.
template <int TW, int TH>
constexpr int step3_window_lds() { return 2 + 13 * (TW + 4) * (TH + 4); }  // values

template <typename R, int TW, int TH, int NT, bool Sourced>
__device__ __forceinline__ void step3_window_tile(R* lds, const Tile& tl, const R* __restrict__ src,
                                                  R* __restrict__ dst, const Dom<R>* __restrict__ doms) {
    constexpr int W1 = TW + 8, H1 = TH + 8, W2 = TW + 4, H2 = TH + 4;
    constexpr int N1 = W1 * H1, N2 = W2 * H2, N3 = TW * TH;
    constexpr int NI1 = (N1 + NT - 1) / NT, NI2 = (N2 + NT - 1) / NT;
    constexpr int kLead = 2;  // keeps the window index of the population in slot 0 non-negative
    const Dom<R>& D = doms[tl.dom];
    const R* __restrict__ a = src + D.off;
    R* __restrict__ o = dst + D.off;
    const int P = D.pitch, S = D.plane;
    const int tid = threadIdx.x;
    constexpr int es = (int)sizeof(R);
    const __amdgpu_buffer_rsrc_t in = buffer_rsrc(a - (2 * P + 2), (unsigned)((13 * S + 2 * P + 2) * es));
    const bool wraps = tl.flags & 4;

    // Phase 1: region (x0 - 4, y0 - 4) + [0, W1) x [0, H1); all loads issued first.
    R g[NI1][13];
    int l1x[NI1], l1y[NI1];
#pragma unroll
    for (int k = 0; k < NI1; ++k) {
        const int r = min(tid + k * NT, N1 - 1);
        l1x[k] = r % W1;
        l1y[k] = r / W1;
        const int X = tl.x0 - 4 + l1x[k], Y = tl.y0 - 4 + l1y[k];
        if (wraps) {
            int xs[5], ys[5];  // X + 2 - v and Y + 2 - v wrapped once, v = 0..4
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                xs[v] = wrap(X + 2 - v, D.nx);
                ys[v] = wrap(Y + 2 - v, D.ny) * P;
            }
#pragma unroll
            for (int i = 0; i < 13; ++i)
                g[k][i] = buffer_load<R>(in, (unsigned)((ys[kVY[i] + 2] + xs[kVX[i] + 2]) * es),
                                         (unsigned)((i * S + 2 * P + 2) * es));
        } else {
            const unsigned c = (unsigned)((Y * P + X) * es);
#pragma unroll
            for (int i = 0; i < 13; ++i)
                g[k][i] = buffer_load<R>(in, c, (unsigned)((i * S + (2 - kVY[i]) * P + 2 - kVX[i]) * es));
        }
    }
#pragma unroll
    for (int k = 0; k < NI1; ++k) {
        if (tid + k * NT < N1) {
            if (D.collide) collide<R, Sourced>(g[k], D);
            const int lx = l1x[k], ly = l1y[k], base = ly * W2 + lx;
#define LBM13_WINDOW1(I)                                                                                   \
    if ((unsigned)(lx - 2 + kVX[I]) < (unsigned)W2 && (unsigned)(ly - 2 + kVY[I]) < (unsigned)H2)          \
        lds[base + (kLead + Slot<I>::value * N2 + (kVY[I] - 2) * W2 + kVX[I] - 2)] = g[k][I];
            LBM13_WINDOW1(0) LBM13_WINDOW1(1) LBM13_WINDOW1(2) LBM13_WINDOW1(3) LBM13_WINDOW1(4)
            LBM13_WINDOW1(5) LBM13_WINDOW1(6) LBM13_WINDOW1(7) LBM13_WINDOW1(8) LBM13_WINDOW1(9)
            LBM13_WINDOW1(10) LBM13_WINDOW1(11) LBM13_WINDOW1(12)
#undef LBM13_WINDOW1
        }
    }
    __syncthreads();

    // Phase 2: region (x0 - 2, y0 - 2) + [0, W2) x [0, H2), node r reads index r of every slot.
    R h[NI2][13];
#pragma unroll
    for (int k = 0; k < NI2; ++k) {
        const int r = tid + k * NT;
        if (r < N2) {
#pragma unroll
            for (int i = 0; i < 13; ++i) h[k][i] = lds[kLead + ((i + 3) % 13) * N2 + r];
            if (D.collide) collide<R, Sourced>(h[k], D);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NI2; ++k) {
        const int r = tid + k * NT;
        if (r < N2) {
            const int lx = r % W2, ly = r / W2, base = ly * TW + lx;
#define LBM13_WINDOW2(I)                                                                                   \
    if ((unsigned)(lx - 2 + kVX[I]) < (unsigned)TW && (unsigned)(ly - 2 + kVY[I]) < (unsigned)TH)          \
        lds[base + (kLead + Slot<I>::value * N3 + (kVY[I] - 2) * TW + kVX[I] - 2)] = h[k][I];
            LBM13_WINDOW2(0) LBM13_WINDOW2(1) LBM13_WINDOW2(2) LBM13_WINDOW2(3) LBM13_WINDOW2(4)
            LBM13_WINDOW2(5) LBM13_WINDOW2(6) LBM13_WINDOW2(7) LBM13_WINDOW2(8) LBM13_WINDOW2(9)
            LBM13_WINDOW2(10) LBM13_WINDOW2(11) LBM13_WINDOW2(12)
#undef LBM13_WINDOW2
        }
    }
    __syncthreads();

    // Phase 3: the tile, node r reads index r of every slot.
    const __amdgpu_buffer_rsrc_t out = buffer_rsrc(o, (unsigned)(13 * S * es));
    for (int r = tid; r < N3; r += NT) {
        const int tx = r % TW, ty = r / TW;
        const unsigned c = (unsigned)(((tl.y0 + ty) * P + tl.x0 + tx) * es);
        R q[13];
#pragma unroll
        for (int i = 0; i < 13; ++i) q[i] = lds[kLead + ((i + 3) % 13) * N3 + r];
        if (D.collide) collide<R, Sourced>(q, D);
#pragma unroll
        for (int i = 0; i < 13; ++i) buffer_store_nt<R>(q[i], out, c, (unsigned)(i * S * es));
    }
}

template <typename R, int TW, int TH, int NT, bool Sourced>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(
    lds_waves_per_eu(step3_window_lds<TW, TH>() * (int)sizeof(R), NT)))) void step3_kernel(
    const R* __restrict__ src, R* __restrict__ dst, const Dom<R>* __restrict__ doms, const Tile* __restrict__ tiles,
    int ntiles) {
    __shared__ R lds[step3_window_lds<TW, TH>()];
    const Tile tl = tiles[xcd_tile(blockIdx.x, ntiles)];
    step3_window_tile<R, TW, TH, NT, Sourced>(lds, tl, src, dst, doms);
}


// ---------------------------------------------------------------------------
// The nodes a level of the general multi-step kernel computes: the slots of
// its region inside the domain (on a walled axis) and within reach of the
// tile's nodes (a ragged tile needs fewer columns or rows), numbered row by row
// over that window, so that waves past its end skip the level.  Slot r of the
// window is region slot (x0 + r mod w, y0 + r div w); the quotient is taken in
// FP32 as (r + 1/2) / w, exact for r < 4096 and w <= 80 (the distance of
// (r + 1/2) / w from an integer, 1 / (2w), exceeds the rounding error).
struct LevelWindow {
    int x0, y0, w, h, n;
    bool col;   // numbered column by column instead (the general kernel's second
                // level in tiles at an x wall: a wave then takes a few columns,
                // so the nodes next to the wall fall into one or two waves)
    float inv;  // 1 / w, or 1 / h by columns
    __device__ __forceinline__ void slot(int r, int& lx, int& ly) const {
        const int q = (int)(((float)r + 0.5f) * inv), m = r - q * (col ? h : w);
        lx = x0 + (col ? q : m);
        ly = y0 + (col ? m : q);
    }
};

// Window of a level whose region starts at (ox, oy) and whose tile's nodes
// reach ex columns and ey rows of it.
template <typename R>
__device__ __forceinline__ LevelWindow level_window(const Dom<R>& D, int ox, int oy, int ex, int ey, bool col = false) {
    const int xa = D.xper ? 0 : max(0, -ox), xb = D.xper ? ex : min(ex, D.nx - ox);
    const int ya = D.yper ? 0 : max(0, -oy), yb = D.yper ? ey : min(ey, D.ny - oy);
    return LevelWindow{xa, ya, xb - xa, yb - ya, (xb - xa) * (yb - ya), col,
                       col ? 1.0f / (float)(yb - ya) : 1.0f / (float)(xb - xa)};
}

// ---------------------------------------------------------------------------
// Three steps per launch on the other tiles: tiles that reach a wall (their
// region, a tile plus four nodes on each side, or its gathers), a ragged
// domain edge or a periodic axis shorter than the region.  Each level's
// result is kept in LDS for the next (WallWindows, below): phase 1 advances
// the (TW + 8) x (TH + 8) region from HBM (wall fix-ups from the side array of
// step t), phase 2 the (TW + 4) x (TH + 4) region from LDS into
// registers (wall fix-ups from the layer values phase 1 kept), then, after a
// barrier, keeps it and its layer values for phase 3; phase 3 advances the
// tile, writes HBM and the side array of step t + 3.  Each level computes only
// the window of its region inside the domain and within reach of the tile's
// nodes (LevelWindow); slots beyond a wall are never written.  A level keeps
// population i in LDS over the slots the next level reads (WallWindows), and
// phases 2 and 3 read every node's sources with the plain stencil, then
// replace the links from beyond a wall (wall_fixups): those reads land in the
// unwritten slots and are discarded.  Each node's arithmetic is the
// single-step kernel's.
//
// WallWindows<W, H, Last>: population i of a level kept over the W x H region
// of the level that reads it, shifted by -v_i, plus the slots past its edges
// that the wall fix-ups read for reflected populations (fix_link, sec. 7: the
// tangential coordinate kept, the normal one mirrored in the wall).  Tiles lie
// on a grid of whole tiles from the domain's origin, so the second level's
// region starts two nodes before a West or South wall; a tile can end one,
// two or three nodes before an East or North wall, whose reflected speed-2
// sources then lie up to three slots past the region (one for speed 1); a
// diagonal reflected at a wall moves one slot along it.  The third level's
// region is the tile itself, whose low edge can be the West or South wall, and
// which can end one to three nodes before the East or North wall: population
// i then needs |v_i| slots on each side v_i points to (three for the speed-2
// populations on the high sides, as above).  Slot u (relative to the reading
// level's origin) of population i is at base(i) + (u_y + ylo(i)) w(i) + u_x +
// xlo(i), w(i) the window's width, made odd when Odd.
template <int W, int H, bool Last, bool Odd = false>
struct WallWindows {
    static constexpr int xhi(int i) { return kVX[i] > 0 ? (kVX[i] == 2 ? 3 : 1) : 0; }
    static constexpr int yhi(int i) { return kVY[i] > 0 ? (kVY[i] == 2 ? 3 : 1) : 0; }
    static constexpr int xlo(int i) { return kVX[i] < 0 ? (Last ? -kVX[i] : (kVY[i] != 0 ? 1 : 0)) : 0; }
    static constexpr int ylo(int i) { return kVY[i] < 0 ? (Last ? -kVY[i] : (kVX[i] != 0 ? 1 : 0)) : 0; }
    static constexpr int w(int i) { return (W + xlo(i) + xhi(i)) | (Odd ? 1 : 0); }  // row pitch
    static constexpr int h(int i) { return H + ylo(i) + yhi(i); }
    static constexpr int base(int i) {
        int b = 0;
        for (int j = 0; j < i; ++j) b += w(j) * h(j);
        return b;
    }
    static constexpr int total() { return base(13); }
    // the slot of population i that the reading level's node u pulls (or the
    // fix-ups read), and whether population i of a node keeps slot u
    static constexpr int at(int i, int ux, int uy) { return base(i) + (uy + ylo(i)) * w(i) + ux + xlo(i); }
    static constexpr bool keeps(int i, int ux, int uy) {
        return ux >= -xlo(i) && ux < W + xhi(i) && uy >= -ylo(i) && uy < H + yhi(i);
    }
};

// A level's populations in its WallWindows, read by absolute coordinates (of
// the producing node) for the fix-ups of the level whose region starts at
// (ox, oy).
template <typename R, int W, int H, bool Last, bool Odd>
struct WinSrc {
    const R* l;
    int ox, oy;
    __device__ __forceinline__ R get(int i, int X, int Y) const {
        return l[WallWindows<W, H, Last, Odd>::at(i, X - ox + kVX[i], Y - oy + kVY[i])];
    }
};

// LDS of the general three-step kernel, in values: the windows of the second
// or third level (the larger) and the wall-layer records xs, ys.
template <int TW, int TH, bool Odd>
constexpr int step3_wall_lds_of() {
    return (WallWindows<TW + 4, TH + 4, false, Odd>::total() > WallWindows<TW, TH, true, Odd>::total()
                ? WallWindows<TW + 4, TH + 4, false, Odd>::total()
                : WallWindows<TW, TH, true, Odd>::total()) +
           6 * (TW + TH + 16);
}
// Odd row pitches, so that the column-numbered second level reads LDS free of
// bank conflicts, where they cost no occupancy (not for FP32 32x16, whose
// even-pitched windows just fit four workgroups per CU).
template <typename R, int TW, int TH, int NT>
constexpr bool step3_wall_odd() {
    return lds_waves_per_eu(step3_wall_lds_of<TW, TH, true>() * (int)sizeof(R), NT) ==
           lds_waves_per_eu(step3_wall_lds_of<TW, TH, false>() * (int)sizeof(R), NT);
}
template <typename R, int TW, int TH, int NT>
constexpr int step3_wall_lds() { return step3_wall_lds_of<TW, TH, step3_wall_odd<R, TW, TH, NT>()>(); }

template <typename R, int TW, int TH, int NT>
__device__ __forceinline__ void step3_wall_tile(R* lds, const Tile& tl, const R* __restrict__ src,
                                                R* __restrict__ dst, const Dom<R>* __restrict__ doms,
                                                R* __restrict__ side, int from) {
    constexpr int W1 = TW + 8, H1 = TH + 8, W2 = TW + 4, H2 = TH + 4;
    constexpr int N1 = W1 * H1, N2 = W2 * H2;
    static_assert(W1 <= 80 && H1 <= 80 && ((N1 + NT - 1) / NT) * NT <= 4096, "LevelWindow's quotient range");
    constexpr int NI1 = (N1 + NT - 1) / NT, NI2 = (N2 + NT - 1) / NT;
    constexpr bool Odd = step3_wall_odd<R, TW, TH, NT>();
    using Win2 = WallWindows<W2, H2, false, Odd>;  // the first level's populations, read by the second
    using Win3 = WallWindows<TW, TH, true, Odd>;   // the second level's, read by the tile
    constexpr int NW = Win2::total() > Win3::total() ? Win2::total() : Win3::total();
    R* xs = lds + NW;         // [2][H1][3]
    R* ys = xs + 2 * H1 * 3;  // [2][W1][3]
    const Dom<R>& D = doms[tl.dom];
    const R* __restrict__ a = src + D.off;
    R* __restrict__ o = dst + D.off;
    const int o1x = tl.x0 - 4, o1y = tl.y0 - 4, o2x = tl.x0 - 2, o2y = tl.y0 - 2;
    const int tid = threadIdx.x;

    // Phase 1: t -> t + 1 over the first level, gathers of all a thread's nodes
    // issued before the first collision.  The window lies inside the domain on
    // a walled axis, so no coordinate needs a clamp.
    const GlobalSrc<R> G{a, D.plane, D.pitch, D.nx, D.ny, D.xper, D.yper};
    const GlobalSide<R> GS{side, from};
    const bool walls1 =
        (!D.xper && (o1x < 2 || o1x + W1 > D.nx - 2)) || (!D.yper && (o1y < 2 || o1y + H1 > D.ny - 2));
    const int tw3 = min(TW, D.nx - tl.x0), th3 = min(TH, D.ny - tl.y0);  // the tile's nodes
    const LevelWindow w1 = level_window(D, o1x, o1y, tw3 + 8, th3 + 8);
    R g[NI1][13];
    int X1[NI1], Y1[NI1], l1x[NI1], l1y[NI1];
    bool v1[NI1];
#pragma unroll
    for (int k = 0; k < NI1; ++k) {
        w1.slot(min(tid + k * NT, w1.n - 1), l1x[k], l1y[k]);
        int X = o1x + l1x[k], Y = o1y + l1y[k];
        // a region wraps at most once around an axis at least as long as itself
        if (D.xper) X = D.nx >= W1 ? wrap(X, D.nx) : pmod(X, D.nx);
        if (D.yper) Y = D.ny >= H1 ? wrap(Y, D.ny) : pmod(Y, D.ny);
        X1[k] = X;
        Y1[k] = Y;
        v1[k] = tid + k * NT < w1.n;
        if (!v1[k]) continue;
        if (walls1) gather_wall(G, GS, D, X, Y, g[k]);
        else gather_bulk(a, D, X, Y, g[k]);
    }
#pragma unroll
    for (int k = 0; k < NI1; ++k) {
        if (!v1[k]) continue;
        const int lx = l1x[k], ly = l1y[k];
        if (D.collide) collide(g[k], D);
#pragma unroll
        for (int i = 0; i < 13; ++i) {
            const int ux = lx - 2 + kVX[i], uy = ly - 2 + kVY[i];  // the second-level slot that pulls it
            if (Win2::keeps(i, ux, uy)) lds[Win2::at(i, ux, uy)] = g[k][i];
        }
        record_region_layers<R, W1, H1>(xs, ys, D, X1[k], Y1[k], lx, ly, g[k]);
    }
    __syncthreads();

    // Phase 2: t + 1 -> t + 2 over the second level, gathers from the first
    // (coordinates unwrapped on periodic axes, as the region stores them).
    // The plain stencil's reads are those of gather_wall for every link it
    // keeps, so the result is the same.
    const WinSrc<R, W2, H2, false, Odd> L1{lds, o2x, o2y};
    const LdsSide<R, W1, H1> S1{xs, ys, o1x, o1y};
    const bool walls2 =
        (!D.xper && (o2x < 2 || o2x + W2 > D.nx - 2)) || (!D.yper && (o2y < 2 || o2y + H2 > D.ny - 2));
    const bool xwall2 = Odd && !D.xper && (o2x < 2 || o2x + W2 > D.nx - 2);
    const LevelWindow w2 = level_window(D, o2x, o2y, tw3 + 4, th3 + 4, xwall2);
    R h[NI2][13];
    int l2x[NI2], l2y[NI2];
    bool v2[NI2];
#pragma unroll
    for (int k = 0; k < NI2; ++k) {
        w2.slot(min(tid + k * NT, w2.n - 1), l2x[k], l2y[k]);
        const int lx = l2x[k], ly = l2y[k], X = o2x + lx, Y = o2y + ly;
        v2[k] = tid + k * NT < w2.n;
        if (!v2[k]) continue;
#pragma unroll
        for (int i = 0; i < 13; ++i) h[k][i] = lds[Win2::at(i, lx, ly)];
        if (walls2) wall_fixups(L1, S1, D, X, Y, h[k]);
        if (D.collide) collide(h[k], D);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NI2; ++k) {
        if (!v2[k]) continue;
        const int lx = l2x[k], ly = l2y[k];
#pragma unroll
        for (int i = 0; i < 13; ++i) {
            const int ux = lx - 2 + kVX[i], uy = ly - 2 + kVY[i];  // the tile slot that pulls it
            if (Win3::keeps(i, ux, uy)) lds[Win3::at(i, ux, uy)] = h[k][i];
        }
        record_region_layers<R, W2, H2>(xs, ys, D, o2x + lx, o2y + ly, lx, ly, h[k]);
    }
    __syncthreads();

    // Phase 3: t + 2 -> t + 3 over the tile, gathers from the second level.
    const WinSrc<R, TW, TH, true, Odd> L2{lds, tl.x0, tl.y0};
    const LdsSide<R, W2, H2> S2{xs, ys, o2x, o2y};
    const bool walls3 = (!D.xper && (tl.x0 < 2 || tl.x0 + TW > D.nx - 2)) ||
                        (!D.yper && (tl.y0 < 2 || tl.y0 + TH > D.ny - 2));
    const LevelWindow w3{2, 2, tw3, th3, tw3 * th3, false, 1.0f / (float)tw3};
    for (int r = tid; r < w3.n; r += NT) {
        int lx, ly;
        w3.slot(r, lx, ly);
        const int X = o2x + lx, Y = o2y + ly;
        R q[13];
#pragma unroll
        for (int i = 0; i < 13; ++i) q[i] = lds[Win3::at(i, lx - 2, ly - 2)];
        if (walls3) wall_fixups(L2, S2, D, X, Y, q);
        if (D.collide) collide(q, D);
        store_node(o, D.plane, Y * D.pitch + X, q);
        record_wall_layers(side, D, 1 - from, X, Y, q);
    }
}

template <typename R, int TW, int TH, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(
    lds_waves_per_eu(step3_wall_lds<R, TW, TH, NT>() * (int)sizeof(R), NT)))) void step3_wall_kernel(
    const R* __restrict__ src, R* __restrict__ dst, const Dom<R>* __restrict__ doms, const Tile* __restrict__ tiles,
    int ntiles, R* __restrict__ side, int from) {
    __shared__ R lds[step3_wall_lds<R, TW, TH, NT>()];
    const Tile tl = tiles[xcd_tile(blockIdx.x, ntiles)];
    step3_wall_tile<R, TW, TH, NT>(lds, tl, src, dst, doms, side, from);
}

// Three steps per launch over a tile table in its spatial order, each tile on
// the window path (flag 2: an interior tile) or the general path in the one
// launch: neighbouring tiles run close together in time, so the halo rows they
// share are read once, and no second kernel runs beside the first.  The LDS is
// the general path's (the larger); the window path uses its start.
template <typename R, int TW, int TH, int NT, bool Sourced>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(
    lds_waves_per_eu(step3_wall_lds<R, TW, TH, NT>() * (int)sizeof(R), NT)))) void step3_mixed_kernel(
    const R* __restrict__ src, R* __restrict__ dst, const Dom<R>* __restrict__ doms, const Tile* __restrict__ tiles,
    int ntiles, R* __restrict__ side, int from) {
    static_assert(step3_wall_lds<R, TW, TH, NT>() >= step3_window_lds<TW, TH>(), "the general path's LDS is the larger");
    __shared__ R lds[step3_wall_lds<R, TW, TH, NT>()];
    const Tile tl = tiles[xcd_tile(blockIdx.x, ntiles)];
    if (tl.flags & 2) step3_window_tile<R, TW, TH, NT, Sourced>(lds, tl, src, dst, doms);
    else step3_wall_tile<R, TW, TH, NT>(lds, tl, src, dst, doms, side, from);
}


// ---------------------------------------------------------------------------
// Initial state: g = f^eq(rho, j = rho u, E = T + 13/2 |u|^2) - f^rest, built in
// FP64 from the equilibrium moments (eq d2q13-moments-equil) and M^T D^-1, then
// one collision in the working precision.
template <typename R>
__global__ __launch_bounds__(256) void init_kernel(R* __restrict__ dst, const Dom<R>* __restrict__ doms, int d,
                                                   const double* __restrict__ rho_in,
                                                   const double* __restrict__ ux_in,
                                                   const double* __restrict__ uy_in,
                                                   const double* __restrict__ T_in,
                                                   const double* __restrict__ coef /* c_er c_eE c_vr c_vE a1 h1 k1 a2 h2 k2 */) {
    const Dom<R>& D = doms[d];
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= D.nx || y >= D.ny) return;
    const int n = y * D.nx + x;
    const double rho = rho_in[n], ux = ux_in[n], uy = uy_in[n];
    const double E = T_in[n] + 6.5 * (ux * ux + uy * uy);
    const double rp = rho - 1.0, Ep = E - D.E0;
    const double jx = rho * ux, jy = rho * uy;
    double m[13];
    m[0] = rp;
    m[1] = Ep;
    m[2] = coef[0] * rp + coef[1] * Ep;
    m[3] = coef[2] * rp + coef[3] * Ep;
    m[4] = jx;
    m[5] = jy;
    const double fq = coef[4] + coef[5] * rp + coef[6] * Ep;
    const double fr = coef[7] + coef[8] * rp + coef[9] * Ep;
    m[6] = jx * fq;
    m[7] = jy * fq;
    m[8] = jx * fr;
    m[9] = jy * fr;
    m[10] = (jx * jx - jy * jy) / rho;
    m[11] = jx * jy / rho;
    m[12] = 0.0;
    R g[13];
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 13; ++k) s += double(c_M[k][i]) * m[k] / double(c_D[k]);
        g[i] = R(s);
    }
    if (D.collide) collide(g, D);
    R* __restrict__ o = dst + D.off;
#pragma unroll
    for (int i = 0; i < 13; ++i) o[i * D.plane + y * D.pitch + x] = g[i];
}

// ---------------------------------------------------------------------------
// Read-back at time t from the kept f*(t): rho = 1 + sum g, E = E0 + sum M_E g - Q_E,
// j = j* - F, u = (j + F/2)/rho = (j* - F/2)/rho, T = E - 13/2 |u|^2 (sec. 7).
template <typename R>
__device__ __forceinline__ void node_macro(const R* __restrict__ a, const Dom<R>& D, int c, double& rho, double& ux,
                                           double& uy, double& T) {
    double r = 0.0, e = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        const double v = double(a[i * D.plane + c]);
        r += v;
        e += double(c_M[1][i]) * v;
        jx += double(c_vx[i]) * v;
        jy += double(c_vy[i]) * v;
    }
    const double Fx = D.F0x_d + D.gx_d * r, Fy = D.F0y_d + D.gy_d * r;
    rho = 1.0 + r;
    ux = (jx - 0.5 * Fx) / rho;
    uy = (jy - 0.5 * Fy) / rho;
    T = D.E0 + (e - D.QE_d) - 6.5 * (ux * ux + uy * uy);
}

template <typename R>
__global__ __launch_bounds__(256) void moments_kernel(const R* __restrict__ src, const Dom<R>* __restrict__ doms,
                                                      int d, double* __restrict__ rho_out,
                                                      double* __restrict__ ux_out, double* __restrict__ uy_out,
                                                      double* __restrict__ T_out) {
    const Dom<R>& D = doms[d];
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= D.nx || y >= D.ny) return;
    double rho, ux, uy, T;
    node_macro(src + D.off, D, y * D.pitch + x, rho, ux, uy, T);
    const int n = y * D.nx + x;
    if (rho_out) rho_out[n] = rho;
    if (ux_out) ux_out[n] = ux;
    if (uy_out) uy_out[n] = uy;
    if (T_out) T_out[n] = T;
}

// State copy-out (absolute FP64 f*) and copy-in.
template <typename R>
__global__ __launch_bounds__(256) void get_state_kernel(const R* __restrict__ src, const Dom<R>* __restrict__ doms,
                                                        int d, double* __restrict__ out) {
    const Dom<R>& D = doms[d];
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= D.nx || y >= D.ny) return;
    const long long n = (long long)D.nx * D.ny;
#pragma unroll
    for (int i = 0; i < 13; ++i)
        out[i * n + y * D.nx + x] = double(src[D.off + i * D.plane + y * D.pitch + x]) + D.frest[c_cls[i]];
}

template <typename R>
__global__ __launch_bounds__(256) void set_state_kernel(R* __restrict__ dst, const Dom<R>* __restrict__ doms, int d,
                                                        const double* __restrict__ in) {
    const Dom<R>& D = doms[d];
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= D.nx || y >= D.ny) return;
    const long long n = (long long)D.nx * D.ny;
#pragma unroll
    for (int i = 0; i < 13; ++i)
        dst[D.off + i * D.plane + y * D.pitch + x] = R(in[i * n + y * D.nx + x] - D.frest[c_cls[i]]);
}

// ---------------------------------------------------------------------------
// Diagnostics, pass 1: one partial record per tile (FP64), in the order of the
// domain-ordered tile table; pass 2 reduces each domain's records in order, so
// results do not depend on scheduling.
//   part[0..3] sum rho', jx, jy, E'     part[4] heat flux (face crossing, see header)
//   part[5] max |u|  part[6] max |u(x) + u(xbar)|  part[7] non-finite count
//   part[8] min rho
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

template <typename R, int TX, int RPT>
__global__ __launch_bounds__(256) void diag_partial_kernel(const R* __restrict__ src, const Dom<R>* __restrict__ doms,
                                                           const Tile* __restrict__ tiles,
                                                           double* __restrict__ part) {
    constexpr int TYB = 256 / TX;
    const int t = blockIdx.x;
    const Tile tl = tiles[t];
    const Dom<R>& D = doms[tl.dom];
    const R* __restrict__ a = src + D.off;
    double acc[5] = {0, 0, 0, 0, 0};
    double umax = 0.0, asym = 0.0, nonfin = 0.0, rmin = INFINITY;
    const int flo = D.xper ? 0 : 1, fhi = D.xper ? D.nx - 1 : D.nx - 3;
    const int x = tl.x0 + threadIdx.x;
    for (int r = 0; r < RPT; ++r) {
        const int y = tl.y0 + threadIdx.y + r * TYB;
        if (x >= D.nx || y >= D.ny) continue;
        const int c = y * D.pitch + x;
        double rp = 0, e = 0, jx = 0, jy = 0, heat = 0;
#pragma unroll
        for (int i = 0; i < 13; ++i) {
            const R vr = a[i * D.plane + c];
            if (!isfinite(double(vr))) nonfin += 1.0;
            const double v = double(vr);
            rp += v;
            e += double(c_M[1][i]) * v;
            jx += double(c_vx[i]) * v;
            jy += double(c_vy[i]) * v;
            const int vx = c_vx[i];
            int cnt = 0;
            if (D.xper) {
                cnt = vx;
            } else if (vx > 0) {
                for (int xf = x; xf < x + vx; ++xf) cnt += (xf >= flo && xf <= fhi);
            } else if (vx < 0) {
                for (int xf = x + vx; xf < x; ++xf) cnt -= (xf >= flo && xf <= fhi);
            }
            heat += (double(c_M[1][i]) - D.B) * double(cnt) * (v + D.frest[c_cls[i]]);
        }
        const double Fx = D.F0x_d + D.gx_d * rp, Fy = D.F0y_d + D.gy_d * rp;
        acc[0] += rp;
        acc[1] += jx - Fx;
        acc[2] += jy - Fy;
        acc[3] += e - D.QE_d;
        acc[4] += heat;
        const double rho = 1.0 + rp;
        const double ux = (jx - 0.5 * Fx) / rho, uy = (jy - 0.5 * Fy) / rho;
        umax = fmax(umax, sqrt(ux * ux + uy * uy));
        rmin = fmin(rmin, rho);
        double rb, uxb, uyb, Tb;
        node_macro(a, D, (D.ny - 1 - y) * D.pitch + (D.nx - 1 - x), rb, uxb, uyb, Tb);
        const double sx = ux + uxb, sy = uy + uyb;
        asym = fmax(asym, sqrt(sx * sx + sy * sy));
    }
    __shared__ double red[4][9];
    const int lane = (threadIdx.y * TX + threadIdx.x) & 63;
    const int wave = (threadIdx.y * TX + threadIdx.x) >> 6;
    double vals[9];
    for (int k = 0; k < 5; ++k) vals[k] = wave_sum(acc[k]);
    vals[5] = wave_max(umax);
    vals[6] = wave_max(asym);
    vals[7] = wave_sum(nonfin);
    vals[8] = wave_min(rmin);
    if (lane == 0)
        for (int k = 0; k < 9; ++k) red[wave][k] = vals[k];
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        double out[9];
        for (int k = 0; k < 9; ++k) out[k] = red[0][k];
        for (int w = 1; w < 4; ++w) {
            for (int k = 0; k < 5; ++k) out[k] += red[w][k];
            out[5] = fmax(out[5], red[w][5]);
            out[6] = fmax(out[6], red[w][6]);
            out[7] += red[w][7];
            out[8] = fmin(out[8], red[w][8]);
        }
        for (int k = 0; k < 9; ++k) part[t * kDiagPartials + k] = out[k];
    }
}

// Pass 2: one 256-thread block per domain.  Thread k combines records
// k, k + 256, ... in that order, then a fixed-shape tree in LDS combines the
// threads, so the result is independent of scheduling.
template <typename R>
__global__ __launch_bounds__(256) void diag_final_kernel(const Dom<R>* __restrict__ doms,
                                                         const double* __restrict__ part,
                                                         double* __restrict__ out) {
    const int d = blockIdx.x;
    const Dom<R>& D = doms[d];
    const int k = threadIdx.x;
    double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, INFINITY};
    for (int t = D.tile0 + k; t < D.tile0 + D.ntiles; t += 256) {
        const double* p = part + t * kDiagPartials;
        for (int j = 0; j < 5; ++j) v[j] += p[j];
        v[5] = fmax(v[5], p[5]);
        v[6] = fmax(v[6], p[6]);
        v[7] += p[7];
        v[8] = fmin(v[8], p[8]);
    }
    __shared__ double red[9][256];
    for (int j = 0; j < 9; ++j) red[j][k] = v[j];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (k < h) {
            for (int j = 0; j < 5; ++j) red[j][k] += red[j][k + h];
            red[5][k] = fmax(red[5][k], red[5][k + h]);
            red[6][k] = fmax(red[6][k], red[6][k + h]);
            red[7][k] += red[7][k + h];
            red[8][k] = fmin(red[8][k], red[8][k + h]);
        }
        __syncthreads();
    }
    if (k != 0) return;
    const double N = double(D.nx) * double(D.ny);
    const int faces = D.xper ? D.nx : D.nx - 3;
    double* o = out + d * kDiagOut;
    const double umax = red[5][0];
    o[0] = N + red[0][0];
    o[1] = red[1][0];
    o[2] = red[2][0];
    o[3] = N * D.E0 + red[3][0];
    o[4] = red[4][0];
    o[5] = (faces > 0) ? red[4][0] / (double(faces) * D.ny) * D.nu_scale : 0.0;
    o[6] = umax;
    o[7] = red[6][0];
    o[8] = umax > 0.0 ? red[6][0] / umax : 0.0;
    o[9] = red[7][0];
    o[10] = red[8][0];
    for (int j = 11; j < kDiagOut; ++j) o[j] = 0.0;  // 11..14: wall_flux_kernel
}

// Energy and mass exchanged with the walls in the next step (sec. 7 walls): an
// incoming link (x, i) whose source x - v_i lies beyond wall w brings its
// bounce-back or anti-bounce-back value f_i(x, t+1); an outgoing link (x, j)
// whose target x + v_j lies beyond w takes f*_j(x, t); a link beyond an x
// wall and a y wall counts for the x wall.  Incoming and outgoing links pair
// up with equal |v|, so rest populations cancel and deviations suffice.  One
// block per domain over the nodes within two nodes of a wall; fixed-shape
// reduction.  Writes Nu at the West and East walls (energy less B times mass,
// per unit wall length, over kappa_E dT / nx), the total energy and the total
// mass taken in.
template <typename R>
__device__ __forceinline__ int beyond_wall(const Dom<R>& D, int X, int Y) {
    if (!D.xper && X < 0) return 0;
    if (!D.xper && X >= D.nx) return 1;
    if (!D.yper && Y < 0) return 2;
    if (!D.yper && Y >= D.ny) return 3;
    return -1;
}

template <typename R>
__global__ __launch_bounds__(256) void wall_flux_kernel(const R* __restrict__ src, const Dom<R>* __restrict__ doms,
                                                        R* __restrict__ side, int buf, double* __restrict__ out) {
    const int d = blockIdx.x;
    const Dom<R>& D = doms[d];
    const R* __restrict__ a = src + D.off;
    const GlobalSrc<R> G{a, D.plane, D.pitch, D.nx, D.ny, D.xper, D.yper};
    const GlobalSide<R> GS{side, buf};
    // columns within two nodes of an x wall (every row), then the rows within
    // two nodes of a y wall outside those columns
    const int ncx = D.xper ? 0 : min(D.nx, 4), nry = D.yper ? 0 : min(D.ny, 4);
    const int xlo = D.xper ? 0 : min(2, D.nx), xhi = D.xper ? D.nx : max(D.nx - 2, xlo);
    const int n1 = ncx * D.ny, n2 = nry * (xhi - xlo);
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // energy W E S N, mass W E S N
    for (int k = threadIdx.x; k < n1 + n2; k += 256) {
        int X, Y;
        if (k < n1) {
            const int cx = k % ncx;
            X = (D.nx >= 4 && cx >= 2) ? D.nx - 4 + cx : cx;
            Y = k / ncx;
        } else {
            const int kk = k - n1, ry = kk % nry;
            X = xlo + kk / nry;
            Y = (D.ny >= 4 && ry >= 2) ? D.ny - 4 + ry : ry;
        }
        R g[13];
        gather_wall(G, GS, D, X, Y, g);
        const int c = Y * D.pitch + X;
#pragma unroll
        for (int i = 0; i < 13; ++i) {
            const int wi = beyond_wall(D, X - kVX[i], Y - kVY[i]);
            if (wi >= 0) {
                acc[wi] += double(kM[1][i]) * double(g[i]);
                acc[4 + wi] += double(g[i]);
            }
            const int wo = beyond_wall(D, X + kVX[i], Y + kVY[i]);
            if (wo >= 0) {
                const double v = double(a[i * D.plane + c]);
                acc[wo] -= double(kM[1][i]) * v;
                acc[4 + wo] -= v;
            }
        }
    }
    __shared__ double red[8][256];
    const int k = threadIdx.x;
    for (int j = 0; j < 8; ++j) red[j][k] = acc[j];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (k < h)
            for (int j = 0; j < 8; ++j) red[j][k] += red[j][k + h];
        __syncthreads();
    }
    if (k != 0) return;
    double* o = out + d * kDiagOut;
    const double scale = D.xper ? 0.0 : D.nu_scale / double(D.ny);
    o[11] = (red[0][0] - D.B * red[4][0]) * scale;
    o[12] = -(red[1][0] - D.B * red[5][0]) * scale;
    o[13] = red[0][0] + red[1][0] + red[2][0] + red[3][0];
    o[14] = red[4][0] + red[5][0] + red[6][0] + red[7][0];
}

// Fourier projection of rho, u_x, u_y and E of one domain (sec. 6 aggregates):
// sum_{x,y} q exp(-2 pi i (kx x/nx + ky y/ny)), FP64 accumulation.  Pass 1: one
// block per tile of the domain (its range of the all-tiles table) writes eight
// partial sums; pass 2: one block combines them in a fixed order.
template <typename R>
__global__ __launch_bounds__(256) void fourier_partial_kernel(const R* __restrict__ src,
                                                              const Dom<R>* __restrict__ doms, int d,
                                                              const Tile* __restrict__ tiles, int tile_x,
                                                              int tile_y, int kx, int ky, double* __restrict__ part) {
    const Dom<R>& D = doms[d];
    const Tile tl = tiles[D.tile0 + blockIdx.x];
    const R* __restrict__ a = src + D.off;
    const long long per = (long long)D.nx * D.ny;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int r = threadIdx.x; r < tile_x * tile_y; r += 256) {
        const int x = tl.x0 + r % tile_x, y = tl.y0 + r / tile_x;
        if (x >= D.nx || y >= D.ny) continue;
        const int c = y * D.pitch + x;
        double rp = 0, e = 0, jx = 0, jy = 0;
#pragma unroll
        for (int i = 0; i < 13; ++i) {
            const double v = double(a[i * D.plane + c]);
            rp += v;
            e += double(kM[1][i]) * v;
            jx += double(kVX[i]) * v;
            jy += double(kVY[i]) * v;
        }
        const double Fx = D.F0x_d + D.gx_d * rp, Fy = D.F0y_d + D.gy_d * rp;
        const double rho = 1.0 + rp;
        const double q[4] = {rho, (jx - 0.5 * Fx) / rho, (jy - 0.5 * Fy) / rho, D.E0 + e - D.QE_d};
        // phase 2 pi m / (nx ny) with m = (kx x ny + ky y nx) mod (nx ny), exact in integers
        long long m = ((long long)kx * x * D.ny + (long long)ky * y * D.nx) % per;
        if (m < 0) m += per;
        double sn, cs;
        sincospi(2.0 * double(m) / double(per), &sn, &cs);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[2 * j] += q[j] * cs;
            acc[2 * j + 1] -= q[j] * sn;
        }
    }
    __shared__ double red[8][256];
    const int k = threadIdx.x;
    for (int j = 0; j < 8; ++j) red[j][k] = acc[j];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (k < h)
            for (int j = 0; j < 8; ++j) red[j][k] += red[j][k + h];
        __syncthreads();
    }
    if (k == 0)
        for (int j = 0; j < 8; ++j) part[blockIdx.x * kDiagPartials + j] = red[j][0];
}

template <typename R>
__global__ __launch_bounds__(256) void fourier_final_kernel(const Dom<R>* __restrict__ doms, int d,
                                                            const double* __restrict__ part,
                                                            double* __restrict__ out) {
    const int n = doms[d].ntiles, k = threadIdx.x;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int t = k; t < n; t += 256)
        for (int j = 0; j < 8; ++j) acc[j] += part[t * kDiagPartials + j];
    __shared__ double red[8][256];
    for (int j = 0; j < 8; ++j) red[j][k] = acc[j];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (k < h)
            for (int j = 0; j < 8; ++j) red[j][k] += red[j][k + h];
        __syncthreads();
    }
    if (k == 0)
        for (int j = 0; j < 8; ++j) out[j] = red[j][0];
}

// ---------------------------------------------------------------------------
// Host launchers (called from lbm13_capi.cpp).

template <typename R, int TX, int RPT>
static hipError_t launch_step_t(const R* src, R* dst, const Dom<R>* doms, const Tile* bulk, int nbulk,
                                const Tile* edge, int nedge, R* side, int from, hipStream_t s) {
    constexpr dim3 blk(TX, 256 / TX);
    if (nbulk > 0) step_kernel<R, TX, RPT, false><<<nbulk, blk, 0, s>>>(src, dst, doms, bulk, nbulk, side, from);
    if (nedge > 0) step_kernel<R, TX, RPT, true><<<nedge, blk, 0, s>>>(src, dst, doms, edge, nedge, side, from);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_step(int tile_x, int tile_y, const R* src, R* dst, const Dom<R>* doms, const Tile* bulk,
                       int nbulk, const Tile* edge, int nedge, R* side, int from, hipStream_t s) {
#define LBM13_STEP_ARGS src, dst, doms, bulk, nbulk, edge, nedge, side, from, s
    if (tile_x == 64 && tile_y == 4) return launch_step_t<R, 64, 1>(LBM13_STEP_ARGS);
    if (tile_x == 64 && tile_y == 8) return launch_step_t<R, 64, 2>(LBM13_STEP_ARGS);
    if (tile_x == 64 && tile_y == 16) return launch_step_t<R, 64, 4>(LBM13_STEP_ARGS);
    if (tile_x == 32 && tile_y == 8) return launch_step_t<R, 32, 1>(LBM13_STEP_ARGS);
    if (tile_x == 32 && tile_y == 16) return launch_step_t<R, 32, 2>(LBM13_STEP_ARGS);
#undef LBM13_STEP_ARGS
    return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_diag(int tile_x, int tile_y, const R* src, const Dom<R>* doms, int ndom, const Tile* all,
                       int nall, double* part, R* side, int buf, double* out, hipStream_t s) {
    if (nall > 0) {
        if (tile_x == 64) {
            const dim3 blk(64, 4);
            if (tile_y == 4) diag_partial_kernel<R, 64, 1><<<nall, blk, 0, s>>>(src, doms, all, part);
            else if (tile_y == 8) diag_partial_kernel<R, 64, 2><<<nall, blk, 0, s>>>(src, doms, all, part);
            else diag_partial_kernel<R, 64, 4><<<nall, blk, 0, s>>>(src, doms, all, part);
        } else {
            const dim3 blk(32, 8);
            if (tile_y == 8) diag_partial_kernel<R, 32, 1><<<nall, blk, 0, s>>>(src, doms, all, part);
            else diag_partial_kernel<R, 32, 2><<<nall, blk, 0, s>>>(src, doms, all, part);
        }
    }
    diag_final_kernel<R><<<ndom, 256, 0, s>>>(doms, part, out);
    wall_flux_kernel<R><<<ndom, 256, 0, s>>>(src, doms, side, buf, out);
    return hipGetLastError();
}

// Fourier projection of domain d (ntiles = its tile count in the all-tiles
// table); out: 8 doubles in device memory.
template <typename R>
hipError_t launch_fourier(int tile_x, int tile_y, const R* src, const Dom<R>* doms, int d, int ntiles,
                          const Tile* all, int kx, int ky, double* part, double* out, hipStream_t s) {
    if (ntiles > 0)
        fourier_partial_kernel<R><<<ntiles, 256, 0, s>>>(src, doms, d, all, tile_x, tile_y, kx, ky, part);
    fourier_final_kernel<R><<<1, 256, 0, s>>>(doms, d, part, out);
    return hipGetLastError();
}

// Two steps per launch: interior tiles tiles[0, nint), then tiles touching a
// wall or a periodic wrap tiles[nint, nint + nedge).  FP32 takes one thread per
// tile node for tiles of 512 and 1024 nodes with registers capped at 64 (eight
// waves per SIMD where the LDS allows it); node slots past the region's end
// collide nothing.
template <typename R>
hipError_t launch_step2(int tw, int th, const R* src, R* dst, const Dom<R>* doms, const Tile* tiles, int nint,
                        int nedge, R* side, int from, hipStream_t s) {
#define LBM13_FUSED(TW, TH)                                                                                    \
    if (tw == TW && th == TH) {                                                                                \
        static_assert(FusedFits<R, TW, TH>::value, "two-step region exceeds LDS");                             \
        constexpr int NT = sizeof(R) == 4 ? (TW * TH >= 1024 ? 1024 : TW * TH >= 512 ? 512 : 256)              \
                                          : (TW * TH >= 1024 ? 512 : 256);                                     \
        if (nint > 0) step2_interior_kernel<R, TW, TH, NT><<<nint, NT, 0, s>>>(src, dst, doms, tiles, nint);  \
        if (nedge > 0)                                                                                         \
            step2_kernel<R, TW, TH, NT><<<nedge, NT, 0, s>>>(src, dst, doms, tiles + nint, nedge, side, from); \
        return hipGetLastError();                                                                              \
    }
    LBM13_FUSED(64, 16)
    LBM13_FUSED(64, 12)
    LBM13_FUSED(64, 8)
    LBM13_FUSED(64, 4)
    LBM13_FUSED(32, 32)
    LBM13_FUSED(32, 16)
    LBM13_FUSED(32, 8)
    LBM13_FUSED(32, 4)
#undef LBM13_FUSED
    return hipErrorInvalidValue;
}

// Three steps per launch: interior tiles tiles[0, nint) (flag 2, plus 4 where
// the region wraps) on step3_kernel, the other tiles tiles[nint, nint + nedge)
// on step3_wall_kernel; sourced = false when no domain has a body force or an
// energy source.  mixed: the nint + nedge tiles in their spatial order, each
// on its path, in one launch of step3_mixed_kernel.
template <typename R>
hipError_t launch_step3(int tw, int th, const R* src, R* dst, const Dom<R>* doms, const Tile* tiles, int nint,
                        int nedge, R* side, int from, bool sourced, hipStream_t s, bool mixed) {
#define LBM13_STEP3(T, TW, TH)                                                                                 \
    if constexpr (std::is_same<R, T>::value) {                                                                 \
        if (tw == TW && th == TH) {                                                                            \
            constexpr int NT = sizeof(R) == 4 ? (TW * TH < 256 ? 256 : TW * TH) : (TW * TH >= 512 ? 512 : 256); \
            if (mixed) {                                                                                       \
                if (nint + nedge == 0) return hipSuccess;                                                      \
                if (sourced)                                                                                   \
                    step3_mixed_kernel<R, TW, TH, NT, true>                                                    \
                        <<<nint + nedge, NT, 0, s>>>(src, dst, doms, tiles, nint + nedge, side, from);         \
                else                                                                                           \
                    step3_mixed_kernel<R, TW, TH, NT, false>                                                   \
                        <<<nint + nedge, NT, 0, s>>>(src, dst, doms, tiles, nint + nedge, side, from);         \
                return hipGetLastError();                                                                      \
            }                                                                                                  \
            if (nint > 0 && sourced)                                                                           \
                step3_kernel<R, TW, TH, NT, true><<<nint, NT, 0, s>>>(src, dst, doms, tiles, nint);            \
            else if (nint > 0)                                                                                 \
                step3_kernel<R, TW, TH, NT, false><<<nint, NT, 0, s>>>(src, dst, doms, tiles, nint);           \
            if (nedge > 0)                                                                                     \
                step3_wall_kernel<R, TW, TH, NT>                                                               \
                    <<<nedge, NT, 0, s>>>(src, dst, doms, tiles + nint, nedge, side, from);                    \
            return hipGetLastError();                                                                          \
        }                                                                                                      \
    }
    LBM13_STEP3(float, 64, 16)
    LBM13_STEP3(float, 32, 32)
    LBM13_STEP3(float, 64, 8)
    LBM13_STEP3(float, 32, 16)
    LBM13_STEP3(float, 32, 8)
    LBM13_STEP3(double, 64, 8)
    LBM13_STEP3(double, 32, 16)
    LBM13_STEP3(double, 32, 8)
#undef LBM13_STEP3
    return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_side_fill(const R* src, const Dom<R>* doms, const WallLine* lines, int nlines, R* side, int buf,
                            int only_dom, hipStream_t s) {
    if (nlines > 0)
        side_fill_kernel<R><<<(nlines + 255) / 256, 256, 0, s>>>(src, doms, lines, nlines, side, buf, only_dom);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_init(int nx, int ny, R* dst, const Dom<R>* doms, int d, const double* rho, const double* ux,
                       const double* uy, const double* T, const double* coef, hipStream_t s) {
    const dim3 blk(64, 4), grd((nx + 63) / 64, (ny + 3) / 4);
    init_kernel<R><<<grd, blk, 0, s>>>(dst, doms, d, rho, ux, uy, T, coef);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_moments(int nx, int ny, const R* src, const Dom<R>* doms, int d, double* rho, double* ux,
                          double* uy, double* T, hipStream_t s) {
    const dim3 blk(64, 4), grd((nx + 63) / 64, (ny + 3) / 4);
    moments_kernel<R><<<grd, blk, 0, s>>>(src, doms, d, rho, ux, uy, T);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_get_state(int nx, int ny, const R* src, const Dom<R>* doms, int d, double* out, hipStream_t s) {
    const dim3 blk(64, 4), grd((nx + 63) / 64, (ny + 3) / 4);
    get_state_kernel<R><<<grd, blk, 0, s>>>(src, doms, d, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_set_state(int nx, int ny, R* dst, const Dom<R>* doms, int d, const double* in, hipStream_t s) {
    const dim3 blk(64, 4), grd((nx + 63) / 64, (ny + 3) / 4);
    set_state_kernel<R><<<grd, blk, 0, s>>>(dst, doms, d, in);
    return hipGetLastError();
}

// Copies one chunk of host data, passed by value, to dst (4-byte aligned).
__global__ __launch_bounds__(256) void upload_kernel(UploadChunk c, unsigned int* __restrict__ dst) {
    for (unsigned int i = threadIdx.x; i < c.words; i += 256) dst[i] = c.w[i];
}

// Uploads `bytes` (a multiple of 4) of host data to device address dst as a
// sequence of upload_kernel launches on s.  Returns once the arguments are
// copied, so the host data may change or be freed right after; safe under
// stream capture (each launch is recorded with its arguments).
hipError_t launch_upload(const void* host, size_t bytes, void* dst, hipStream_t s) {
    if (bytes % 4 != 0 || reinterpret_cast<uintptr_t>(dst) % 4 != 0) return hipErrorInvalidValue;
    const unsigned char* src = static_cast<const unsigned char*>(host);
    unsigned char* out = static_cast<unsigned char*>(dst);
    UploadChunk c;
    for (size_t off = 0; off < bytes; off += 4 * (size_t)kUploadWords) {
        const size_t n = std::min(bytes - off, 4 * (size_t)kUploadWords);
        c.words = (unsigned int)(n / 4);
        std::memcpy(c.w, src + off, n);
        upload_kernel<<<1, 256, 0, s>>>(c, reinterpret_cast<unsigned int*>(out + off));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The allocation-free entry point's buffers: one array per device, held until
// the process ends.  Host code must not use the name `scratch` as an address
// (on the host it is a stand-in, not device memory); it takes the device
// address from noalloc_scratch().
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

// Device address of `scratch` on the current device, taken once per device
// (with that device current) by hipGetSymbolAddress and kept.
hipError_t noalloc_scratch(void** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* ptr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return hipSuccess;
}

// Writes a checkpoint header (passed by value, so the launch owns its copy).
__global__ __launch_bounds__(64) void ckpt_header_kernel(CkptHeader h, CkptHeader* __restrict__ dst) {
    if (threadIdx.x == 0) *dst = h;
}

hipError_t launch_ckpt_header(const CkptHeader& h, void* dst, hipStream_t s) {
    ckpt_header_kernel<<<1, 64, 0, s>>>(h, static_cast<CkptHeader*>(dst));
    return hipGetLastError();
}

#define LBM13_INSTANTIATE(R)                                                                                      \
    template hipError_t launch_step<R>(int, int, const R*, R*, const Dom<R>*, const Tile*, int, const Tile*, int, \
                                       R*, int, hipStream_t);                                                     \
    template hipError_t launch_step2<R>(int, int, const R*, R*, const Dom<R>*, const Tile*, int, int, R*, int,     \
                                        hipStream_t);                                                             \
    template hipError_t launch_step3<R>(int, int, const R*, R*, const Dom<R>*, const Tile*, int, int, R*, int,     \
                                        bool, hipStream_t, bool);                                                 \
    template hipError_t launch_side_fill<R>(const R*, const Dom<R>*, const WallLine*, int, R*, int, int,          \
                                            hipStream_t);                                                         \
    template hipError_t launch_diag<R>(int, int, const R*, const Dom<R>*, int, const Tile*, int, double*, R*,     \
                                       int, double*, hipStream_t);                                                \
    template hipError_t launch_fourier<R>(int, int, const R*, const Dom<R>*, int, int, const Tile*, int, int,    \
                                          double*, double*, hipStream_t);                                         \
    template hipError_t launch_init<R>(int, int, R*, const Dom<R>*, int, const double*, const double*,           \
                                       const double*, const double*, const double*, hipStream_t);                 \
    template hipError_t launch_moments<R>(int, int, const R*, const Dom<R>*, int, double*, double*, double*,     \
                                          double*, hipStream_t);                                                  \
    template hipError_t launch_get_state<R>(int, int, const R*, const Dom<R>*, int, double*, hipStream_t);        \
    template hipError_t launch_set_state<R>(int, int, R*, const Dom<R>*, int, const double*, hipStream_t);

LBM13_INSTANTIATE(double)
LBM13_INSTANTIATE(float)

}  // namespace lbm13
