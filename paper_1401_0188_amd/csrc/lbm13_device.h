// lbm13_device.h -- device-side data structures of the D2Q13 step (gfx950).
//
// Populations are stored as deviations g_i = f*_i - f_i^rest from the rest
// populations f^rest = f^eq(rho = 1, j = 0, E = E0), one plane per velocity
// (structure of arrays): element (i, y, x) of a domain sits at
//   base + off + i * plane + y * pitch + x.
// Keeping deviations lets the FP32 form collide without cancelling O(1) terms.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm13 {

enum SideKind { kPeriodic = 0, kAdiabatic = 1, kDirichletT = 2 };

// Per-domain descriptor: geometry, collision constants in the working precision
// R (deviation form), FP64 constants for read-back and diagnostics.
template <typename R>
struct alignas(16) Dom {
    long long off;    // element offset of plane 0 of this domain in each population buffer
    long long woff;   // element offset of this domain's wall-layer side array: 2 buffers x 2 (nx + ny) lines x 4
    int plane;        // elements between two velocity planes
    int pitch;        // elements between two rows
    int nx, ny;
    int xper, yper;   // 1 when the axis is periodic
    int kind[4];      // W, E, S, N
    int tile0, ntiles;  // range of this domain in the domain-ordered tile table
    int collide;
    int pad0;
    // equilibria about rest: eps' = c_er rho' + c_eE E', varpi' = c_vr rho' + c_vE E',
    // q = j (a1 + h1 rho' + k1 E'), r = j (a2 + h2 rho' + k2 E'),  (rho', E' deviations)
    R c_er, c_eE, c_vr, c_vE;
    R a1, h1, k1, a2, h2, k2;
    R QE;  // Q_E, the energy source: the kept post-collision state carries E(t) + Q_E
    // relaxation folded with the norms D_k for the collision:
    //   s_eps (eps - eps^eq) / 42196 = sum_j aeps[j] (g0, S1, S2, S3)_j and
    //   s_varpi (varpi - varpi^eq) / 548 = sum_j avp[j] (g0, S1, S2, S3)_j, with
    //   S1, S2, S3 the sums over the classes |v|^2 = 1, 2, 4 (both are linear in
    //   the populations); eQ[c] = -M_E,c Q_E / 4004, the energy source as
    //   Delta_E = -Q_E for the rest population and the three classes;
    //   kX = s_XX / 68, kY = s_XX / 4, kXe = s_XXe / 68, kq = s_q / 20, kr = s_r / 70,
    //   -F / 14 = fjx + gjx rho' (and y) for the body force F = F0 + g (rho - rho0)
    R aeps[4], avp[4];
    R eQ[4];
    // odd moments: per axis, the update patterns of the speed-1 link, the
    // speed-2 link and the diagonal are ow[2c] nq + ow[2c+1] nr (c = 0, 1, 2),
    // nq = q - q^eq, nr = r - r^eq: ow = (-2 kq, 4 kr, 2 kq, kr, -kq, -3 kr)
    R ow[6];
    R kX, kY, kXe, kq, kr;
    R fjx, fjy, gjx, gjy;
    // walls: tangential velocity, E_W - E0 for temperature walls
    R wall_u[4];
    R wall_dE[4];
    // FP64 constants
    double E0;
    double frest[4];  // rest populations of the |v|^2 = 0, 1, 2, 4 classes
    double F0x_d, F0y_d, gx_d, gy_d;  // F = (F0x_d, F0y_d) + (gx_d, gy_d) rho
    double B;         // equilibrium E flux per unit momentum
    double QE_d;      // Q_E in FP64
    double nu_scale;  // nx / (kappa_E (T_W - T_E)), 0 when T_W == T_E
};

// One tile of the tile tables: domain index, origin, flags (bit 0: tile holds
// nodes within two nodes of a wall; bit 1, two-step tiles: the tile, its
// two-node halo and their sources lie inside the domain, at least two nodes
// from every wall, with no periodic wrap).
struct alignas(16) Tile {
    int dom, x0, y0, flags;
};

// One wall line: the position `pos` along wall `w` (0 W, 1 E, 2 S, 3 N) of
// domain `dom`; `line` is its index among the domain's 2 (nx + ny) lines
// (W: y, E: ny + y, S: 2 ny + x, N: 2 ny + nx + x).  Each line keeps, per
// state buffer, (rho', E') of the first fluid layer and rho' of the second.
struct alignas(16) WallLine {
    int dom, w, pos, line;
};

// Tiles of the two-steps-per-launch kernels.  For tiles that touch a wall or a
// periodic wrap the region (TW + 4) x (TH + 4) x 13 populations plus the
// wall-layer side values must fit the 160 KB of LDS a gfx950 workgroup can
// address; Fused<R> is the default shape.
template <typename R>
struct Fused;
template <>
struct Fused<float> {
    static constexpr int TW = 32, TH = 32;
};
template <>
struct Fused<double> {
    static constexpr int TW = 32, TH = 16;
};
template <typename R, int TW, int TH>
struct FusedFits {
    static constexpr bool value = 13 * (TW + 4) * (TH + 4) * sizeof(R) + 6 * (TW + TH + 8) * sizeof(R) <= 163840;
};

// Header of a raw checkpoint: the first kCkptHeaderBytes bytes of the blob,
// followed by the stored deviations of one domain, dense [13][ny][nx].
struct CkptHeader {
    char magic[8];              // "LBM13CK" and a terminating zero
    int version;                // kCkptVersion
    int precision;              // LBM13_FP64 or LBM13_FP32_DEV
    int nx, ny;
    long long steps;            // steps taken when the checkpoint was written
    unsigned long long payload;  // bytes of populations after the header
};
constexpr int kCkptVersion = 1;
constexpr size_t kCkptHeaderBytes = 256;

// Size of the static device array that the allocation-free entry point
// (lbm13_advance_noalloc) keeps its buffers in, per device.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;

// Host data handed to a kernel by value (kernel arguments are copied at
// launch and into a captured graph), for uploads that must not depend on host
// memory outliving the call: kUploadWords 32-bit words per launch.
constexpr int kUploadWords = 768;
struct UploadChunk {
    unsigned int words;
    unsigned int w[kUploadWords];
};

constexpr int kDiagPartials = 10;  // per-tile partial reductions
constexpr int kDiagOut = 16;       // values per domain

}  // namespace lbm13
