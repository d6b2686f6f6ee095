// common.hpp -- types shared by the host side of the C ABI and the HIP kernels.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "lattice.hpp"

namespace lbm {

enum StorageId : int { kF64 = 0, kF32 = 1, kF16 = 2, kBF16 = 3 };

// Per-step constants in the arithmetic precision C, passed by value as a kernel argument
// (they land in scalar registers). Index 0 of the per-pair arrays is the rest velocity.
//
// With u = c.s, k = c.(K s) and |s|^2 for one velocity, the equilibrium in lattice units
// (cs^2 = 1/3) splits as f^eq = rho r + w rho P'(s) with the rest part r = w (1 + 1.5 c.K.c
// - 0.5 tr K) and the velocity part
//     P'(s) = [4.5 u^2 - 1.5 |s|^2]                               (even in c)
//           + [u (A_p - 4.5 |s|^2 + 4.5 u^2) - 3 k]               (odd in c, order 3)
//           + [3 u]                                               (odd in c, order 2)
// where A_p = 3 + 4.5 c.K.c - 1.5 tr K. The stored deviation is g = f - sigma, so
//     g^eq = r (rho - rho0) + (rho0 r - sigma) + w rho P'(s).
template <typename C> struct StepConsts {
    C omega;            // 1 / tau
    C keep;             // 1 - omega
    C rho0;             // reference density of the shift
    C k[6];             // K_xx, K_yy, K_zz, K_xy, K_xz, K_yz
    C km3[6];           // -3 K, the same entries (the odd part's K s term)
    C w[kMaxPairs + 1];     // weight w_p
    C rest[kMaxPairs + 1];  // r_p
    C eoff[kMaxPairs + 1];  // rho0 r_p - sigma_p (zero for the rest-equilibrium shift)
    C ow[kMaxPairs + 1];    // omega w_p     (omega g^eq, the relaxed equilibrium)
    C orest[kMaxPairs + 1]; // omega r_p
    C oeoff[kMaxPairs + 1]; // omega (rho0 r_p - sigma_p)
    C a[kMaxPairs + 1];     // A_p of the odd part (order 3)
    C sigma[kMaxPairs + 1]; // sigma_p (read-out only)
    C force[3];             // body force F (exact-difference method)
    int32_t forced;         // F != 0
};

// Grid extents and the storage layout of its population arrays (both state buffers and the
// adjoint's lam buffers; counted in elements, so one layout serves every element type).
// Populations are stored z-plane by z-plane. A z-plane is cut into ny / rows blocks of `rows`
// consecutive y-rows (rows divides ny), and a block holds its q direction planes one after
// another, bc = rows nx cells each. Direction i of cell (x, y, z) is element
//     z zs + (y / rows) bq + i bc + (y mod rows) nx + x,      bq = q bc,  zs = q nx ny.
// Batched domains use linear blocks of 2^lb canonical cells instead (bc = 2^lb, bq = q bc;
// FlatCell). Canonical arrays (masks, link words, per-cell fields, exported populations) keep
// the plain order x + nx (y + ny z).
struct Grid {
    int32_t nx, ny, nz;
    uint32_t n;     // cells = nx * ny * nz (< 2^31)
    uint32_t rows;  // y-rows per block
    uint32_t mr;    // floor(2^32 / rows) (0xffffffff for rows = 1): y -> (y / rows, y mod rows)
    uint32_t bc;    // rows nx: cells per block and direction
    uint32_t bq;    // q bc: elements per block
    uint32_t zs;    // q nx ny: elements per z-plane (the bytes of one z-plane stay below 4 GiB)
    uint32_t lb;    // batched domains only: log2 of the cells per linear block (bc = 2^lb)
};

// ---- launchers (kernels.hip) -----------------------------------------------------------
// All return hipSuccess or the launch error; they enqueue on `stream` and never synchronise.

// links: per-cell link words (bit 0: the cell is solid; bit i: the cell x - c_i is solid) or
// null for a grid without solid cells.
hipError_t launch_links(int lattice, const Grid &g, const uint8_t *mask, uint32_t *links, hipStream_t stream);

hipError_t launch_init(int lattice, int storage, int order, const Grid &g, const StepConsts<double> &k,
                       const double *rho, const double *s, const uint32_t *links, void *dst, hipStream_t stream);

// Launch flags of the step kernel (same values as LBM_LAUNCH_* in lbm.h).
constexpr int kLaunchXcdSlabs = 1;     // XCD-contiguous tile order
constexpr int kLaunchShiftedPull = 2;  // every pull a shifted load (no lane exchange)
constexpr int kLaunchStreamOnly = 1 << 8;  // library-internal: pulls and stores only (no collision)

// gray: per-cell gray fraction m (partial bounce-back) or null.
hipError_t launch_step(int lattice, int storage, int order, const Grid &g, const StepConsts<double> &k64,
                       const StepConsts<float> &k32, const uint32_t *links, const float *gray, const void *src,
                       void *dst, int block_x, int block_y, int flags, hipStream_t stream);

// ---- the gradient path (reverse sweep) ----
constexpr int kGradPartialsHost = 7;  // per work-group: dJ/dK (6, symmetric part: xx yy zz xy xz yz), dJ/dtau
// lam: adjoint populations (q N elements, the population layout of Grid) in the arithmetic
// precision of the storage; launch_seed writes them unless lam is null. jpart: one double per
// work-group of the seed launch (moments_groups(g)).
// links: the link words of a masked grid or null.
hipError_t launch_seed(int lattice, int storage, const Grid &g, const StepConsts<double> &k64,
                       const StepConsts<float> &k32, const void *src, void *lam, double *jpart, int kind, int plane,
                       const uint32_t *links, hipStream_t stream);
hipError_t launch_adjoint(int lattice, int storage, int order, const Grid &g, const StepConsts<double> &k64,
                          const StepConsts<float> &k32, const void *state, const void *lam_in, void *lam_out,
                          const float *gray, const uint32_t *links, double *dmask, double *gpart, hipStream_t stream);
hipError_t launch_sum(const double *part, uint32_t nblocks, int m, double *out, hipStream_t stream);
hipError_t launch_zero(double *p, uint64_t n, hipStream_t stream);

// rho / s may be null. partials: scratch of kPartials * moments_groups(g) doubles; totals:
// kPartials doubles of scratch (sum drho, sum rho s_x, _y, _z, fluid cells).
// LDS for a launch to reserve without using it so that at most `groups` work-groups share a
// compute unit (160 KiB of LDS each on gfx950): a little over 160 KiB / (groups + 1). LDS is
// allocated in 512-byte blocks, so `groups` of them still fit for up to 17 groups.
constexpr unsigned cap_lds(unsigned groups) { return 160u * 1024u / (groups + 1u) + 512u; }

// Work-groups per compute unit for an FP32 or FP64 streaming step (work-groups of `threads`
// lanes, one cell each, q pulls of `bytes` per cell): the count that keeps about 78 KiB of pulls
// in flight per compute unit, and at least 8 waves. Measured best caps for 256-lane work-groups
// (D3Q19 and D3Q27 256^3, D2Q9 256 x 65536): D3Q19 FP32 4, D3Q19 FP64 2, D3Q27 FP32 3, D3Q27
// FP64 2 (1 is far slower), D2Q9 FP64 4; D2Q9 FP32 gains nothing from a cap (the rule gives 9,
// more than fit).
constexpr unsigned stream_groups(unsigned q, unsigned bytes, unsigned threads = 256u)
{
    const unsigned per = threads * q * bytes;
    const unsigned n = (79872u + per / 2u) / per;
    const unsigned least = (8u * 64u + threads - 1u) / threads;
    return n < least ? least : n;
}
// The LDS to reserve for that cap, or 0 where the cap is no lower than the most work-groups of
// that size a compute unit holds (32 waves).
constexpr unsigned stream_lds(unsigned q, unsigned bytes, unsigned threads = 256u)
{
    const unsigned most = 32u / ((threads + 63u) / 64u);
    return stream_groups(q, bytes, threads) >= most ? 0u : cap_lds(stream_groups(q, bytes, threads));
}
static_assert(stream_groups(19, 4) == 4 && stream_groups(19, 8) == 2 && stream_groups(27, 4) == 3 &&
                  stream_groups(27, 8) == 2 && stream_groups(9, 8) == 4 && stream_lds(9, 4) == 0 &&
                  stream_groups(19, 4, 64) == 16 && stream_groups(27, 8, 64) == 8,
              "the measured caps, and the same bytes in flight for smaller work-groups");

constexpr int kPartials = 5;
constexpr uint32_t kMomentGroups = 2048;  // most work-groups of a moments launch
hipError_t launch_moments(int lattice, int storage, const Grid &g, const StepConsts<double> &k,
                          const uint32_t *links, const void *src, double *rho, double *s, double *partials,
                          double *totals, hipStream_t stream);
// Work-groups of one launch_moments (at most kMomentGroups).
uint32_t moments_groups(const Grid &g);
// Work-groups of the row-spanning launches over a grid (init, permute).
uint32_t row_blocks(const Grid &g);
// Work-groups of one launch_adjoint (the gpart partial sets it adds to).
uint32_t adjoint_blocks(const Grid &g);

// mode 0: out[i][x] = the state's canonical g_i(x) (raw storage type), mode 1: the inverse,
// mode 2: out[i][x] = double(g_i(x)) + sigma_i. Solid cells: zeros out / ignored in.
hipError_t launch_permute(int lattice, int storage, int mode, const Grid &g, const StepConsts<double> &k,
                          const uint32_t *links, const void *src, void *dst, hipStream_t stream);

hipError_t launch_copy(void *dst, const void *src, int64_t nbytes, hipStream_t stream);

}  // namespace lbm
