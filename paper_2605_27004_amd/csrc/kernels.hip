// kernels.hip -- gfx950 kernels of the anisotropic-equilibrium BGK lattice Boltzmann update.
//
// State layout. Populations live in two buffers of deviations g_i = f_i - sigma_i in the
// storage type S, in the blocked layout of Grid (each z-plane a run of blocks of a few
// y-rows, every block holding its q direction planes back to back). After k steps the
// current buffer holds the POST-collision values of step k-1 at their own cell, so the
// canonical pre-collision state is the gather f_i(k, x) = sigma_i + state_i(x - c_i)
// (periodic wrap). One step is therefore a single pass over HBM: gather q values along
// -c_i (pull streaming), form rho and s, build the equilibrium, relax, and store q values
// at the cell itself into the other buffer (eq:LBE_BGK). The initial state is written to
// the same gather positions, and every read-out applies the same gather, so no
// separate streaming pass exists anywhere.
//
// Equilibrium (eq:3rd_order_equilibrium with cs^2 = 1/3, per opposite pair c / -c):
//   f^eq = rho r + w rho P'(s),  r = w (1 + 1.5 c.K.c - 0.5 tr K),
//   P'   = 4.5 u^2 - 1.5 |s|^2  +/-  [u (A - 4.5 |s|^2 + 4.5 u^2) - 3 c.(K s)]   (order 3)
//   P'   = 4.5 u^2 - 1.5 |s|^2  +/-  3 u                                         (order 2)
// with u = c.s and A = 3 + 4.5 c.K.c - 1.5 tr K; the odd part changes sign between the two
// members of a pair, the even part and r do not. The arithmetic runs on the stored
// deviations, rho = rho0 + sum_i g_i and rho s = sum_i g_i c_i (sum_i sigma_i c_i = 0), which
// keeps FP32 mass conservation at round-off of the deviations rather than of f.
//
// The path is bound by HBM bandwidth (2 q sizeof(S) bytes per cell update), so there is no
// MFMA: each lane owns one cell and loads are coalesced along x. Where a wave lies inside one
// grid row, x-shifted pulls load the lane's own x and shift one lane with DPP, exchanging the
// wave-edge values through LDS (pull_aligned); otherwise the periodic wrap is a per-lane offset
// select.
#include <hip/hip_runtime.h>

#include "cell.hpp"
#include "common.hpp"

// No implicit contraction: every fused multiply-add below is written out, so the rounding of
// each cell update is fixed by the source and identical in every kernel variant and launch
// shape.
#pragma clang fp contract(off)

namespace lbm {
namespace {

using namespace cell;

// ---- kernels -------------------------------------------------------------------------------

// Work-group -> tile mapping of the step kernel. Work-groups of a 1-D launch are handed to the
// eight XCDs round-robin (flat id b runs on XCD b mod 8). With `xcd_slabs` set, the tile
// order is permuted so that XCD k processes one contiguous range of tiles -- a slab of the
// grid -- and the neighbour rows and the x-boundary cache lines a pull gathers are mostly
// fetched into, and found in, that XCD's own L2.
struct TileMap {
    uint32_t tiles_x, tiles_y, nblocks;
    uint32_t xcd_slabs;
    uint32_t row_xcd;  // the tiles of one row on one XCD (see tile_of)
};

__device__ inline uint32_t tile_of(const TileMap &m, uint32_t b)
{
    if (!m.xcd_slabs) {
        // Work-groups go to the 8 XCDs in turn (b mod 8). With row_xcd, each group of 8 rows of
        // tiles_x tiles is dispatched so that the tiles of one row share an XCD and follow each
        // other: block b of the group takes row b mod 8, tile b / 8. The links step reads lines
        // that the tiles of a row share (shifted and bounce-back pulls), which the XCD's L2 then
        // serves once: 512^3 porous medium FP16 2,778 -> 2,647 us, FP32 4,854 -> 4,812 us. The
        // periodic step with shifted pulls got slower with it (D3Q19 512^3: 3,377 -> 3,484 us).
        const uint32_t tx = m.tiles_x, grp = 8u * tx;
        if (!m.row_xcd || tx == 1u) return b;
        const uint32_t full = (m.nblocks / grp) * grp;  // a ragged last group keeps the plain order
        if (b >= full) return b;
        const uint32_t j = b % grp;
        return (b - j) + (j % 8u) * tx + j / 8u;
    }
    const uint32_t q = m.nblocks / 8u, r = m.nblocks % 8u;
    const uint32_t xcd = b % 8u, local = b / 8u;
    return xcd < r ? xcd * (q + 1u) + local : r * (q + 1u) + (xcd - r) * q + local;
}

// Step variants: kPlain (periodic fluid: q pulls, collision, q streaming stores per cell);
// kLinks (link word per cell: solid cells write zeros, links to solid cells bounce back, plus
// the body force); kGray (gray fraction m per cell: f* = (1 - m) f^BGK + m f_opp, plus the
// body force).
// kStream: the kPlain pulls and stores without the collision (free streaming), a measurement
// aid that moves exactly the step's bytes in the step's pattern.
enum StepMode : int { kPlain = 0, kLinks = 1, kGray = 2, kStream = 3 };

// Pull of a cell's q pre-collision deviations when every work-group spans whole grid rows: nx
// is a multiple of 64 and the work-group is nx wide (launch_step checks this). An x-shifted pull
// would make each wave read three cache lines of which two are shared with the neighbouring
// waves; measured on the bare D3Q19 256^3 FP32 pattern, that costs 4% of the pass against
// loading the source row at the lane's own x (every line then read by one wave,
// non-temporally) and moving the values one lane across the wave with DPP. The one value that
// crosses a wave's edge comes from the neighbouring wave of the same row through LDS. The
// result is the same gather, bit for bit. `live` (the wave's row exists) is uniform over each
// wave; every wave reaches the barrier. Where a row spans several work-groups the end waves'
// edge values would need loads of their own; measured that way, the exchange lost to shifted
// loads (D3Q19 FP32 512^3: 3.55 vs 3.40 ms per step; 448^3 in 64-wide work-groups: 2.83 vs
// 2.24 ms), so such launches use the shifted pull.
// How the step kernel pulls (launch_step picks): every population with its own shifted load, or
// the lane exchange inside whole rows (pull_aligned, or pull_rows_lds for FP16 storage).
enum PullKind : int { kPullShifted = 0, kPullRows = 1 };

template <int LAT, typename S, int PULL>
__device__ inline void pull_aligned(const S *__restrict__ src, const Grid &g, const Cell &c, int32_t x, bool live,
                                    typename Conv<S>::C *gp, typename Conv<S>::C *gm)
{
    static_assert(PULL == kPullRows, "lane-exchange pulls only");
    using L = Lattice<LAT>;
    using C = typename Conv<S>::C;
    constexpr PullOrder<LAT> kPull{};
    __shared__ C edge[L::Q][256 / 64];  // [direction][wave]: the value a neighbouring wave needs
    const uint32_t wpr = blockDim.x >> 6;  // waves per row of the work-group
    const uint32_t pos = threadIdx.x >> 6;  // this wave's place in its row
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = threadIdx.y * wpr + pos;
    const uint32_t wl = threadIdx.y * wpr + (pos == 0u ? wpr - 1u : pos - 1u);  // holds x0 - 1 (row wrap)
    const uint32_t wr = threadIdx.y * wpr + (pos == wpr - 1u ? 0u : pos + 1u);  // holds x0 + 64
    if (live) {
#pragma unroll
        for (int j = 0; j < L::Q; ++j) {
            const int i = kPull.dir[j];
            if (i == 0) {
                gp[0] = Conv<S>::ld(ld_nt_at(pop_base(src, g, 0, own_ref(c)), own_ref(c).idx));
                continue;
            }
            const int p = (i - 1) / 2, sg = (i & 1) ? 1 : -1;
            const PairRow v = L::pair(p);
            const Ref r = nbr(c, 0, sg * v.cy, sg * v.cz);  // the source row at this lane's x
            const C val = Conv<S>::ld(ld_nt_at(pop_base(src, g, i, r), r.idx));
            if (i & 1) gp[p + 1] = val; else gm[p + 1] = val;
        }
        // after all loads have been issued: the edge values the neighbouring waves pull
        if (lane == 63u) {  // pulled from x - 1 by lane 0 of the next wave
#pragma unroll
            for (int p = 0; p < L::NP; ++p) {
                const int cx = L::pair(p).cx;
                if (cx > 0) edge[2 * p + 1][wv] = gp[p + 1];
                if (cx < 0) edge[2 * p + 2][wv] = gm[p + 1];
            }
        }
        if (lane == 0u) {  // pulled from x + 1 by lane 63 of the previous wave
#pragma unroll
            for (int p = 0; p < L::NP; ++p) {
                const int cx = L::pair(p).cx;
                if (cx < 0) edge[2 * p + 1][wv] = gp[p + 1];
                if (cx > 0) edge[2 * p + 2][wv] = gm[p + 1];
            }
        }
    }
    __syncthreads();
    if (!live) return;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const int p = (i - 1) / 2, sg = (i & 1) ? 1 : -1;
        const PairRow v = L::pair(p);
        const int cx = sg * v.cx;
        if (cx == 0) continue;
        C &val = (i & 1) ? gp[p + 1] : gm[p + 1];
        if (cx > 0)  // pulled from x - 1
            val = wave_shift<kFromLeft>(edge[i][wl], val);
        else         // pulled from x + 1
            val = wave_shift<kFromRight>(edge[i][wr], val);
    }
}

// Index of direction i among the directions with c_x != 0 (-1 for the others).
template <int LAT> struct XShifted {
    int slot[Lattice<LAT>::Q];
    int count;
    constexpr XShifted() : slot(), count(0)
    {
        for (int i = 0; i < Lattice<LAT>::Q; ++i) {
            slot[i] = -1;
            if (i > 0 && Lattice<LAT>::pair((i - 1) / 2).cx != 0) slot[i] = count++;
        }
    }
};

// The lane exchange with every x-shifted value passed through LDS: each lane leaves its loaded
// value of every direction with c_x != 0 at its own place in the row and, after one barrier,
// reads its row neighbour's (x - 1 for c_x > 0, x + 1 for c_x < 0, wrapping inside the row).
// Work-groups span whole rows (blockDim.x == nx). Values travel in the storage type.
template <int LAT, typename S>
__device__ inline void pull_rows_lds(const S *__restrict__ src, const Grid &g, const Cell &c, bool live,
                                     typename Conv<S>::C *gp, typename Conv<S>::C *gm)
{
    using L = Lattice<LAT>;
    constexpr PullOrder<LAT> kPull{};
    constexpr XShifted<LAT> kX{};
    __shared__ S xb[kX.count][256];
    const uint32_t me = threadIdx.y * blockDim.x + threadIdx.x;
    const uint32_t row0 = me - threadIdx.x;
    const uint32_t left = row0 + (threadIdx.x == 0u ? blockDim.x - 1u : threadIdx.x - 1u);
    const uint32_t right = row0 + (threadIdx.x == blockDim.x - 1u ? 0u : threadIdx.x + 1u);
    S raw[L::Q];
    if (live) {
#pragma unroll
        for (int j = 0; j < L::Q; ++j) {
            const int i = kPull.dir[j];
            if (i == 0) {
                raw[0] = ld_nt_at(pop_base(src, g, 0, own_ref(c)), own_ref(c).idx);
                continue;
            }
            const int p = (i - 1) / 2, sg = (i & 1) ? 1 : -1;
            const PairRow v = L::pair(p);
            const Ref r = nbr(c, 0, sg * v.cy, sg * v.cz);  // the source row at this lane's x
            raw[i] = ld_nt_at(pop_base(src, g, i, r), r.idx);
        }
#pragma unroll
        for (int i = 1; i < L::Q; ++i)
            if (kX.slot[i] >= 0) xb[kX.slot[i]][me] = raw[i];
    }
    __syncthreads();
    if (!live) return;
    gp[0] = Conv<S>::ld(raw[0]);
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const int p = (i - 1) / 2, sg = (i & 1) ? 1 : -1;
        const int cx = sg * L::pair(p).cx;
        S v = raw[i];
        if (cx > 0) v = xb[kX.slot[i]][left];   // pulled from x - 1
        if (cx < 0) v = xb[kX.slot[i]][right];  // pulled from x + 1
        if (i & 1) gp[p + 1] = Conv<S>::ld(v); else gm[p + 1] = Conv<S>::ld(v);
    }
}

template <int LAT, typename S, int ORDER, int MODE, int PULL>
__global__ __launch_bounds__(256) void k_step(const S *__restrict__ src, S *__restrict__ dst, const Grid g,
                                              const StepConsts<typename Conv<S>::C> k, const TileMap m,
                                              const uint32_t *__restrict__ links, const float *__restrict__ gray)
{
    constexpr bool GENERAL = MODE == kLinks;
    constexpr bool ALIGNED = PULL != kPullShifted;
    static_assert(!(ALIGNED && GENERAL), "the lane-exchange pull serves the periodic, gray and streaming steps");
    using L = Lattice<LAT>;
    constexpr PullOrder<LAT> kPull{};
    using C = typename Conv<S>::C;
    constexpr int NP = L::NP;
    const uint32_t t = tile_of(m, blockIdx.x);
    const uint32_t tx = t % m.tiles_x, tyz = t / m.tiles_x;
    const int32_t x = (int32_t)(tx * blockDim.x + threadIdx.x);
    const int32_t y = (int32_t)((tyz % m.tiles_y) * blockDim.y + threadIdx.y);
    const int32_t z = (int32_t)(tyz / m.tiles_y);

    C gp[NP + 1], gm[NP + 1];
    Cell c;
    if constexpr (ALIGNED) {
        const bool live = y < g.ny;
        c = cell_of(g, x, live ? y : 0, z);
        // FP16 passes the x-shifted values through LDS, the other storages use DPP shifts:
        // measured on the D3Q19 256^3 step, FP16 211.8 -> 204.0 us through LDS, while BF16
        // went 200.5 -> 208.5 us and FP32 400.2 -> 401.4 us
        if constexpr (std::is_same<S, _Float16>::value)
            pull_rows_lds<LAT, S>(src, g, c, live, gp, gm);
        else
            pull_aligned<LAT, S, PULL>(src, g, c, x, live, gp, gm);
        if (!live) return;
    } else if constexpr (GENERAL) {
        if (x >= g.nx || y >= g.ny) return;
        c = cell_of(g, x, y, z);
        // A solid cell has no state and none of its slots is ever read (links route around
        // it), but its lane still stores zeros so that every store of the wave covers whole
        // cache lines; partial-line stores along solid boundaries measured far slower.
        const uint32_t lk = links ? links[c.own] : 0u;
        if (lk & 1u) {
#pragma unroll
            for (int p = 0; p <= NP; ++p) gp[p] = gm[p] = C(0);
        } else {
#pragma unroll
            for (int j = 0; j < L::Q; ++j) {
                const int i = kPull.dir[j], p = (i - 1) / 2;
                if (i == 0)
                    gp[0] = Conv<S>::ld(ld_pop(src, g, 0, own_ref(c)));
                else if (i & 1)
                    gp[p + 1] = Conv<S>::ld(ld_slot(src, g, slot_plus<LAT>(c, p, lk)));
                else
                    gm[p + 1] = Conv<S>::ld(ld_slot(src, g, slot_minus<LAT>(c, p, lk)));
            }
            collide_cell<LAT, ORDER, true, C, kClose<S>>(k, gp, gm);
        }
    } else {
        if (x >= g.nx || y >= g.ny) return;
        c = cell_of(g, x, y, z);
#pragma unroll
        for (int j = 0; j < L::Q; ++j) {
            const int i = kPull.dir[j], p = (i - 1) / 2;
            if (i == 0)
                gp[0] = Conv<S>::ld(ld_pop(src, g, 0, own_ref(c)));
            else if (i & 1)
                gp[p + 1] = Conv<S>::ld(ld_pop(src, g, i, src_plus<LAT>(c, p)));
            else
                gm[p + 1] = Conv<S>::ld(ld_pop(src, g, i, src_minus<LAT>(c, p)));
        }
    }

    if constexpr (MODE == kPlain) collide_cell<LAT, ORDER, false, C, kClose<S>>(k, gp, gm);
    if constexpr (MODE == kGray) {
        C pp[NP + 1], pm[NP + 1];
#pragma unroll
        for (int p = 0; p <= NP; ++p) {
            pp[p] = gp[p];
            pm[p] = gm[p];
        }
        collide_cell<LAT, ORDER, true, C, kClose<S>>(k, gp, gm);
        // partial bounce-back on the node: the opposite of +c is -c of the same pair
        const C mg = (C)gray[c.own];
        gp[0] = fmad(mg, pp[0] - gp[0], gp[0]);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const C a = gp[p + 1];
            gp[p + 1] = fmad(mg, pm[p + 1] - a, a);
            gm[p + 1] = fmad(mg, pp[p + 1] - gm[p + 1], gm[p + 1]);
        }
    }
    const PlaneStores ps = plane_stores(dst, g, own_ref(c));
    st_plane(ps, 0, Conv<S>::st(gp[0]));
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        st_plane(ps, 2 * p + 1, Conv<S>::st(gp[p + 1]));
        st_plane(ps, 2 * p + 2, Conv<S>::st(gm[p + 1]));
    }
}

// Link words from a uint8 solid mask: bit 0 = the cell is solid, bit i = the cell x - c_i is.
template <int LAT>
__global__ __launch_bounds__(256) void k_links(const uint8_t *__restrict__ mask, uint32_t *__restrict__ links,
                                               const Grid g)
{
    using L = Lattice<LAT>;
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t y = blockIdx.y * blockDim.y + threadIdx.y;
    const int32_t z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const FlatCell c = canon_cell_of(g, (uint32_t)x, (uint32_t)y, (uint32_t)z);
    uint32_t w = mask[c.own] ? 1u : 0u;
#pragma unroll
    for (int p = 0; p < L::NP; ++p) {
        if (mask[src_plus<LAT>(c, p).idx]) w |= 1u << (2 * p + 1);
        if (mask[src_minus<LAT>(c, p).idx]) w |= 1u << (2 * p + 2);
    }
    links[c.own] = w;
}

// f_i(0, x) = f^eq_i(rho(x), s(x)) in FP64, stored as a deviation in the slot the canonical
// gather reads for direction i at x (solid cells are skipped).
template <int LAT, typename S, int ORDER>
__global__ __launch_bounds__(256) void k_init(const double *__restrict__ rho_in, const double *__restrict__ s_in,
                                              const uint32_t *__restrict__ links, S *__restrict__ dst,
                                              const Grid g, const StepConsts<double> k)
{
    using L = Lattice<LAT>;
    using C = typename Conv<S>::C;
    constexpr int NP = L::NP;
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t y = blockIdx.y * blockDim.y + threadIdx.y;
    const int32_t z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const Cell c = cell_of(g, x, y, z);
    const uint32_t lk = links ? links[c.own] : 0u;
    if (lk & 1u) {  // solid: no state; its own slots are set to zero like every step does
        for (int i = 0; i < L::Q; ++i) st_pop(dst, g, i, own_ref(c), Conv<S>::st(C(0)));
        return;
    }
    const double rho = rho_in[c.own];
    const double sx = s_in[c.own];
    const double sy = s_in[(size_t)g.n + c.own];
    const double sz = (L::D == 3) ? s_in[2 * (size_t)g.n + c.own] : 0.0;
    double eqp[NP + 1], eqm[NP + 1];
    equilibrium_pairs<LAT, ORDER, double>(k, rho - k.rho0, rho, sx, sy, sz, eqp, eqm);
    st_pop(dst, g, 0, own_ref(c), Conv<S>::st((C)eqp[0]));
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const Slot sp = slot_plus<LAT>(c, p, lk), sm = slot_minus<LAT>(c, p, lk);
        st_slot(dst, g, sp, Conv<S>::st((C)eqp[p + 1]));
        st_slot(dst, g, sm, Conv<S>::st((C)eqm[p + 1]));
    }
}

constexpr int kRedThreads = 256;

// Moments of the canonical state in FP64 plus per-work-group partial sums of (drho, rho u_x,
// rho u_y, rho u_z, fluid cells); u = (j + F/2) / rho. The launch has a fixed number of
// work-groups (at most kMomentGroups, whatever the grid): work-group w takes the row tiles
// w, w + G, w + 2G, ... of the row_grid order, each lane sums its cells in that order, and the
// work-group adds its lanes in a fixed tree, so the totals are reproducible bit for bit and
// the partials need a small scratch of constant size.
template <int LAT, typename S>
__global__ __launch_bounds__(kRedThreads) void k_moments(const S *__restrict__ src, const uint32_t *__restrict__ links,
                                                         double *__restrict__ rho_out, double *__restrict__ s_out,
                                                         double *__restrict__ partials, const Grid g,
                                                         const StepConsts<double> k, const uint32_t tiles_x,
                                                         const uint32_t tiles_y)
{
    using L = Lattice<LAT>;
    constexpr int NP = L::NP;
    __shared__ double red[kPartials][kRedThreads];
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const uint32_t tiles = tiles_x * tiles_y * (uint32_t)g.nz;
    double acc[kPartials] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (uint32_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int32_t x = (int32_t)((t % tiles_x) * blockDim.x + threadIdx.x);
        const int32_t y = (int32_t)(((t / tiles_x) % tiles_y) * blockDim.y + threadIdx.y);
        const int32_t z = (int32_t)(t / (tiles_x * tiles_y));
        if (x >= g.nx || y >= g.ny) continue;
        const Cell c = cell_of(g, x, y, z);
        const uint32_t lk = links ? links[c.own] : 0u;
        double rho = 0.0, ux = 0.0, uy = 0.0, uz = 0.0;
        if (!(lk & 1u)) {
            double gp[NP + 1], gm[NP + 1];
            gp[0] = (double)Conv<S>::ld(ld_pop(src, g, 0, own_ref(c)));
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const Slot sp = slot_plus<LAT>(c, p, lk), sm = slot_minus<LAT>(c, p, lk);
                gp[p + 1] = (double)Conv<S>::ld(ld_slot(src, g, sp));
                gm[p + 1] = (double)Conv<S>::ld(ld_slot(src, g, sm));
            }
            double drho, jx, jy, jz;
            moments_of<LAT>(gp, gm, drho, jx, jy, jz);
            rho = k.rho0 + drho;
            const double mx = jx + 0.5 * k.force[0], my = jy + 0.5 * k.force[1], mz = jz + 0.5 * k.force[2];
            ux = mx / rho;
            uy = my / rho;
            uz = mz / rho;
            acc[0] += drho;
            acc[1] += mx;
            acc[2] += my;
            acc[3] += (L::D == 3) ? mz : 0.0;
            acc[4] += 1.0;
        }
        if (rho_out) rho_out[c.own] = rho;
        if (s_out) {
            s_out[c.own] = ux;
            s_out[(size_t)g.n + c.own] = uy;
            if (L::D == 3) s_out[2 * (size_t)g.n + c.own] = uz;
        }
    }
    for (int m = 0; m < kPartials; ++m) red[m][tid] = acc[m];
    __syncthreads();
    for (int h = kRedThreads / 2; h > 0; h >>= 1) {
        if (tid < h)
            for (int m = 0; m < kPartials; ++m) red[m][tid] += red[m][tid + h];
        __syncthreads();
    }
    if (tid < kPartials) partials[kPartials * (size_t)blockIdx.x + tid] = red[tid][0];
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_partials(const double *__restrict__ partials, uint32_t nblocks,
                                                                 double *__restrict__ totals)
{
    __shared__ double red[kPartials][kRedThreads];
    const int tid = threadIdx.x;
    double acc[kPartials] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (uint32_t b = tid; b < nblocks; b += kRedThreads)
        for (int m = 0; m < kPartials; ++m) acc[m] += partials[kPartials * (size_t)b + m];
    for (int m = 0; m < kPartials; ++m) red[m][tid] = acc[m];
    __syncthreads();
    for (int h = kRedThreads / 2; h > 0; h >>= 1) {
        if (tid < h)
            for (int m = 0; m < kPartials; ++m) red[m][tid] += red[m][tid + h];
        __syncthreads();
    }
    if (tid < kPartials) totals[tid] = red[tid][0];
}

// Canonical-order permutations of the state (see the file header and Slot).
template <int LAT, typename S, int MODE>
__global__ __launch_bounds__(256) void k_permute(const void *__restrict__ in, void *__restrict__ out,
                                                 const uint32_t *__restrict__ links, const Grid g,
                                                 const StepConsts<double> k)
{
    using L = Lattice<LAT>;
    constexpr int NP = L::NP;
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t y = blockIdx.y * blockDim.y + threadIdx.y;
    const int32_t z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const Cell c = cell_of(g, x, y, z);
    const uint32_t lk = links ? links[c.own] : 0u;
    const bool solid = lk & 1u;
    auto move = [&](int i, Slot sl, double sigma) {
        if constexpr (MODE == 0) {
            st_at(plane((S *)out, i, g.n), c.own,
                  solid ? Conv<S>::st(typename Conv<S>::C(0)) : ld_slot((const S *)in, g, sl));
        } else if constexpr (MODE == 1) {
            if (!solid) st_slot((S *)out, g, sl, ld_at(plane((const S *)in, i, g.n), c.own));
        } else {
            // FP64 output: 8 bytes per cell, so 64-bit indexing (the storage-type planes above
            // stay below 4 GiB, this one need not)
            const double v = solid ? 0.0 : (double)Conv<S>::ld(ld_slot((const S *)in, g, sl)) + sigma;
            ((double *)out)[(size_t)i * g.n + c.own] = v;
        }
    };
    move(0, fixed_slot(0, own_ref(c)), k.sigma[0]);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        move(2 * p + 1, slot_plus<LAT>(c, p, lk), k.sigma[p + 1]);
        move(2 * p + 2, slot_minus<LAT>(c, p, lk), k.sigma[p + 1]);
    }
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// ---- the discrete adjoint ----------------------------------------------------------------------
//
// One forward step maps the pre-collision state f(t) to f(t+1) by
//   b_k  = (1 - w) f_k + w f^eq_k(rho, s) + [f^eq_k(rho, s') - f^eq_k(rho, s)]   (force: s' = s + F/rho)
//   f*_k = (1 - m) b_k + m f_opp(k)                                                 (gray cells)
//   f_k(t+1, x + c_k) = f*_k(x)
// with w = 1/tau. Its transpose takes the adjoint lam(t+1) of f(t+1) to lam(t):
//   mu_k(x) = lam_k(t+1, x + c_k),  nu_k = (1 - m) mu_k,
//   lam_i(t, x) = (1 - w) nu_i + a VJP_s(nu)_i + [VJP_s'(nu)_i] + m mu_opp(i),
// a = w without force and w - 1 with it, and VJP_s(nu)_i = sum_k nu_k d f^eq_k / d f_i =
// A0 + sum_a A_a (c_ia - s_a) / rho through rho = sum f and s = sum f c / rho. Parameter
// sensitivities accumulate per cell: d tau += -w^2 sum_k nu_k (f^eq_k - f_k),
// d K += a G_s(nu) [+ G_s'(nu)], d m += sum_k mu_k (f_opp(k) - b_k). All formulas are in terms
// of f; the stored deviations differ from f by constants, which cancel in every difference.

// Moments of the deviations nu_k - nu_0 of nu_k = keep mu_k from the rest direction's value
// nu_0, weighted by w_k over all q directions: M0 = sum w (nu - nu_0), M1_a, M2_ab likewise with
// c_a and c_a c_b, and the third moments that are not M1 on these lattices (c_a^3 = c_a):
// M3_aab (a != b) and M3_xyz. The moments of nu itself follow exactly: the constant nu_0 adds
// nu_0 to M0 and nu_0 cs^2 to the diagonal of M2 (sum w = 1, sum w c c = cs^2 I, odd moments of w
// vanish). nu_0 cancels exactly from the K-sensitivity and from d tau and d m, so these are
// formed from the deviations: their common part, often far larger than the direction-dependent
// part, then adds no rounding (in FP32 it otherwise dominated the tensor gradient's error). The
// moments do not depend on s, so one pass over the directions serves the transposed Jacobian at
// s and, with a force, at s + F / rho.
template <typename C> struct NuMoments {
    C ref;    // nu_0
    C m0;
    C m1[3];
    C m2[6];  // xx yy zz xy xz yz
    C m3[7];  // xxy xxz yyx yyz zzx zzy xyz
};

template <int LAT, typename C>
__device__ inline NuMoments<C> nu_moments(const StepConsts<C> &k, const C *mup, const C *mum, C keep)
{
    using L = Lattice<LAT>;
    NuMoments<C> m;
    m.ref = keep * mup[0];
    // every sum starts from its first term (IEEE arithmetic keeps a leading 0 + x as an
    // instruction); the flags are constants after unrolling
    bool b0 = false, b1[3] = {false, false, false}, b2[6] = {false, false, false, false, false, false};
    bool b3[7] = {false, false, false, false, false, false, false};
    const auto add = [](C &acc, bool &started, C v, bool neg) {
        acc = started ? (neg ? acc - v : acc + v) : (neg ? -v : v);
        started = true;
    };
    m.m0 = C(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) m.m1[a] = C(0);
#pragma unroll
    for (int e = 0; e < 6; ++e) m.m2[e] = C(0);
#pragma unroll
    for (int e = 0; e < 7; ++e) m.m3[e] = C(0);
#pragma unroll
    for (int p = 0; p < L::NP; ++p) {
        const PairRow v = L::pair(p);
        // even and odd parts of the pair, each formed from the raw pair first: where mu is
        // dominated by its odd part (a flux objective seeds mu_i = c_ix), mu+ + mu- is a small
        // difference of two large values and is exact before any scaling rounds it
        const C sum = fmad(keep, mup[p + 1] + mum[p + 1], C(-2) * m.ref) * k.w[p + 1];
        const C dif = (keep * (mup[p + 1] - mum[p + 1])) * k.w[p + 1];
        const int c[3] = {v.cx, v.cy, v.cz};
        add(m.m0, b0, sum, false);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (c[a] != 0) add(m.m1[a], b1[a], dif, c[a] < 0);
            if (c[a] != 0) add(m.m2[a], b2[a], sum, false);
        }
        const int ab[3][2] = {{0, 1}, {0, 2}, {1, 2}};
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const int cc = c[ab[e][0]] * c[ab[e][1]];
            if (cc != 0) add(m.m2[3 + e], b2[3 + e], sum, cc < 0);
        }
        // M3_aab: index 2a + (b > a ? b - 1 : b) over b != a, i.e. xxy xxz yyx yyz zzx zzy
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if (a == b || c[a] == 0 || c[b] == 0) continue;
                const int e = 2 * a + (b > a ? b - 1 : b);
                add(m.m3[e], b3[e], dif, c[b] < 0);
            }
        const int cxyz = c[0] * c[1] * c[2];
        if (cxyz != 0) add(m.m3[6], b3[6], dif, cxyz < 0);
    }
    return m;
}

// M3_abc from the stored entries (c_a^3 = c_a makes M3_aaa = M1_a).
template <typename C> __device__ inline C m3_at(const NuMoments<C> &m, int a, int b, int c)
{
    if (a == b && b == c) return m.m1[a];
    if (a != b && b != c && a != c) return m.m3[6];
    const int r = (a == b) ? a : (a == c ? a : b);  // the repeated index
    const int o = (a == b) ? c : (a == c ? b : a);  // the other one
    return m.m3[2 * r + (o > r ? o - 1 : o)];
}

// The contractions of K with the nu-moments, which do not depend on s: K:M2, (K:M3)_a =
// K_bc M3_bca and (K M1)_a. With a force the transposed Jacobian is taken at s and at s + F/rho
// from the same moments, so they are formed once per cell.
template <typename C> struct KContract {
    C KM2;
    C KM3[3];
    C KM1[3];
};

template <int D, int ORDER, typename C>
__device__ inline KContract<C> k_contract(const StepConsts<C> &k, const NuMoments<C> &m)
{
    const C Km[3][3] = {{k.k[0], k.k[3], k.k[4]}, {k.k[3], k.k[1], k.k[5]}, {k.k[4], k.k[5], k.k[2]}};
    const C rc = m.ref * C(1.0 / 3.0);
    const C M2[3][3] = {{m.m2[0] + rc, m.m2[3], m.m2[4]},
                        {m.m2[3], m.m2[1] + rc, m.m2[5]},
                        {m.m2[4], m.m2[5], D == 3 ? m.m2[2] + rc : m.m2[2]}};
    KContract<C> kc;
    kc.KM2 = C(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) kc.KM2 = fmad(Km[a][b], M2[a][b], kc.KM2);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        kc.KM3[a] = C(0);
        kc.KM1[a] = C(0);
        if constexpr (ORDER == 3) {
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int c = 0; c < 3; ++c) kc.KM3[a] = fmad(Km[b][c], m3_at(m, b, c, a), kc.KM3[a]);
            kc.KM1[a] = fmad(Km[a][0], m.m1[0], fmad(Km[a][1], m.m1[1], Km[a][2] * m.m1[2]));
        }
    }
    return kc;
}

// A0 = d/drho, A_a = d/ds_a (times rho) and the K-sensitivity G of sum_k nu_k f^eq_k(rho, s)
// for f^eq_k = rho r_k + w_k rho P'_k(s), from the nu-moments. With u = c.s, kc = c.(K s),
// r = w (1 + 1.5 c.K.c - 0.5 tr K) and P' = 4.5 u^2 - 1.5 |s|^2 + u (A - 4.5 |s|^2 + 4.5 u^2)
// - 3 kc, A = 3 + 4.5 c.K.c - 1.5 tr K (order 3; P' = 4.5 u^2 - 1.5 |s|^2 + 3 u at order 2):
//   sum nu f^eq / rho = M0 (1 - tr K / 2) + 1.5 K:M2 + 4.5 s.M2.s - 1.5 |s|^2 M0
//                       + (3 - 1.5 tr K) s.M1 + 4.5 s.(K:M3) - 4.5 |s|^2 s.M1 + 4.5 M3:sss
//                       - 3 M1.(K s).
// A0 and A take the moments of nu (M0 = nu_0 + D0, M2 = nu_0 cs^2 I + D2 over the lattice's d
// axes); G, in which nu_0 cancels (1.5 M2 - 0.5 M0 I), takes the deviation moments D0, D2.
// K is symmetric and every tensor gradient the library reports depends on G only through
// G + G^T, so G holds the symmetric part (G_ab + G_ba) / 2 as 6 entries xx, yy, zz, xy, xz, yz;
// add coef * G.
template <int D, int ORDER, typename C>
__device__ inline void moment_vjp(const StepConsts<C> &k, const NuMoments<C> &m, const KContract<C> &kc, C rho, C sx,
                                  C sy, C sz, C &A0, C &Ax, C &Ay, C &Az, C coef, C *G)
{
    const C s[3] = {sx, sy, sz};
    const C D2[3][3] = {{m.m2[0], m.m2[3], m.m2[4]}, {m.m2[3], m.m2[1], m.m2[5]}, {m.m2[4], m.m2[5], m.m2[2]}};
    const C rc = m.ref * C(1.0 / 3.0);
    const C M2[3][3] = {{D2[0][0] + rc, D2[0][1], D2[0][2]},
                        {D2[1][0], D2[1][1] + rc, D2[1][2]},
                        {D2[2][0], D2[2][1], D == 3 ? D2[2][2] + rc : D2[2][2]}};
    const C M0 = m.m0 + m.ref;
    const C trK = k.k[0] + k.k[1] + k.k[2];
    const C usq = fmad(sx, sx, fmad(sy, sy, sz * sz));
    C M2s[3], sM2s = C(0), sM1 = C(0);
    const C KM2 = kc.KM2;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        M2s[a] = fmad(M2[a][0], s[0], fmad(M2[a][1], s[1], M2[a][2] * s[2]));
        sM2s = fmad(s[a], M2s[a], sM2s);
        sM1 = fmad(s[a], m.m1[a], sM1);
    }
    const C base0 = fmad(C(-0.5) * trK, M0, M0);  // M0 (1 - tr K / 2)
    const C g = C(1.5) * fmad(C(-1), trK, C(2));  // 3 - 1.5 tr K
    C bracket = fmad(C(1.5), KM2, base0);
    bracket = fmad(C(4.5), sM2s, bracket);
    bracket = fmad(C(-1.5) * usq, M0, bracket);
    C Aa[3];
    const int ea[6] = {0, 1, 2, 0, 0, 1}, eb[6] = {0, 1, 2, 1, 2, 2};
    const C rcoef = rho * coef;
    if constexpr (ORDER == 3) {
        const C *KM3 = kc.KM3, *KM1 = kc.KM1;
        C M3ss[3], T3 = C(0), sKM3 = C(0), sKM1 = C(0);
        C M3s[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int b = 0; b < 3; ++b)
                M3s[a][b] = fmad(m3_at(m, a, b, 0), s[0], fmad(m3_at(m, a, b, 1), s[1], m3_at(m, a, b, 2) * s[2]));
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            M3ss[a] = fmad(M3s[a][0], s[0], fmad(M3s[a][1], s[1], M3s[a][2] * s[2]));
            T3 = fmad(s[a], M3ss[a], T3);
            sKM3 = fmad(s[a], KM3[a], sKM3);
            sKM1 = fmad(s[a], KM1[a], sKM1);
        }
        bracket = fmad(g, sM1, bracket);
        bracket = fmad(C(4.5), sKM3, bracket);
        bracket = fmad(C(-4.5) * usq, sM1, bracket);
        bracket = fmad(C(4.5), T3, bracket);
        bracket = fmad(C(-3), sKM1, bracket);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            C t = C(9) * M2s[a];
            t = fmad(C(-3) * s[a], M0, t);
            t = fmad(g, m.m1[a], t);
            t = fmad(C(4.5), KM3[a], t);
            t = fmad(C(-9) * s[a], sM1, t);
            t = fmad(C(-4.5) * usq, m.m1[a], t);
            t = fmad(C(13.5), M3ss[a], t);
            t = fmad(C(-3), KM1[a], t);
            Aa[a] = t;
        }
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const int a = ea[e], b = eb[e];
            C t = C(1.5) * D2[a][b];  // 1.5 M2 - 0.5 M0 I: nu_0 cancels
            if (a == b) t = fmad(C(-0.5), m.m0, fmad(C(-1.5), sM1, t));
            t = fmad(C(4.5), M3s[a][b], t);
            t -= C(1.5) * fmad(m.m1[a], s[b], m.m1[b] * s[a]);
            G[e] = fmad(rcoef, t, G[e]);
        }
    } else {
        bracket = fmad(C(3), sM1, bracket);
#pragma unroll
        for (int a = 0; a < 3; ++a) Aa[a] = fmad(C(9), M2s[a], fmad(C(-3) * s[a], M0, C(3) * m.m1[a]));
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const int a = ea[e], b = eb[e];
            C t = C(1.5) * D2[a][b];  // 1.5 M2 - 0.5 M0 I: nu_0 cancels
            if (a == b) t = fmad(C(-0.5), m.m0, t);
            G[e] = fmad(rcoef, t, G[e]);
        }
    }
    A0 = bracket;
    Ax = rho * Aa[0];
    Ay = rho * Aa[1];
    Az = rho * Aa[2];
}

constexpr int kGradPartials = 7;  // symmetric G (6) and d tau, per work-group

// Seed of the reverse sweep from the final state: lam_i = dJ / d f_i (skipped when lam is null,
// which leaves the evaluation of J alone), and the objective's partial sums, one per
// work-group. kind 0: flux through the plane x = plane_x, J = sum (j_x + F_x/2); kind 1: kinetic
// energy, J = sum |j + F/2|^2 / (2 rho). Like k_moments, the launch has a fixed number of
// work-groups that stride over the row tiles in a fixed order (reproducible sums).
template <int LAT, typename S>
__global__ __launch_bounds__(256) void k_seed(const S *__restrict__ src, typename Conv<S>::C *__restrict__ lam,
                                              double *__restrict__ jpart, const Grid g,
                                              const StepConsts<typename Conv<S>::C> k, const int kind, const int plane_x,
                                              const uint32_t *__restrict__ links, const uint32_t tiles_x,
                                              const uint32_t tiles_y)
{
    using L = Lattice<LAT>;
    using C = typename Conv<S>::C;
    constexpr int NP = L::NP;
    __shared__ double red[256];
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const uint32_t tiles = tiles_x * tiles_y * (uint32_t)g.nz;
    double jv = 0.0;
    for (uint32_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int32_t x = (int32_t)((t % tiles_x) * blockDim.x + threadIdx.x);
        const int32_t y = (int32_t)(((t / tiles_x) % tiles_y) * blockDim.y + threadIdx.y);
        const int32_t z = (int32_t)(t / (tiles_x * tiles_y));
        if (x >= g.nx || y >= g.ny) continue;
        const Cell c = cell_of(g, x, y, z);
        const uint32_t lk = links ? links[c.own] : 0u;
        C gp[NP + 1], gm[NP + 1];
        gp[0] = Conv<S>::ld(ld_pop(src, g, 0, own_ref(c)));
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const Slot sp = slot_plus<LAT>(c, p, lk), sm = slot_minus<LAT>(c, p, lk);
            gp[p + 1] = Conv<S>::ld(ld_slot(src, g, sp));
            gm[p + 1] = Conv<S>::ld(ld_slot(src, g, sm));
        }
        C drho, jx, jy, jz;
        moments_of<LAT>(gp, gm, drho, jx, jy, jz);
        const C rho = k.rho0 + drho;
        const C mx = jx + C(0.5) * k.force[0], my = jy + C(0.5) * k.force[1], mz = jz + C(0.5) * k.force[2];
        C base = C(0), ux = C(0), uy = C(0), uz = C(0);
        if (lk & 1u) {
            // a solid cell holds no fluid: it adds nothing to J (and its lam is never read)
        } else if (kind == 0) {
            if (x == plane_x) {
                ux = C(1);
                jv += (double)mx;
            }
        } else {
            ux = mx / rho;
            uy = my / rho;
            uz = mz / rho;
            base = C(-0.5) * fmad(ux, ux, fmad(uy, uy, uz * uz));
            jv += 0.5 * ((double)mx * mx + (double)my * my + (double)mz * mz) / (double)rho;
        }
        if (lam) {
            // lam_i = base + u . c_i
            st_pop(lam, g, 0, own_ref(c), base);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const PairRow v = L::pair(p);
                const C uc = (C)v.cx * ux + (C)v.cy * uy + (C)v.cz * uz;
                st_pop(lam, g, 2 * p + 1, own_ref(c), base + uc);
                st_pop(lam, g, 2 * p + 2, own_ref(c), base - uc);
            }
        }
    }
    red[tid] = jv;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0) jpart[blockIdx.x] = red[0];
}

// Where the adjoint of the post-collision population of direction +c (resp. -c) of pair p at x
// is read from lam(t+1): the slot of x + c (resp. x - c) in the same direction, or -- when that
// cell is solid and the population bounces back -- x's own slot of the opposite direction. The
// link word's bit for direction i marks x - c_i solid, so x + c is bit 2p+2 and x - c bit 2p+1.
template <int LAT> __device__ inline Slot adjoint_slot_plus(const Cell &c, int p, uint32_t links)
{
    const bool bounce = (links >> (2 * p + 2) & 1u) != 0u;
    return Slot{bounce, same_z(c, Lattice<LAT>::pair(p).cz), 2 * p + 2, 2 * p + 1, own_ref(c), src_minus<LAT>(c, p)};
}

template <int LAT> __device__ inline Slot adjoint_slot_minus(const Cell &c, int p, uint32_t links)
{
    const bool bounce = (links >> (2 * p + 1) & 1u) != 0u;
    return Slot{bounce, same_z(c, Lattice<LAT>::pair(p).cz), 2 * p + 1, 2 * p + 2, own_ref(c), src_plus<LAT>(c, p)};
}

// One reverse step at one cell: lam_in = lam(t+1) (canonical), state = the buffer whose gather
// gives f(t); writes lam(t) at the cell, adds d m to dmask and the cell's G / d tau to G, dtau.
// LINKS = false compiles the grid without solid cells (links is null): every slot is then a
// plain pull and the bounce-back selections drop out of the code.
template <int LAT, typename S, int ORDER, bool FORCED, bool LINKS>
__device__ inline void adjoint_cell(const S *__restrict__ state, const typename Conv<S>::C *__restrict__ lam_in,
                                    typename Conv<S>::C *__restrict__ lam_out, const float *__restrict__ gray,
                                    const uint32_t *__restrict__ links, double *__restrict__ dmask, const Grid &g,
                                    const StepConsts<typename Conv<S>::C> &k, int32_t x, int32_t y, int32_t z,
                                    typename Conv<S>::C *G, typename Conv<S>::C &dtau)
{
    using L = Lattice<LAT>;
    using C = typename Conv<S>::C;
    constexpr int NP = L::NP;
    const bool inside = x < g.nx && y < g.ny;
    const Cell c = cell_of(g, inside ? x : 0, inside ? y : 0, z);
    const uint32_t lk = (LINKS && inside && links) ? links[c.own] : 0u;
    const PlaneStores out = plane_stores(lam_out, g, own_ref(c));
    if (LINKS && inside && (lk & 1u)) {
        // a solid cell holds no state: its adjoint is zero and it adds no sensitivity
#pragma unroll
        for (int i = 0; i < L::Q; ++i) st_plane(out, i, C(0));
    } else if (inside) {
        // forward quantities at x (the canonical gather, bounce-back slots included)
        C gp[NP + 1], gm[NP + 1];
        // every input and output of a reverse step is touched once per launch: non-temporal loads
        // and stores (D3Q19 FP32 128^3: 94.5 -> 86.4-88.3 us against cached ones)
        gp[0] = Conv<S>::ld(ld_nt_at(pop_base(state, g, 0, own_ref(c)), own_ref(c).idx));
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const Slot sp = slot_plus<LAT>(c, p, lk), sm = slot_minus<LAT>(c, p, lk);
            gp[p + 1] = Conv<S>::ld(ld_slot_nt(state, g, sp));
            gm[p + 1] = Conv<S>::ld(ld_slot_nt(state, g, sm));
        }
        C drho, jx, jy, jz;
        moments_of<LAT>(gp, gm, drho, jx, jy, jz);
        const C rho = k.rho0 + drho;
        const C inv = C(1) / rho;
        const C sx = jx * inv, sy = jy * inv, sz = jz * inv;
        // adjoint of the post-collision populations: mu_k(x) = lam_k(t+1, x + c_k), or, when
        // x + c_k is solid (halfway bounce-back), lam_opp(k)(t+1, x)
        C mup[NP + 1], mum[NP + 1];
        mup[0] = ld_nt_at(pop_base(lam_in, g, 0, own_ref(c)), own_ref(c).idx);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const Slot ap = adjoint_slot_plus<LAT>(c, p, lk), am = adjoint_slot_minus<LAT>(c, p, lk);
            mup[p + 1] = ld_slot_nt(lam_in, g, ap);
            mum[p + 1] = ld_slot_nt(lam_in, g, am);
        }
        const C mg = gray ? (C)gray[c.own] : C(0);
        const C keep = C(1) - mg;  // nu_k = keep * mu_k
        const C w = k.omega;
        const C a = FORCED ? w - C(1) : w;
        // first pass over the directions: the transposed equilibrium Jacobian (and G)
        const NuMoments<C> nm = nu_moments<LAT>(k, mup, mum, keep);
        const KContract<C> kcn = k_contract<L::D, ORDER, C>(k, nm);
        C A0, Ax, Ay, Az;
        moment_vjp<L::D, ORDER, C>(k, nm, kcn, rho, sx, sy, sz, A0, Ax, Ay, Az, a, G);
        C base = a * (A0 - (Ax * sx + Ay * sy + Az * sz) * inv);
        C ax = a * Ax * inv, ay = a * Ay * inv, az = a * Az * inv;
        C tx = C(0), ty = C(0), tz = C(0);
        if constexpr (FORCED) {
            tx = (jx + k.force[0]) * inv;
            ty = (jy + k.force[1]) * inv;
            tz = (jz + k.force[2]) * inv;
            C B0, Bx, By, Bz;
            moment_vjp<L::D, ORDER, C>(k, nm, kcn, rho, tx, ty, tz, B0, Bx, By, Bz, C(1), G);
            base += B0 - (Bx * tx + By * ty + Bz * tz) * inv;
            ax += Bx * inv;
            ay += By * inv;
            az += Bz * inv;
        }
        // second pass: per direction the equilibrium again (cheaper than holding it in
        // registers), the post-BGK value b, d tau, d m and lam(t) at x
        __builtin_amdgcn_sched_barrier(0);
        const EqCell<C> e = eq_cell(k, drho, rho, sx, sy, sz);
        const EqCell<C> ef = eq_cell(k, drho, rho, tx, ty, tz);
        const C om = C(1) - w;
        C dm;
        // d tau = -w^2 sum_k nu_k (f^eq_k - f_k) and d m = sum_k mu_k (f_opp(k) - b_k): both
        // differences sum to zero over k (mass), so nu_0 and mu_0 drop out and the sums run over
        // nu_k - nu_0 and mu_k - mu_0 (the rest direction then adds nothing)
        dtau = C(0);
        dm = C(0);
        st_plane(out, 0, fmad(mg, mup[0], fmad(om, nm.ref, base)));
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            C ep, em;
            eq_pair<LAT, ORDER, C>(k, e, p, ep, em);
            const C dp = ep - gp[p + 1], dq = em - gm[p + 1];
            dtau = fmad(fmad(keep, mup[p + 1], -nm.ref), dp, dtau);
            dtau = fmad(fmad(keep, mum[p + 1], -nm.ref), dq, dtau);
            // b = g + w (g^eq - g), plus g^eq(s + F/rho) - g^eq(s) with the force:
            // b = (1 - w) (g - g^eq(s)) + g^eq(s + F/rho)
            C bp, bm;
            if constexpr (FORCED) {
                C fp, fm;
                eq_pair<LAT, ORDER, C>(k, ef, p, fp, fm);
                bp = fmad(-om, dp, fp);
                bm = fmad(-om, dq, fm);
            } else {
                bp = fmad(w, dp, gp[p + 1]);
                bm = fmad(w, dq, gm[p + 1]);
            }
            const PairRow v = L::pair(p);
            const C vc = (C)v.cx * ax + (C)v.cy * ay + (C)v.cz * az;
            st_plane(out, 2 * p + 1, fmad(mg, mum[p + 1], fmad(om, keep * mup[p + 1], base + vc)));
            st_plane(out, 2 * p + 2, fmad(mg, mup[p + 1], fmad(om, keep * mum[p + 1], base - vc)));
            dm = fmad(mup[p + 1] - mup[0], gm[p + 1] - bp, dm);
            dm = fmad(mum[p + 1] - mup[0], gp[p + 1] - bm, dm);
        }
        dtau *= -w * w;
        if (dmask) dmask[c.own] += (double)dm;
    }
}

// One reverse step over the grid, one row tile (a y-tile of one z-plane, 256 cells) per
// work-group: each lane's G / d tau go to FP64 and the work-group adds its sums to its own
// entries of gpart (in the same order every step, so the totals are reproducible). With no sums
// carried from row to row the D3Q19 FP32 kernel needs 113 VGPRs (4 waves per SIMD). Work-groups
// of several row tiles, carrying per-lane FP64 sums across the rows, measured slower at 128^3:
// 95 us per step for one row against 107.5 (2 rows), 109 (4) and 112 (11) with the sums in
// registers (138 VGPRs), and 103 (2 rows) with the sums in LDS.
template <int LAT, typename S, int ORDER, bool FORCED, bool LINKS>
__global__ __launch_bounds__(256) void k_adjoint(const S *__restrict__ state, const typename Conv<S>::C *__restrict__ lam_in,
                                                 typename Conv<S>::C *__restrict__ lam_out,
                                                 const float *__restrict__ gray, const uint32_t *__restrict__ links,
                                                 double *__restrict__ dmask, double *__restrict__ gpart, const Grid g,
                                                 const StepConsts<typename Conv<S>::C> k, const uint32_t tiles_x)
{
    using C = typename Conv<S>::C;
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const uint32_t tiles_y = ((uint32_t)g.ny + blockDim.y - 1u) / blockDim.y;
    const uint32_t f = blockIdx.x / tiles_x;  // the row tile: y-tile f % tiles_y of z-plane f / tiles_y
    const int32_t x = (int32_t)((blockIdx.x % tiles_x) * blockDim.x + threadIdx.x);
    const int32_t y = (int32_t)((f % tiles_y) * blockDim.y + threadIdx.y);
    const int32_t z = (int32_t)(f / tiles_y);
    C G[6] = {C(0), C(0), C(0), C(0), C(0), C(0)};
    C dtau = C(0);
    adjoint_cell<LAT, S, ORDER, FORCED, LINKS>(state, lam_in, lam_out, gray, links, dmask, g, k, x, y, z, G, dtau);
    // work-group sums of G and d tau through LDS in a fixed order: 224 lanes add 8 lane values
    // each, then one lane per quantity adds those 32 sums
    __shared__ double part[kGradPartials][256];
    __shared__ double part2[kGradPartials][32];
#pragma unroll
    for (int e = 0; e < 6; ++e) part[e][tid] = (double)G[e];
    part[6][tid] = (double)dtau;
    __syncthreads();
    if (tid < kGradPartials * 32) {
        const int e = tid >> 5, j = tid & 31;
        double t = part[e][j];
#pragma unroll
        for (int r = 1; r < 8; ++r) t += part[e][j + 32 * r];
        part2[e][j] = t;
    }
    __syncthreads();
    if (tid < kGradPartials) {
        double t = part2[tid][0];
#pragma unroll
        for (int j = 1; j < 32; ++j) t += part2[tid][j];
        gpart[kGradPartials * (size_t)blockIdx.x + tid] += t;
    }
}

// Sum of per-work-group partials (m values per block) in a fixed order.
__global__ __launch_bounds__(256) void k_sum_partials(const double *__restrict__ part, uint32_t nblocks, int m,
                                                      double *__restrict__ out)
{
    __shared__ double red[256];
    for (int e = 0; e < m; ++e) {
        double acc = 0.0;
        for (uint32_t b = threadIdx.x; b < nblocks; b += 256) acc += part[(size_t)m * b + e];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[e] = red[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_fill(double *__restrict__ p, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// ---- dispatch helpers ------------------------------------------------------------------------

template <typename F> hipError_t by_lattice(int lattice, F &&f)
{
    switch (lattice) {
    case kD2Q9: return f(std::integral_constant<int, kD2Q9>{});
    case kD3Q19: return f(std::integral_constant<int, kD3Q19>{});
    case kD3Q27: return f(std::integral_constant<int, kD3Q27>{});
    default: return hipErrorInvalidValue;
    }
}

template <typename F> hipError_t by_storage(int storage, F &&f)
{
    switch (storage) {
    case kF64: return f(double{});
    case kF32: return f(float{});
    case kF16: return f(_Float16{});
    case kBF16: return f(__bf16{});
    default: return hipErrorInvalidValue;
    }
}

dim3 cell_grid(const Grid &g, int bx, int by)
{
    return dim3((uint32_t)((g.nx + bx - 1) / bx), (uint32_t)((g.ny + by - 1) / by), (uint32_t)g.nz);
}

// Work-group shape of every kernel except the step: 256 threads spanning whole x rows where
// the grid allows (256 x 1, 128 x 2 or 64 x 4), so that each direction's loads and stores of a
// work-group are full row runs inside one population block.
dim3 row_block(const Grid &g)
{
    const int bx = g.nx > 128 ? 256 : (g.nx > 64 ? 128 : 64);
    return dim3((uint32_t)bx, (uint32_t)(256 / bx));
}

dim3 row_grid(const Grid &g)
{
    const dim3 b = row_block(g);
    return cell_grid(g, (int)b.x, (int)b.y);
}

}  // namespace

hipError_t launch_links(int lattice, const Grid &g, const uint8_t *mask, uint32_t *links, hipStream_t stream)
{
    return by_lattice(lattice, [&](auto lat) {
        constexpr int LAT = decltype(lat)::value;
        const dim3 grid = row_grid(g), block = row_block(g);
        hipLaunchKernelGGL((k_links<LAT>), grid, block, 0, stream, mask, links, g);
        return hipGetLastError();
    });
}

hipError_t launch_init(int lattice, int storage, int order, const Grid &g, const StepConsts<double> &k,
                       const double *rho, const double *s, const uint32_t *links, void *dst, hipStream_t stream)
{
    return by_lattice(lattice, [&](auto lat) {
        return by_storage(storage, [&](auto sv) {
            using S = decltype(sv);
            constexpr int LAT = decltype(lat)::value;
            const dim3 grid = row_grid(g), block = row_block(g);
            if (order == 2)
                hipLaunchKernelGGL((k_init<LAT, S, 2>), grid, block, 0, stream, rho, s, links, (S *)dst, g, k);
            else
                hipLaunchKernelGGL((k_init<LAT, S, 3>), grid, block, 0, stream, rho, s, links, (S *)dst, g, k);
            return hipGetLastError();
        });
    });
}

// LDS that a step launch reserves without using it (cap_lds), to cap the work-groups resident
// on a compute unit. Fewer work-groups in flight keep fewer rows' cache lines and HBM pages open
// at once. FP32 and FP64 streaming steps take stream_groups(q, sizeof(S)); measured on the
// D3Q19 256^3 lane-exchange step (us per step, uncapped -> capped):
//   FP32 at 4 per CU: 399.7 -> 390.7 (3: 390.8, 5: 394.0, 2: 429.7)
//   FP64 at 2 per CU: 832.7 -> 803.7 (3: 817.3, 4: 827.3)
// and D3Q27 256^3 FP32 at 3: 571.5 -> 556 (FP64 at 2: 1,205 -> 1,171.5), D2Q9 256 x 65536 FP64
// at 4: 378.9 -> 368.5. FP16 and BF16 lose with any cap (4 per CU: 198 -> 215 and 222 us; D3Q27
// FP16 at 5: no change): their steps issue more instructions per byte and need the waves, and so
// does the gray step of the gradient workload (D3Q19 FP32 128^3, 3 per CU: 2.6% slower).
// The FP32 links step (80 VGPRs, 6 resident) at 4 per CU: 4,962 -> 4,851 us on the 512^3
// porous medium (3: 4,890, 5: 4,882), where the extra work-groups re-fetched lines. Rows longer
// than a work-group (shifted pulls), FP32 at 4 per CU: 512^3 3,388 -> 3,339 us, 384^3 unchanged.
template <int LAT, typename S, int M> unsigned step_lds(unsigned threads)
{
    constexpr bool f32 = std::is_same<S, float>::value, f64 = std::is_same<S, double>::value;
    if (M == kLinks) {  // 4 work-groups of 256 lanes, the same lanes in smaller work-groups
        const unsigned n = 4u * 256u / threads, most = 32u / ((threads + 63u) / 64u);
        return f32 && n < most ? cap_lds(n) : 0u;
    }
    if (M == kPlain || M == kStream) return (f32 || f64) ? stream_lds(Lattice<LAT>::Q, sizeof(S), threads) : 0u;
    return 0u;
}

hipError_t launch_step(int lattice, int storage, int order, const Grid &g, const StepConsts<double> &k64,
                       const StepConsts<float> &k32, const uint32_t *links, const float *gray, const void *src,
                       void *dst, int block_x, int block_y, int flags, hipStream_t stream)
{
    return by_lattice(lattice, [&](auto lat) {
        return by_storage(storage, [&](auto sv) {
            using S = decltype(sv);
            using C = typename Conv<S>::C;
            constexpr int LAT = decltype(lat)::value;
            const StepConsts<C> *kc;
            if constexpr (sizeof(C) == 8) kc = &k64; else kc = &k32;
            const dim3 g3 = cell_grid(g, block_x, block_y), block(block_x, block_y);
            const unsigned threads = (unsigned)(block_x * block_y);
            TileMap m;
            m.tiles_x = g3.x;
            m.tiles_y = g3.y;
            m.nblocks = g3.x * g3.y * g3.z;
            m.xcd_slabs = (flags & kLaunchXcdSlabs) ? 1u : 0u;
            const dim3 grid(m.nblocks);
            const int mode = (flags & kLaunchStreamOnly) ? kStream
                             : gray ? kGray : ((links != nullptr || kc->forced) ? kLinks : kPlain);
            m.row_xcd = mode == kLinks ? 1u : 0u;
            // the lane-exchange pull needs work-groups of whole rows (see pull_aligned)
            const bool aligned = mode != kLinks && !(flags & kLaunchShiftedPull) && g.nx % 64 == 0 &&
                                 block_x == g.nx;
            const S *in = (const S *)src;
            S *out = (S *)dst;
#define LBM_STEP(O, M)                                                                                           \
    do {                                                                                                         \
        if constexpr (M != kLinks) {                                                                             \
            if (aligned) {                                                                                       \
                hipLaunchKernelGGL((k_step<LAT, S, O, M, kPullRows>), grid, block, (step_lds<LAT, S, M>(threads)),  \
                                   stream, in, out, g, *kc, m, links, gray);                                     \
                break;                                                                                           \
            }                                                                                                    \
        }                                                                                                        \
        hipLaunchKernelGGL((k_step<LAT, S, O, M, kPullShifted>), grid, block, (step_lds<LAT, S, M>(threads)), stream, in, out, g, \
                           *kc, m, links, gray);                                                                 \
    } while (0)
            if (mode == kStream) {
                LBM_STEP(3, kStream);
            } else if (order == 2) {
                if (mode == kGray) LBM_STEP(2, kGray);
                else if (mode == kLinks) LBM_STEP(2, kLinks);
                else LBM_STEP(2, kPlain);
            } else {
                if (mode == kGray) LBM_STEP(3, kGray);
                else if (mode == kLinks) LBM_STEP(3, kLinks);
                else LBM_STEP(3, kPlain);
            }
#undef LBM_STEP
            return hipGetLastError();
        });
    });
}

// The adjoint launch: one work-group per row tile, in a one-dimensional grid.
uint32_t adjoint_blocks(const Grid &g)
{
    const dim3 t = row_grid(g);
    return t.x * t.y * t.z;
}

uint32_t row_blocks(const Grid &g)
{
    const dim3 grid = row_grid(g);
    return grid.x * grid.y * grid.z;
}

uint32_t moments_groups(const Grid &g)
{
    const uint32_t t = row_blocks(g);
    return t < kMomentGroups ? t : kMomentGroups;
}

hipError_t launch_moments(int lattice, int storage, const Grid &g, const StepConsts<double> &k,
                          const uint32_t *links, const void *src, double *rho, double *s, double *partials,
                          double *totals, hipStream_t stream)
{
    return by_lattice(lattice, [&](auto lat) {
        return by_storage(storage, [&](auto sv) {
            using S = decltype(sv);
            constexpr int LAT = decltype(lat)::value;
            const dim3 tiles = row_grid(g), block = row_block(g);
            const uint32_t groups = moments_groups(g);
            hipLaunchKernelGGL((k_moments<LAT, S>), dim3(groups), block, 0, stream, (const S *)src, links, rho, s,
                               partials, g, k, tiles.x, tiles.y);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kRedThreads), 0, stream, partials, groups, totals);
            return hipGetLastError();
        });
    });
}

hipError_t launch_permute(int lattice, int storage, int mode, const Grid &g, const StepConsts<double> &k,
                          const uint32_t *links, const void *src, void *dst, hipStream_t stream)
{
    return by_lattice(lattice, [&](auto lat) {
        return by_storage(storage, [&](auto sv) {
            using S = decltype(sv);
            constexpr int LAT = decltype(lat)::value;
            const dim3 grid = row_grid(g), block = row_block(g);
            if (mode == 0)
                hipLaunchKernelGGL((k_permute<LAT, S, 0>), grid, block, 0, stream, src, dst, links, g, k);
            else if (mode == 1)
                hipLaunchKernelGGL((k_permute<LAT, S, 1>), grid, block, 0, stream, src, dst, links, g, k);
            else
                hipLaunchKernelGGL((k_permute<LAT, S, 2>), grid, block, 0, stream, src, dst, links, g, k);
            return hipGetLastError();
        });
    });
}

hipError_t launch_seed(int lattice, int storage, const Grid &g, const StepConsts<double> &k64,
                       const StepConsts<float> &k32, const void *src, void *lam, double *jpart, int kind, int plane,
                       const uint32_t *links, hipStream_t stream)
{
    return by_lattice(lattice, [&](auto lat) {
        return by_storage(storage, [&](auto sv) {
            using S = decltype(sv);
            using C = typename Conv<S>::C;
            constexpr int LAT = decltype(lat)::value;
            const StepConsts<C> *kc;
            if constexpr (sizeof(C) == 8) kc = &k64; else kc = &k32;
            const dim3 tiles = row_grid(g), block = row_block(g);
            hipLaunchKernelGGL((k_seed<LAT, S>), dim3(moments_groups(g)), block, 0, stream, (const S *)src, (C *)lam,
                               jpart, g, *kc, kind, plane, links, tiles.x, tiles.y);
            return hipGetLastError();
        });
    });
}

hipError_t launch_adjoint(int lattice, int storage, int order, const Grid &g, const StepConsts<double> &k64,
                          const StepConsts<float> &k32, const void *state, const void *lam_in, void *lam_out,
                          const float *gray, const uint32_t *links, double *dmask, double *gpart, hipStream_t stream)
{
    return by_lattice(lattice, [&](auto lat) {
        return by_storage(storage, [&](auto sv) {
            using S = decltype(sv);
            using C = typename Conv<S>::C;
            constexpr int LAT = decltype(lat)::value;
            const StepConsts<C> *kc;
            if constexpr (sizeof(C) == 8) kc = &k64; else kc = &k32;
            const dim3 grid(adjoint_blocks(g)), block = row_block(g);
            const uint32_t tiles_x = row_grid(g).x;
#define LBM_ADJ(O, F, L)                                                                                         \
    hipLaunchKernelGGL((k_adjoint<LAT, S, O, F, L>), grid, block, 0, stream, (const S *)state, (const C *)lam_in,  \
                       (C *)lam_out, gray, links, dmask, gpart, g, *kc, tiles_x)
#define LBM_ADJ_L(O, F)                                                                                          \
    do {                                                                                                         \
        if (links) LBM_ADJ(O, F, true); else LBM_ADJ(O, F, false);                                               \
    } while (0)
            if (order == 2) {
                if (kc->forced) LBM_ADJ_L(2, true); else LBM_ADJ_L(2, false);
            } else {
                if (kc->forced) LBM_ADJ_L(3, true); else LBM_ADJ_L(3, false);
            }
#undef LBM_ADJ_L
#undef LBM_ADJ
            return hipGetLastError();
        });
    });
}

hipError_t launch_sum(const double *part, uint32_t nblocks, int m, double *out, hipStream_t stream)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, stream, part, nblocks, m, out);
    return hipGetLastError();
}

hipError_t launch_zero(double *p, uint64_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, int64_t nbytes, hipStream_t stream)
{
    const uint64_t n = (uint64_t)nbytes / 16;
    if (n == 0) return hipSuccess;
    const uint64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_copy, dim3((uint32_t)blocks), dim3(256), 0, stream, (const u32x4 *)src, (u32x4 *)dst, n);
    return hipGetLastError();
}

}  // namespace lbm
