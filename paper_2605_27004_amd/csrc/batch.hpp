// batch.hpp -- types shared by the host side (batch.cpp) and the kernels (batch.hip) of the
// batched update: many independent periodic domains of uneven sizes, each with its own
// tensor and relaxation time, advanced together.
//
// Storage. Domain d owns a stretch of both population arrays starting at element `base`,
// holding its populations in linear blocks (FlatCell): block b holds canonical cells
// [b B, (b + 1) B) as q direction planes of B = 2^g.lb cells (8 KiB each, 32 KiB in FP64), and the last block
// is padded to B cells, so every domain and every tile of 256 cells starts on a whole cache
// line in every plane. Host arrays of rho and s concatenate the domains' cells (x fastest)
// without padding, from cell offset `cell0`.
//
// Work units. A tile is 256 consecutive cells of one domain (the last tile of a domain may be
// short). The step-per-launch mode runs one work-group per tile. The persistent mode hands
// each work-group a list of items -- a run of whole tiles of one domain -- and runs all steps
// in one launch; a domain's items meet at a per-domain arrival counter after every step.
#pragma once

#include <cstdint>

#include "common.hpp"

namespace lbm {

constexpr int kTileCells = 256;

struct BatchDomain {
    Grid g;            // extents and population layout of the domain
    uint32_t cells;    // nx * ny * nz
    uint32_t mx, my;   // floor(2^32 / nx), floor(2^32 / ny) (0xffffffff for 1): cell index -> x, y, z
    uint32_t tile0;    // first tile of this domain in the natural (domain-major) tile order
    uint32_t ntiles;
    uint32_t pad_;
    uint64_t base;     // element offset of the domain's plane 0 in each population array
    uint64_t cell0;    // offset of the domain's first cell in concatenated per-cell arrays
};

constexpr uint32_t kPadTile = 0xffffffffu;  // TileRec::dom of a padding tile (no work)

struct TileRec {
    uint32_t dom;
    uint32_t first;    // first cell of the tile within its domain
};

struct BatchItem {
    uint32_t dom;
    uint32_t first;    // first cell (a multiple of kTileCells)
    uint32_t count;    // cells
    uint32_t group;    // items of one group run all their steps before the next group starts
};

// ---- launchers (batch.hip); all enqueue on `stream` and never synchronise ----

// Per-domain constants: k64 / k32 arrays of StepConsts, one per domain.
hipError_t launch_batch_init(int lattice, int storage, int order, uint32_t ntiles, const TileRec *tiles,
                             const BatchDomain *doms, const StepConsts<double> *k64, const double *rho,
                             const double *s, uint64_t ncells, void *dst, hipStream_t stream);

// One step over the tiles in launch order `tiles` (ntiles work-groups).
hipError_t launch_batch_step(int lattice, int storage, int order, uint32_t ntiles, const TileRec *tiles,
                             const BatchDomain *doms, const StepConsts<double> *k64, const StepConsts<float> *k32,
                             const void *src, void *dst, hipStream_t stream);

struct PersistArgs {
    void *pop0, *pop1;
    uint32_t parity;          // step t reads pop[(parity + t) & 1] and writes the other
    int32_t nsteps;
    const BatchDomain *doms;
    const void *consts;       // StepConsts<C> [ndomains] in the arithmetic precision
    const BatchItem *items;
    const uint32_t *wg_first; // [nwg + 1] item ranges per work-group
    const uint32_t *chunks;   // [ndomains] items per domain and step
    uint32_t *ctr;            // [ndomains] arrival counters, zero at launch
    uint32_t *status;         // set to 1 by a work-group whose wait ran out of spins
    uint32_t spin_limit;      // polls of a counter before a wait gives up
};

// All steps in one cooperative launch of nwg work-groups.
hipError_t launch_batch_persist(int lattice, int storage, int order, uint32_t nwg, const PersistArgs &a,
                                hipStream_t stream);
// Work-groups of the persistent kernel that fit on one compute unit at once.
hipError_t batch_persist_occupancy(int lattice, int storage, int order, int *wg_per_cu);

// rho [ncells], s [3][ncells] (FP64, either may be null) and per-tile partial sums
// (drho, j_x, j_y, j_z), then per-domain totals [ndomains][4] in a fixed order.
hipError_t launch_batch_moments(int lattice, int storage, uint32_t ntiles, const TileRec *tiles,
                                const BatchDomain *doms, const StepConsts<double> *k64, const void *src,
                                double *rho, double *s, uint64_t ncells, double *partials, uint32_t ndomains,
                                double *totals, hipStream_t stream);

// Canonical pre-collision f in FP64: domain d at out + q * cell0_d, [q][cells_d].
hipError_t launch_batch_export(int lattice, int storage, uint32_t ntiles, const TileRec *tiles,
                               const BatchDomain *doms, const StepConsts<double> *k64, const void *src, double *out,
                               hipStream_t stream);

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, hipStream_t stream);

}  // namespace lbm
