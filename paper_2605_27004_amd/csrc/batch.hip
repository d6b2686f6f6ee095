// batch.hip -- gfx950 kernels of the batched update: many independent periodic domains of
// uneven sizes, each with its own tensor and relaxation time (per-domain StepConsts), in one
// population array pair (layout in batch.hpp).
//
// Every cell update is the single-grid update of eq:LBE_BGK (pull gather along -c_i, the
// folded anisotropic equilibrium, BGK, streaming store) through the same per-cell functions,
// so a domain advanced here is bitwise the same as that domain advanced alone.
//
// Two ways to run the steps:
//  * one launch per step, one work-group per 256-cell tile, in a tile order the host chooses
//    (domain-to-XCD placement: flat work-group b runs on XCD b mod 8);
//  * one persistent cooperative launch for all steps: work-group w owns a fixed list of
//    items (runs of whole tiles of one domain) and, for every step, processes its items in
//    order. Before it touches a domain at step t it waits until every item of that domain has
//    arrived from step t-1 (a per-domain counter in global memory); after writing an item it
//    arrives. The wait/arrive pair also orders the overwrite of step t-1's source, so two
//    buffers suffice. Every wait is bounded: on running out of spins a work-group raises the
//    status word and returns, and the others return at their next poll.
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "cell.hpp"

#pragma clang fp contract(off)

namespace lbm {
namespace {

using namespace cell;

// Cell n (x fastest) of a domain; a tile may span z-planes, so batched domains use one 32-bit
// index over the domain's whole block of the population arrays.
__device__ inline FlatCell batch_cell(const BatchDomain &dm, uint32_t n)
{
    uint32_t x, y;
    const uint32_t r = div_by(n, dm.mx, (uint32_t)dm.g.nx, x);
    const uint32_t z = div_by(r, dm.my, (uint32_t)dm.g.ny, y);
    return flat_cell_of(dm.g, x, y, z);
}

// One periodic cell update: q pulls, the collision, q streaming stores.
template <int LAT, typename S, int ORDER>
__device__ inline void step_cell(const S *__restrict__ src, S *__restrict__ dst, const Grid &g, const FlatCell &c,
                                 const StepConsts<typename Conv<S>::C> &k)
{
    using C = typename Conv<S>::C;
    constexpr int NP = Lattice<LAT>::NP;
    constexpr PullOrder<LAT> kPull{};
    C gp[NP + 1], gm[NP + 1];
#pragma unroll
    for (int j = 0; j < Lattice<LAT>::Q; ++j) {
        const int i = kPull.dir[j], p = (i - 1) / 2;
        if (i == 0)
            gp[0] = Conv<S>::ld(ld_pop(src, g, 0, own_ref(c)));
        else if (i & 1)
            gp[p + 1] = Conv<S>::ld(ld_pop(src, g, i, src_plus<LAT>(c, p)));
        else
            gm[p + 1] = Conv<S>::ld(ld_pop(src, g, i, src_minus<LAT>(c, p)));
    }
    collide_cell<LAT, ORDER, false, C, kClose<S>>(k, gp, gm);
    const PlaneStores ps = plane_stores(dst, g, own_ref(c));
    st_plane(ps, 0, Conv<S>::st(gp[0]));
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        st_plane(ps, 2 * p + 1, Conv<S>::st(gp[p + 1]));
        st_plane(ps, 2 * p + 2, Conv<S>::st(gm[p + 1]));
    }
}

template <int LAT, typename S, int ORDER>
__global__ __launch_bounds__(kTileCells) void k_batch_step(const S *__restrict__ src, S *__restrict__ dst,
                                                           const TileRec *__restrict__ tiles,
                                                           const BatchDomain *__restrict__ doms,
                                                           const StepConsts<typename Conv<S>::C> *__restrict__ kc)
{
    const TileRec t = tiles[blockIdx.x];
    if (t.dom == kPadTile) return;  // padding of an XCD-placed order
    const BatchDomain dm = doms[t.dom];
    const uint32_t n = t.first + threadIdx.x;
    if (n >= dm.cells) return;
    const StepConsts<typename Conv<S>::C> k = kc[t.dom];
    step_cell<LAT, S, ORDER>(src + dm.base, dst + dm.base, dm.g, batch_cell(dm, n), k);
}

// ---- the persistent launch ------------------------------------------------------------------

// Block until *ctr >= target (every item of the domain has arrived from the previous step).
// Returns false, with the status word raised, when the wait runs out of spins or another
// work-group has already raised it; all threads of the work-group get the same answer. One
// lane polls and then acquires at device scope (invalidating this compute unit's vector cache
// and the XCD's stale L2 lines); the barrier then releases the whole work-group, whose waves
// share that cache.
__device__ inline bool wait_arrivals(uint32_t *ctr, uint32_t target, uint32_t *status, uint32_t spin_limit,
                                     uint32_t &shared_ok)
{
    if (threadIdx.x == 0) {
        uint32_t ok = 1u, spins = 0u;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++spins > spin_limit) {
                ok = 0u;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (!ok) __hip_atomic_store(status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        shared_ok = ok;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return shared_ok != 0u;
}

// Publish this work-group's stores of the item and count it as arrived: every wave waits for
// its own stores to reach the L2 (vmcnt = 0), then one lane releases at device scope (the L2
// write-back that makes them visible to the other XCDs) and increments the counter. One
// release per work-group instead of one per wave measured 1.56 -> 1.12 ms per step on the
// 512-domain batch.
__device__ inline void arrive(uint32_t *ctr)
{
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0) expcnt(7) lgkmcnt(15)
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __builtin_amdgcn_s_waitcnt(0x0F70);  // the write-back completes before the counter moves
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The read-only tables come as separate restrict-qualified arguments: the compiler may then
// read them through scalar loads into scalar registers (they cannot alias the stores), which
// took the kernel from 126 to 82 VGPRs.
template <int LAT, typename S, int ORDER>
__global__ __launch_bounds__(kTileCells) void k_batch_persist(
    void *pop0, void *pop1, const uint32_t parity, const int32_t nsteps, const BatchDomain *__restrict__ doms,
    const StepConsts<typename Conv<S>::C> *__restrict__ kc, const BatchItem *__restrict__ items,
    const uint32_t *__restrict__ wg_first, const uint32_t *__restrict__ chunks, uint32_t *ctr, uint32_t *status,
    const uint32_t spin_limit)
{
    using C = typename Conv<S>::C;
    __shared__ uint32_t shared_ok;
    const uint32_t i1 = wg_first[blockIdx.x + 1];
    uint32_t ga = wg_first[blockIdx.x];
    while (ga < i1) {
        // the run [ga, gb) of this work-group's items that belong to one group
        const uint32_t grp = __builtin_amdgcn_readfirstlane(items[ga].group);
        uint32_t gb = ga + 1u;
        while (gb < i1 && __builtin_amdgcn_readfirstlane(items[gb].group) == grp) ++gb;
        for (int32_t t = 0; t < nsteps; ++t) {
            const bool odd = ((parity + (uint32_t)t) & 1u) != 0u;
            const S *src = (const S *)(odd ? pop1 : pop0);
            S *dst = (S *)(odd ? pop0 : pop1);
            for (uint32_t it = ga; it < gb; ++it) {
                // the item is the same for every lane: its fields (and through them the
                // domain's descriptor and constants) stay in scalar registers
                const uint32_t dom = __builtin_amdgcn_readfirstlane(items[it].dom);
                const uint32_t first = __builtin_amdgcn_readfirstlane(items[it].first);
                const uint32_t count = __builtin_amdgcn_readfirstlane(items[it].count);
                if (t > 0 && !wait_arrivals(ctr + dom, chunks[dom] * (uint32_t)t, status, spin_limit, shared_ok))
                    return;
                const BatchDomain dm = doms[dom];
                const StepConsts<C> k = kc[dom];
                for (uint32_t off = threadIdx.x; off < count; off += kTileCells)
                    step_cell<LAT, S, ORDER>(src + dm.base, dst + dm.base, dm.g, batch_cell(dm, first + off), k);
                arrive(ctr + dom);
            }
        }
        ga = gb;
    }
}

// ---- init, read-out, export ---------------------------------------------------------------------

// f_i(0, x) = f^eq_i(rho(x), s(x)) in FP64, stored as a deviation in the slot the canonical
// gather reads for direction i at x.
template <int LAT, typename S, int ORDER>
__global__ __launch_bounds__(kTileCells) void k_batch_init(const TileRec *__restrict__ tiles,
                                                           const BatchDomain *__restrict__ doms,
                                                           const StepConsts<double> *__restrict__ kc,
                                                           const double *__restrict__ rho_in,
                                                           const double *__restrict__ s_in, uint64_t ncells,
                                                           S *__restrict__ dst)
{
    using L = Lattice<LAT>;
    using C = typename Conv<S>::C;
    constexpr int NP = L::NP;
    const TileRec t = tiles[blockIdx.x];
    const BatchDomain dm = doms[t.dom];
    const uint32_t n = t.first + threadIdx.x;
    if (n >= dm.cells) return;
    const StepConsts<double> &k = kc[t.dom];
    const FlatCell c = batch_cell(dm, n);
    const uint64_t at = dm.cell0 + n;
    const double rho = rho_in[at];
    const double sx = s_in[at], sy = s_in[ncells + at];
    const double sz = (L::D == 3) ? s_in[2 * ncells + at] : 0.0;
    double eqp[NP + 1], eqm[NP + 1];
    equilibrium_pairs<LAT, ORDER, double>(k, rho - k.rho0, rho, sx, sy, sz, eqp, eqm);
    S *out = dst + dm.base;
    st_pop(out, dm.g, 0, own_ref(c), Conv<S>::st((C)eqp[0]));
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        st_pop(out, dm.g, 2 * p + 1, src_plus<LAT>(c, p), Conv<S>::st((C)eqp[p + 1]));
        st_pop(out, dm.g, 2 * p + 2, src_minus<LAT>(c, p), Conv<S>::st((C)eqm[p + 1]));
    }
}

constexpr int kBatchPartials = 4;  // drho, j_x, j_y, j_z

template <int LAT, typename S>
__global__ __launch_bounds__(kTileCells) void k_batch_moments(const TileRec *__restrict__ tiles,
                                                              const BatchDomain *__restrict__ doms,
                                                              const StepConsts<double> *__restrict__ kc,
                                                              const S *__restrict__ src, double *__restrict__ rho_out,
                                                              double *__restrict__ s_out, uint64_t ncells,
                                                              double *__restrict__ partials)
{
    using L = Lattice<LAT>;
    constexpr int NP = L::NP;
    __shared__ double red[kBatchPartials][kTileCells];
    const TileRec t = tiles[blockIdx.x];
    const BatchDomain dm = doms[t.dom];
    const uint32_t n = t.first + threadIdx.x;
    double acc[kBatchPartials] = {0.0, 0.0, 0.0, 0.0};
    if (n < dm.cells) {
        const FlatCell c = batch_cell(dm, n);
        const S *in = src + dm.base;
        double gp[NP + 1], gm[NP + 1];
        gp[0] = (double)Conv<S>::ld(ld_pop(in, dm.g, 0, own_ref(c)));
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            gp[p + 1] = (double)Conv<S>::ld(ld_pop(in, dm.g, 2 * p + 1, src_plus<LAT>(c, p)));
            gm[p + 1] = (double)Conv<S>::ld(ld_pop(in, dm.g, 2 * p + 2, src_minus<LAT>(c, p)));
        }
        double drho, jx, jy, jz;
        moments_of<LAT>(gp, gm, drho, jx, jy, jz);
        const double rho = kc[t.dom].rho0 + drho;
        const uint64_t at = dm.cell0 + n;
        if (rho_out) rho_out[at] = rho;
        if (s_out) {
            s_out[at] = jx / rho;
            s_out[ncells + at] = jy / rho;
            if (L::D == 3) s_out[2 * ncells + at] = jz / rho;
        }
        acc[0] = drho;
        acc[1] = jx;
        acc[2] = jy;
        acc[3] = (L::D == 3) ? jz : 0.0;
    }
    for (int m = 0; m < kBatchPartials; ++m) red[m][threadIdx.x] = acc[m];
    __syncthreads();
    for (int h = kTileCells / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int m = 0; m < kBatchPartials; ++m) red[m][threadIdx.x] += red[m][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < kBatchPartials) partials[kBatchPartials * (size_t)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// Per-domain totals: work-group d sums the partials of the domain's tiles in a fixed order.
__global__ __launch_bounds__(kTileCells) void k_batch_reduce(const BatchDomain *__restrict__ doms,
                                                             const double *__restrict__ partials,
                                                             double *__restrict__ totals)
{
    __shared__ double red[kBatchPartials][kTileCells];
    const BatchDomain dm = doms[blockIdx.x];
    double acc[kBatchPartials] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t b = threadIdx.x; b < dm.ntiles; b += kTileCells)
        for (int m = 0; m < kBatchPartials; ++m) acc[m] += partials[kBatchPartials * (size_t)(dm.tile0 + b) + m];
    for (int m = 0; m < kBatchPartials; ++m) red[m][threadIdx.x] = acc[m];
    __syncthreads();
    for (int h = kTileCells / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int m = 0; m < kBatchPartials; ++m) red[m][threadIdx.x] += red[m][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < kBatchPartials) totals[kBatchPartials * (size_t)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

template <int LAT, typename S>
__global__ __launch_bounds__(kTileCells) void k_batch_export(const TileRec *__restrict__ tiles,
                                                             const BatchDomain *__restrict__ doms,
                                                             const StepConsts<double> *__restrict__ kc,
                                                             const S *__restrict__ src, double *__restrict__ out)
{
    using L = Lattice<LAT>;
    constexpr int NP = L::NP;
    const TileRec t = tiles[blockIdx.x];
    const BatchDomain dm = doms[t.dom];
    const uint32_t n = t.first + threadIdx.x;
    if (n >= dm.cells) return;
    const StepConsts<double> &k = kc[t.dom];
    const FlatCell c = batch_cell(dm, n);
    const S *in = src + dm.base;
    double *o = out + (uint64_t)L::Q * dm.cell0;
    o[n] = (double)Conv<S>::ld(ld_pop(in, dm.g, 0, own_ref(c))) + k.sigma[0];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        o[(uint64_t)(2 * p + 1) * dm.cells + n] =
            (double)Conv<S>::ld(ld_pop(in, dm.g, 2 * p + 1, src_plus<LAT>(c, p))) + k.sigma[p + 1];
        o[(uint64_t)(2 * p + 2) * dm.cells + n] =
            (double)Conv<S>::ld(ld_pop(in, dm.g, 2 * p + 2, src_minus<LAT>(c, p))) + k.sigma[p + 1];
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ---- dispatch -------------------------------------------------------------------------------------

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

template <typename F> hipError_t by_order(int order, F &&f)
{
    return order == 2 ? f(std::integral_constant<int, 2>{}) : f(std::integral_constant<int, 3>{});
}

}  // namespace

hipError_t launch_batch_init(int lattice, int storage, int order, uint32_t ntiles, const TileRec *tiles,
                             const BatchDomain *doms, const StepConsts<double> *k64, const double *rho,
                             const double *s, uint64_t ncells, void *dst, hipStream_t stream)
{
    if (ntiles == 0) return hipSuccess;
    return by_lattice(lattice, [&](auto lat) {
        return by_storage(storage, [&](auto sv) {
            return by_order(order, [&](auto ord) {
                using S = decltype(sv);
                hipLaunchKernelGGL((k_batch_init<decltype(lat)::value, S, decltype(ord)::value>), dim3(ntiles),
                                   dim3(kTileCells), 0, stream, tiles, doms, k64, rho, s, ncells, (S *)dst);
                return hipGetLastError();
            });
        });
    });
}

hipError_t launch_batch_step(int lattice, int storage, int order, uint32_t ntiles, const TileRec *tiles,
                             const BatchDomain *doms, const StepConsts<double> *k64, const StepConsts<float> *k32,
                             const void *src, void *dst, hipStream_t stream)
{
    if (ntiles == 0) return hipSuccess;
    return by_lattice(lattice, [&](auto lat) {
        return by_storage(storage, [&](auto sv) {
            return by_order(order, [&](auto ord) {
                using S = decltype(sv);
                using C = typename Conv<S>::C;
                const StepConsts<C> *kc;
                if constexpr (sizeof(C) == 8) kc = k64; else kc = k32;
                // FP32 / FP64: the resident work-groups of a single-grid step (stream_groups, reserved
                // LDS); 512 D3Q19 FP32 domains 817 -> 785 us per step at 4 (3: 842, 5: 802)
                constexpr bool wide = std::is_same<S, float>::value || std::is_same<S, double>::value;
                const unsigned lds = wide ? stream_lds(Lattice<decltype(lat)::value>::Q, sizeof(S)) : 0u;
                hipLaunchKernelGGL((k_batch_step<decltype(lat)::value, S, decltype(ord)::value>), dim3(ntiles),
                                   dim3(kTileCells), lds, stream, (const S *)src, (S *)dst, tiles, doms, kc);
                return hipGetLastError();
            });
        });
    });
}

hipError_t launch_batch_persist(int lattice, int storage, int order, uint32_t nwg, const PersistArgs &a,
                                hipStream_t stream)
{
    if (nwg == 0) return hipSuccess;
    return by_lattice(lattice, [&](auto lat) {
        return by_storage(storage, [&](auto sv) {
            return by_order(order, [&](auto ord) {
                using S = decltype(sv);
                using C = typename Conv<S>::C;
                void *pop0 = a.pop0, *pop1 = a.pop1;
                uint32_t parity = a.parity, spin = a.spin_limit;
                int32_t nsteps = a.nsteps;
                const BatchDomain *doms = a.doms;
                const StepConsts<C> *kc = (const StepConsts<C> *)a.consts;
                const BatchItem *items = a.items;
                const uint32_t *wg_first = a.wg_first, *chunks = a.chunks;
                uint32_t *ctr = a.ctr, *status = a.status;
                void *kargs[] = {(void *)&pop0,  (void *)&pop1,     (void *)&parity, (void *)&nsteps,
                                 (void *)&doms,  (void *)&kc,       (void *)&items,  (void *)&wg_first,
                                 (void *)&chunks, (void *)&ctr,     (void *)&status, (void *)&spin};
                return hipLaunchCooperativeKernel(
                    reinterpret_cast<const void *>(&k_batch_persist<decltype(lat)::value, S, decltype(ord)::value>),
                    dim3(nwg), dim3(kTileCells), kargs, 0, stream);
            });
        });
    });
}

hipError_t batch_persist_occupancy(int lattice, int storage, int order, int *wg_per_cu)
{
    return by_lattice(lattice, [&](auto lat) {
        return by_storage(storage, [&](auto sv) {
            return by_order(order, [&](auto ord) {
                using S = decltype(sv);
                return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    wg_per_cu, k_batch_persist<decltype(lat)::value, S, decltype(ord)::value>, kTileCells, 0);
            });
        });
    });
}

hipError_t launch_batch_moments(int lattice, int storage, uint32_t ntiles, const TileRec *tiles,
                                const BatchDomain *doms, const StepConsts<double> *k64, const void *src,
                                double *rho, double *s, uint64_t ncells, double *partials, uint32_t ndomains,
                                double *totals, hipStream_t stream)
{
    if (ntiles == 0) return hipSuccess;
    return by_lattice(lattice, [&](auto lat) {
        return by_storage(storage, [&](auto sv) {
            using S = decltype(sv);
            hipLaunchKernelGGL((k_batch_moments<decltype(lat)::value, S>), dim3(ntiles), dim3(kTileCells), 0, stream,
                               tiles, doms, k64, (const S *)src, rho, s, ncells, partials);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess || ndomains == 0) return e;
            hipLaunchKernelGGL(k_batch_reduce, dim3(ndomains), dim3(kTileCells), 0, stream, doms, partials, totals);
            return hipGetLastError();
        });
    });
}

hipError_t launch_batch_export(int lattice, int storage, uint32_t ntiles, const TileRec *tiles,
                               const BatchDomain *doms, const StepConsts<double> *k64, const void *src, double *out,
                               hipStream_t stream)
{
    if (ntiles == 0) return hipSuccess;
    return by_lattice(lattice, [&](auto lat) {
        return by_storage(storage, [&](auto sv) {
            using S = decltype(sv);
            hipLaunchKernelGGL((k_batch_export<decltype(lat)::value, S>), dim3(ntiles), dim3(kTileCells), 0, stream,
                               tiles, doms, k64, (const S *)src, out);
            return hipGetLastError();
        });
    });
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

}  // namespace lbm
