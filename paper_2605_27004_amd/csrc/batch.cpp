// batch.cpp -- host side of the batched C ABI (lbm_batch_* in include/lbm.h): validation of
// every domain, the storage plan, the work schedules (tile orders and the persistent
// work-group lists, balanced by longest-processing-time-first assignment) and the autotuner
// that picks among them by measurement. No device memory is allocated here.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <queue>
#include <string>
#include <utility>
#include <vector>

#include "../../include/lbm.h"
#include "batch.hpp"
#include "common.hpp"
#include "host.hpp"

using namespace lbm;
using namespace lbm::host;

namespace {

constexpr int64_t kMaxWorkGroups = 16384;      // persistent grid bound (work-group lists in scratch)
constexpr int64_t kMaxDomains = 1 << 24;
constexpr uint32_t kDefaultSpinLimit = 1u << 20;

// Everything that follows from the parameters alone.
struct Plan {
    int lattice = 0, storage = 0, order = 3, q = 0, d = 0, bytes = 0;
    double rho0 = 1.0;
    std::vector<lbm_params> params;
    std::vector<Prepared> prep;
    std::vector<BatchDomain> dom;
    std::vector<TileRec> tiles;  // natural order: domain-major
    int64_t cells = 0;           // total cells C
    int64_t pop_elems = 0;       // elements of one population array
};

int plan_of(const lbm_batch_params *p, Plan &pl)
{
    if (!p) return fail(LBM_ERR_ARG, "params is NULL");
    if (p->ndomains < 1 || p->ndomains > kMaxDomains)
        return fail(LBM_ERR_ARG, "ndomains must be in 1 .. 2^24 (got %lld)", (long long)p->ndomains);
    if (!p->domains) return fail(LBM_ERR_ARG, "domains is NULL");
    pl.lattice = p->lattice;
    pl.storage = p->storage;
    pl.order = p->order;
    pl.rho0 = p->rho0;
    pl.params.resize((size_t)p->ndomains);
    pl.prep.resize((size_t)p->ndomains);
    pl.dom.resize((size_t)p->ndomains);
    int64_t base = 0, cell0 = 0, tile0 = 0;
    for (int64_t i = 0; i < p->ndomains; ++i) {
        const lbm_domain &dm = p->domains[i];
        if (dm.reserved != 0) return fail(LBM_ERR_ARG, "domain %lld: reserved must be 0", (long long)i);
        lbm_params &q = pl.params[(size_t)i];
        std::memset(&q, 0, sizeof q);
        q.lattice = p->lattice;
        q.storage = p->storage;
        q.order = p->order;
        q.tensor_kind = dm.tensor_kind;
        q.shift_kind = p->shift_kind;
        q.flags = 0;
        q.nx = dm.nx;
        q.ny = dm.ny;
        q.nz = dm.nz;
        std::memcpy(q.tensor, dm.tensor, sizeof q.tensor);
        q.tau = dm.tau;
        q.rho0 = p->rho0;
        const int rc = prepare(&q, pl.prep[(size_t)i]);
        if (rc) {
            g_last_error = "domain " + std::to_string((long long)i) + ": " + g_last_error;
            return rc;
        }
        const Prepared &pr = pl.prep[(size_t)i];
        pl.q = pr.q;
        pl.d = pr.d;
        pl.bytes = pr.bytes;
        BatchDomain &b = pl.dom[(size_t)i];
        std::memset(&b, 0, sizeof b);
        const int64_t n = (int64_t)pr.n;
        // a domain is addressed with one 32-bit byte offset (tiles may span its z-planes)
        // linear blocks of block_bytes per direction plane (a power of two >= the 256-cell tile)
        const int64_t block = block_bytes(pr.bytes) / pr.bytes;
        int lb = 0;
        while ((int64_t)1 << lb < block) ++lb;
        const int64_t elems = (n + block - 1) / block * block * pr.q;
        b.g = grid_of(dm.nx, dm.ny, dm.nz, pr.q, pr.bytes);
        b.g.lb = (uint32_t)lb;
        b.g.bc = (uint32_t)block;
        b.g.bq = (uint32_t)(pr.q * block);
        if ((double)elems * pr.bytes >= 4294967296.0)
            return fail(LBM_ERR_SIZE, "domain %lld holds 4 GiB or more of populations", (long long)i);
        b.cells = pr.n;
        b.mx = dm.nx == 1 ? 0xffffffffu : (uint32_t)(4294967296.0 / (double)dm.nx);
        b.my = dm.ny == 1 ? 0xffffffffu : (uint32_t)(4294967296.0 / (double)dm.ny);
        // floor(2^32 / d) exactly (the double quotient can round up at the last bit)
        if (dm.nx > 1 && (uint64_t)b.mx * (uint64_t)dm.nx > 4294967296ull) --b.mx;
        if (dm.ny > 1 && (uint64_t)b.my * (uint64_t)dm.ny > 4294967296ull) --b.my;
        const int64_t nt = (n + kTileCells - 1) / kTileCells;
        b.tile0 = (uint32_t)tile0;
        b.ntiles = (uint32_t)nt;
        b.base = (uint64_t)base;
        b.cell0 = (uint64_t)cell0;
        for (int64_t t = 0; t < nt; ++t) pl.tiles.push_back(TileRec{(uint32_t)i, (uint32_t)(t * kTileCells)});
        base += elems;
        cell0 += n;
        tile0 += nt;
        if (tile0 >= 2147483647LL) return fail(LBM_ERR_SIZE, "batch exceeds 2^31 tiles");
    }
    pl.cells = cell0;
    pl.pop_elems = base;
    return LBM_OK;
}

struct ScratchLayout {
    int64_t dom, k64, k32, tiles_nat, tiles_launch, items, wg_first, chunks, ctr, status, partials, totals, total;
};

ScratchLayout layout_of(const Plan &pl)
{
    const int64_t nd = (int64_t)pl.dom.size(), nt = (int64_t)pl.tiles.size();
    ScratchLayout l;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = off;
        off += align256(bytes);
        return at;
    };
    l.dom = take(nd * (int64_t)sizeof(BatchDomain));
    l.k64 = take(nd * (int64_t)sizeof(StepConsts<double>));
    l.k32 = take(nd * (int64_t)sizeof(StepConsts<float>));
    l.tiles_nat = take(nt * (int64_t)sizeof(TileRec));
    // an XCD-placed order pads each XCD's queue to the longest one: at most 8 x the tiles
    l.tiles_launch = take(8 * nt * (int64_t)sizeof(TileRec));
    l.items = take(nt * (int64_t)sizeof(BatchItem));
    l.wg_first = take((kMaxWorkGroups + 1) * 4);
    l.chunks = take(nd * 4);
    l.ctr = take(nd * 4);
    l.status = take(4);
    l.partials = take(nt * 4 * 8);
    l.totals = take(nd * 4 * 8);
    l.total = off;
    return l;
}

}  // namespace

struct lbm_batch {
    Plan pl;
    ScratchLayout sl;
    char *scratch;
    BatchDomain *ddom;
    StepConsts<double> *dk64;
    StepConsts<float> *dk32;
    TileRec *dtiles;         // natural order
    TileRec *dlaunch;        // launch order of the step-per-launch mode
    BatchItem *ditems;
    uint32_t *dwg_first, *dchunks, *dctr, *dstatus;
    double *dpart, *dtot;
    void *pop[2];
    int cur;
    hipStream_t stream;
    int64_t t;
    int cu_count;
    uint32_t spin_limit;
    lbm_batch_schedule sched;
    uint32_t nlaunch;        // tiles in the launch order
    uint32_t nwg;            // persistent work-groups
    uint32_t max_chunks;     // largest items-per-domain count of the persistent lists
    // host copies of the schedule (kept alive across the uploads)
    std::vector<TileRec> launch;
    std::vector<BatchItem> items;
    std::vector<uint32_t> wg_first, chunks;
};

namespace {

int upload(lbm_batch *b, void *dst, const void *src, size_t bytes)
{
    if (bytes == 0) return LBM_OK;
    const hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, b->stream);
    return e == hipSuccess ? LBM_OK : fail_hip(e, "hipMemcpyAsync");
}

// Longest-processing-time-first: each job (in order of decreasing size) goes to the bin with
// the least load so far; returns the bin of every job.
std::vector<int> lpt(const std::vector<int64_t> &size, int bins)
{
    std::vector<size_t> order(size.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t c) { return size[a] > size[c]; });
    using Load = std::pair<int64_t, int>;  // (load, bin): ties go to the lower bin
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (int k = 0; k < bins; ++k) heap.push(Load{0, k});
    std::vector<int> bin(size.size(), 0);
    for (size_t j : order) {
        Load l = heap.top();
        heap.pop();
        bin[j] = l.second;
        l.first += size[j];
        heap.push(l);
    }
    return bin;
}

// XCD of every domain: longest-processing-time over the 8 XCDs by cell count.
std::vector<int> domains_to_xcds(const Plan &pl, const std::vector<size_t> &doms)
{
    std::vector<int64_t> size;
    for (size_t d : doms) size.push_back(pl.dom[d].cells);
    return lpt(size, 8);
}

void build_launch_order(lbm_batch *b, bool xcd)
{
    const Plan &pl = b->pl;
    b->launch.clear();
    if (!xcd) {
        b->launch = pl.tiles;
    } else {
        std::vector<size_t> all(pl.dom.size());
        for (size_t i = 0; i < all.size(); ++i) all[i] = i;
        const std::vector<int> x = domains_to_xcds(pl, all);
        std::vector<std::vector<TileRec>> queue(8);
        for (size_t d = 0; d < pl.dom.size(); ++d)
            for (uint32_t t = 0; t < pl.dom[d].ntiles; ++t)
                queue[(size_t)x[d]].push_back(pl.tiles[pl.dom[d].tile0 + t]);
        size_t len = 0;
        for (auto &qq : queue) len = std::max(len, qq.size());
        // position 8 j + k holds the j-th tile of XCD k's queue; short queues are padded
        for (size_t j = 0; j < len; ++j)
            for (int k = 0; k < 8; ++k)
                b->launch.push_back(j < queue[(size_t)k].size() ? queue[(size_t)k][j] : TileRec{kPadTile, 0});
    }
    b->nlaunch = (uint32_t)b->launch.size();
}

// Work lists of the persistent schedule: items in the order each work-group runs them.
struct PersistPlan {
    std::vector<BatchItem> items;
    std::vector<uint32_t> item_wg;   // work-group of each item
    std::vector<uint32_t> wg_first;  // [nwg + 1] item ranges per work-group
    std::vector<uint32_t> chunks;    // items per domain and step
    uint32_t nwg = 0, max_chunks = 1;
};

int check_persistent(const lbm_batch_schedule &s)
{
    if (s.chunk_cells < kTileCells || s.chunk_cells % kTileCells != 0)
        return fail(LBM_ERR_ARG, "chunk_cells must be a positive multiple of %d (got %lld)", kTileCells,
                    (long long)s.chunk_cells);
    if (s.group_bytes < 0) return fail(LBM_ERR_ARG, "group_bytes must be >= 0");
    if (s.wg_per_cu < 1) return fail(LBM_ERR_ARG, "wg_per_cu must be >= 1 (got %d)", s.wg_per_cu);
    return LBM_OK;
}

int plan_persistent(const Plan &pl, const lbm_batch_schedule &s, int cu_count, PersistPlan &out)
{
    const int64_t nwg = (int64_t)s.wg_per_cu * cu_count;
    if (nwg > kMaxWorkGroups) return fail(LBM_ERR_ARG, "%lld work-groups exceed the limit %lld", (long long)nwg,
                                          (long long)kMaxWorkGroups);
    // groups of consecutive domains within the byte budget
    std::vector<std::vector<size_t>> groups(1);
    int64_t used = 0;
    for (size_t d = 0; d < pl.dom.size(); ++d) {
        const int64_t bytes = 2LL * pl.q * (int64_t)pl.dom[d].cells * pl.bytes;
        if (s.group_bytes > 0 && !groups.back().empty() && used + bytes > s.group_bytes) {
            groups.emplace_back();
            used = 0;
        }
        groups.back().push_back(d);
        used += bytes;
    }
    struct Job {
        BatchItem item;
        int wg;
    };
    std::vector<Job> jobs;
    out.chunks.assign(pl.dom.size(), 0u);
    for (size_t g = 0; g < groups.size(); ++g) {
        // split each domain into near-equal runs of whole tiles, at most chunk_cells each
        std::vector<BatchItem> its;
        std::vector<int> home;  // XCD of the item's domain, or -1
        const std::vector<int> x = s.xcd_group ? domains_to_xcds(pl, groups[g]) : std::vector<int>();
        for (size_t gi = 0; gi < groups[g].size(); ++gi) {
            const size_t d = groups[g][gi];
            const int64_t nt = pl.dom[d].ntiles;
            const int64_t per = std::max<int64_t>(1, s.chunk_cells / kTileCells);
            const int64_t parts = (nt + per - 1) / per;
            for (int64_t k = 0; k < parts; ++k) {
                const int64_t t0 = nt * k / parts, t1 = nt * (k + 1) / parts;
                const int64_t c0 = t0 * kTileCells, c1 = std::min<int64_t>(t1 * kTileCells, pl.dom[d].cells);
                its.push_back(BatchItem{(uint32_t)d, (uint32_t)c0, (uint32_t)(c1 - c0), (uint32_t)g});
                home.push_back(s.xcd_group ? x[gi] : -1);
            }
            out.chunks[d] = (uint32_t)parts;
        }
        if (s.xcd_group) {
            // per XCD: its items over its own work-groups (w = k mod 8)
            for (int k = 0; k < 8; ++k) {
                std::vector<size_t> mine;
                for (size_t j = 0; j < its.size(); ++j)
                    if (home[j] == k) mine.push_back(j);
                const int64_t nk = nwg > k ? (nwg - 1 - k) / 8 + 1 : 0;
                if (mine.empty()) continue;
                if (nk == 0) return fail(LBM_ERR_ARG, "fewer than 8 work-groups for an XCD-placed schedule");
                std::vector<int64_t> size;
                for (size_t j : mine) size.push_back(its[j].count);
                const std::vector<int> w = lpt(size, (int)nk);
                for (size_t m = 0; m < mine.size(); ++m) jobs.push_back(Job{its[mine[m]], k + 8 * w[m]});
            }
        } else {
            std::vector<int64_t> size;
            for (auto &it : its) size.push_back(it.count);
            const std::vector<int> w = lpt(size, (int)nwg);
            for (size_t j = 0; j < its.size(); ++j) jobs.push_back(Job{its[j], w[j]});
        }
    }
    std::stable_sort(jobs.begin(), jobs.end(), [](const Job &a, const Job &c) {
        if (a.wg != c.wg) return a.wg < c.wg;
        if (a.item.group != c.item.group) return a.item.group < c.item.group;
        if (a.item.dom != c.item.dom) return a.item.dom < c.item.dom;
        return a.item.first < c.item.first;
    });
    out.items.clear();
    out.item_wg.clear();
    out.wg_first.assign((size_t)nwg + 1, 0u);
    for (const Job &j : jobs) {
        out.items.push_back(j.item);
        out.item_wg.push_back((uint32_t)j.wg);
        ++out.wg_first[(size_t)j.wg + 1];
    }
    for (int64_t w = 0; w < nwg; ++w) out.wg_first[(size_t)w + 1] += out.wg_first[(size_t)w];
    out.nwg = (uint32_t)nwg;
    out.max_chunks = 1;
    for (uint32_t c : out.chunks) out.max_chunks = std::max(out.max_chunks, c);
    return LBM_OK;
}

int build_persistent(lbm_batch *b, const lbm_batch_schedule &s)
{
    PersistPlan pp;
    const int rc = plan_persistent(b->pl, s, b->cu_count, pp);
    if (rc) return rc;
    b->items = std::move(pp.items);
    b->wg_first = std::move(pp.wg_first);
    b->chunks = std::move(pp.chunks);
    b->nwg = pp.nwg;
    b->max_chunks = pp.max_chunks;
    return LBM_OK;
}

int apply_schedule(lbm_batch *b, const lbm_batch_schedule &s)
{
    if (s.mode != LBM_BATCH_STEPWISE && s.mode != LBM_BATCH_PERSISTENT)
        return fail(LBM_ERR_ARG, "unknown schedule mode %d", s.mode);
    if (s.reserved != 0) return fail(LBM_ERR_ARG, "schedule reserved must be 0");
    if (s.xcd_group != 0 && s.xcd_group != 1) return fail(LBM_ERR_ARG, "xcd_group must be 0 or 1");
    if (s.mode == LBM_BATCH_STEPWISE) {
        build_launch_order(b, s.xcd_group != 0);
        int rc = upload(b, b->dlaunch, b->launch.data(), b->launch.size() * sizeof(TileRec));
        if (rc) return rc;
    } else {
        int rc = check_persistent(s);
        if (rc) return rc;
        int occ = 0;
        hipError_t e = batch_persist_occupancy(b->pl.lattice, b->pl.storage, b->pl.order, &occ);
        if (e != hipSuccess) return fail_hip(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
        if (s.wg_per_cu < 1 || s.wg_per_cu > occ)
            return fail(LBM_ERR_ARG, "wg_per_cu must be in 1 .. %d for this kernel (got %d)", occ, s.wg_per_cu);
        rc = build_persistent(b, s);
        if (rc) return rc;
        rc = upload(b, b->ditems, b->items.data(), b->items.size() * sizeof(BatchItem));
        if (!rc) rc = upload(b, b->dwg_first, b->wg_first.data(), b->wg_first.size() * sizeof(uint32_t));
        if (!rc) rc = upload(b, b->dchunks, b->chunks.data(), b->chunks.size() * sizeof(uint32_t));
        if (rc) return rc;
    }
    const hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
    b->sched = s;
    return LBM_OK;
}

int run_steps(lbm_batch *b, int64_t nsteps)
{
    const Plan &pl = b->pl;
    if (b->sched.mode == LBM_BATCH_STEPWISE) {
        for (int64_t i = 0; i < nsteps; ++i) {
            const hipError_t e = launch_batch_step(pl.lattice, pl.storage, pl.order, b->nlaunch, b->dlaunch, b->ddom,
                                                   b->dk64, b->dk32, b->pop[b->cur], b->pop[1 - b->cur], b->stream);
            if (e != hipSuccess) return fail_hip(e, "batch step launch");
            b->cur = 1 - b->cur;
        }
        return LBM_OK;
    }
    // the arrival counters count chunks * steps of one launch in 32 bits
    const int64_t per_launch = std::max<int64_t>(1, (int64_t)(0xffffffffu / b->max_chunks) - 1);
    int64_t left = nsteps;
    while (left > 0) {
        const int64_t n = std::min<int64_t>(left, std::min<int64_t>(per_launch, 1 << 30));
        hipError_t e = launch_fill_u32(b->dctr, pl.dom.size(), b->stream);
        if (e != hipSuccess) return fail_hip(e, "counter reset");
        PersistArgs a;
        a.pop0 = b->pop[0];
        a.pop1 = b->pop[1];
        a.parity = (uint32_t)b->cur;
        a.nsteps = (int32_t)n;
        a.doms = b->ddom;
        a.consts = pl.storage == LBM_F64 ? (const void *)b->dk64 : (const void *)b->dk32;
        a.items = b->ditems;
        a.wg_first = b->dwg_first;
        a.chunks = b->dchunks;
        a.ctr = b->dctr;
        a.status = b->dstatus;
        a.spin_limit = b->spin_limit;
        e = launch_batch_persist(pl.lattice, pl.storage, pl.order, b->nwg, a, b->stream);
        if (e != hipSuccess) return fail_hip(e, "persistent batch launch");
        b->cur = (int)((b->cur + n) & 1);
        left -= n;
    }
    return LBM_OK;
}

int check_status(lbm_batch *b)
{
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
    uint32_t st = 0;
    e = hipMemcpy(&st, b->dstatus, sizeof st, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpy");
    if (st != 0) {
        e = launch_fill_u32(b->dstatus, 1, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return fail_hip(e, "status reset");
        return fail(LBM_ERR_HIP, "a persistent batch launch gave up waiting for a domain's step (spin limit %u); "
                                 "the state is undefined", b->spin_limit);
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

int64_t lbm_batch_cells(const lbm_batch_params *p, int64_t *offsets)
{
    Plan pl;
    const int rc = plan_of(p, pl);
    if (rc) return rc;
    if (offsets) {
        for (size_t d = 0; d < pl.dom.size(); ++d) offsets[d] = (int64_t)pl.dom[d].cell0;
        offsets[pl.dom.size()] = pl.cells;
    }
    return pl.cells;
}

int64_t lbm_batch_plan(const lbm_batch_params *p, const lbm_batch_schedule *s, int32_t cu_count,
                       lbm_batch_item *items, int64_t cap)
{
    if (!s) return fail(LBM_ERR_ARG, "schedule is NULL");
    if (s->mode != LBM_BATCH_PERSISTENT) return fail(LBM_ERR_ARG, "only persistent schedules have work lists");
    if (s->reserved != 0 || (s->xcd_group != 0 && s->xcd_group != 1)) return fail(LBM_ERR_ARG, "invalid schedule");
    if (cu_count < 1) return fail(LBM_ERR_ARG, "cu_count must be >= 1");
    if (cap < 0 || (cap > 0 && !items)) return fail(LBM_ERR_ARG, "items must hold cap entries");
    int rc = check_persistent(*s);
    if (rc) return rc;
    Plan pl;
    rc = plan_of(p, pl);
    if (rc) return rc;
    PersistPlan pp;
    rc = plan_persistent(pl, *s, cu_count, pp);
    if (rc) return rc;
    const int64_t n = (int64_t)pp.items.size();
    for (int64_t i = 0; i < std::min(n, cap); ++i) {
        const BatchItem &it = pp.items[(size_t)i];
        items[i].domain = it.dom;
        items[i].first_cell = it.first;
        items[i].cells = it.count;
        items[i].group = it.group;
        items[i].work_group = pp.item_wg[(size_t)i];
    }
    return n;
}

int64_t lbm_batch_pop_bytes(const lbm_batch_params *p)
{
    Plan pl;
    const int rc = plan_of(p, pl);
    return rc ? rc : pl.pop_elems * pl.bytes;
}

int64_t lbm_batch_scratch_bytes(const lbm_batch_params *p)
{
    Plan pl;
    const int rc = plan_of(p, pl);
    return rc ? rc : layout_of(pl).total;
}

int lbm_batch_init(lbm_batch **out, const lbm_batch_params *p, void *pop_a, void *pop_b, void *scratch,
                   const double *rho0, const double *s0, void *hip_stream)
{
    if (!out) return fail(LBM_ERR_ARG, "out is NULL");
    *out = nullptr;
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return fail(LBM_ERR_ARG, "out of host memory");
    int rc = plan_of(p, b->pl);
    if (rc) {
        delete b;
        return rc;
    }
    if (!pop_a || !pop_b || !scratch || !rho0 || !s0) {
        delete b;
        return fail(LBM_ERR_ARG, "a device pointer is NULL");
    }
    if (!aligned256(pop_a) || !aligned256(pop_b) || !aligned256(scratch)) {
        delete b;
        return fail(LBM_ERR_ALIGN, "population arrays and scratch must be 256-byte aligned");
    }
    const Plan &pl = b->pl;
    b->sl = layout_of(pl);
    char *sc = (char *)scratch;
    b->scratch = sc;
    b->ddom = (BatchDomain *)(sc + b->sl.dom);
    b->dk64 = (StepConsts<double> *)(sc + b->sl.k64);
    b->dk32 = (StepConsts<float> *)(sc + b->sl.k32);
    b->dtiles = (TileRec *)(sc + b->sl.tiles_nat);
    b->dlaunch = (TileRec *)(sc + b->sl.tiles_launch);
    b->ditems = (BatchItem *)(sc + b->sl.items);
    b->dwg_first = (uint32_t *)(sc + b->sl.wg_first);
    b->dchunks = (uint32_t *)(sc + b->sl.chunks);
    b->dctr = (uint32_t *)(sc + b->sl.ctr);
    b->dstatus = (uint32_t *)(sc + b->sl.status);
    b->dpart = (double *)(sc + b->sl.partials);
    b->dtot = (double *)(sc + b->sl.totals);
    b->pop[0] = pop_a;
    b->pop[1] = pop_b;
    b->cur = 0;
    b->stream = (hipStream_t)hip_stream;
    b->t = 0;
    b->spin_limit = kDefaultSpinLimit;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cu_count, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) {
        delete b;
        return fail_hip(e, "device query");
    }
    std::vector<StepConsts<double>> k64(pl.dom.size());
    std::vector<StepConsts<float>> k32(pl.dom.size());
    for (size_t d = 0; d < pl.dom.size(); ++d) {
        k64[d] = consts_for<double>(pl.params[d], pl.prep[d]);
        k32[d] = consts_for<float>(pl.params[d], pl.prep[d]);
    }
    rc = upload(b, b->ddom, pl.dom.data(), pl.dom.size() * sizeof(BatchDomain));
    if (!rc) rc = upload(b, b->dk64, k64.data(), k64.size() * sizeof(StepConsts<double>));
    if (!rc) rc = upload(b, b->dk32, k32.data(), k32.size() * sizeof(StepConsts<float>));
    if (!rc) rc = upload(b, b->dtiles, pl.tiles.data(), pl.tiles.size() * sizeof(TileRec));
    if (!rc) {
        e = launch_fill_u32(b->dstatus, 1, b->stream);
        if (e == hipSuccess)
            e = launch_batch_init(pl.lattice, pl.storage, pl.order, (uint32_t)pl.tiles.size(), b->dtiles, b->ddom,
                                  b->dk64, rho0, s0, (uint64_t)pl.cells, b->pop[0], b->stream);
        if (e != hipSuccess) rc = fail_hip(e, "batch init launch");
    }
    if (!rc) {
        e = hipStreamSynchronize(b->stream);  // the host copies above must outlive the uploads
        if (e != hipSuccess) rc = fail_hip(e, "hipStreamSynchronize");
    }
    if (!rc) {
        lbm_batch_schedule s;
        std::memset(&s, 0, sizeof s);
        s.mode = LBM_BATCH_STEPWISE;
        rc = apply_schedule(b, s);
    }
    if (rc) {
        delete b;
        return rc;
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_set_schedule(lbm_batch *b, const lbm_batch_schedule *s)
{
    if (!b || !s) return fail(LBM_ERR_ARG, "NULL argument");
    const lbm_batch_schedule keep = b->sched;
    const int rc = apply_schedule(b, *s);
    if (rc) {
        const std::string msg = g_last_error;
        apply_schedule(b, keep);  // the previous schedule stays in force
        g_last_error = msg;
    }
    return rc;
}

int lbm_batch_get_schedule(const lbm_batch *b, lbm_batch_schedule *s)
{
    if (!b || !s) return fail(LBM_ERR_ARG, "NULL argument");
    *s = b->sched;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch *b, int64_t nsteps)
{
    if (!b) return fail(LBM_ERR_ARG, "batch is NULL");
    if (nsteps < 0) return fail(LBM_ERR_ARG, "nsteps must be >= 0");
    const int rc = run_steps(b, nsteps);
    if (!rc) b->t += nsteps;
    return rc;
}

int lbm_batch_status(lbm_batch *b)
{
    if (!b) return fail(LBM_ERR_ARG, "batch is NULL");
    return check_status(b);
}

int lbm_batch_autotune(lbm_batch *b, void *backup, int32_t trial_steps, lbm_batch_schedule *best, double *best_ms)
{
    if (!b || !backup) return fail(LBM_ERR_ARG, "NULL argument");
    if (!aligned256(backup)) return fail(LBM_ERR_ALIGN, "backup must be 256-byte aligned");
    if (trial_steps < 1) return fail(LBM_ERR_ARG, "trial_steps must be >= 1");
    const Plan &pl = b->pl;
    const int64_t bytes = pl.pop_elems * pl.bytes;
    int rc = check_status(b);
    if (rc) return rc;
    const int cur0 = b->cur;
    hipError_t e = launch_copy(backup, b->pop[cur0], (bytes + 15) / 16 * 16, b->stream);
    if (e != hipSuccess) return fail_hip(e, "state backup");

    std::vector<lbm_batch_schedule> cand;
    for (int x = 0; x <= 1; ++x) {
        lbm_batch_schedule s;
        std::memset(&s, 0, sizeof s);
        s.mode = LBM_BATCH_STEPWISE;
        s.xcd_group = x;
        cand.push_back(s);
    }
    int occ = 0;
    e = batch_persist_occupancy(pl.lattice, pl.storage, pl.order, &occ);
    if (e != hipSuccess) return fail_hip(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    const int64_t pair_bytes = 2 * bytes;
    for (int wpc : {1, 2, 4, 8})
        for (int64_t chunk : {4096, 16384, 65536})
            for (int64_t grp : {(int64_t)0, (int64_t)192 << 20, (int64_t)96 << 20}) {
                if (wpc > occ || (grp > 0 && grp >= pair_bytes)) continue;
                lbm_batch_schedule s;
                std::memset(&s, 0, sizeof s);
                s.mode = LBM_BATCH_PERSISTENT;
                s.xcd_group = 1;
                s.wg_per_cu = wpc;
                s.chunk_cells = chunk;
                s.group_bytes = grp;
                cand.push_back(s);
            }

    hipEvent_t ev[2];
    e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e != hipSuccess) return fail_hip(e, "hipEventCreate");
    const lbm_batch_schedule keep = b->sched;
    double best_t = 1e300;
    lbm_batch_schedule chosen = keep;
    for (const lbm_batch_schedule &s : cand) {
        if (apply_schedule(b, s) != LBM_OK) continue;
        if (run_steps(b, 2) != LBM_OK) continue;
        if (hipEventRecord(ev[0], b->stream) != hipSuccess) continue;
        if (run_steps(b, trial_steps) != LBM_OK) continue;
        if (hipEventRecord(ev[1], b->stream) != hipSuccess) continue;
        if (check_status(b) != LBM_OK) continue;  // a trial whose waits gave up is not a candidate
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) continue;
        const double per = (double)ms / trial_steps;
        if (per < best_t) {
            best_t = per;
            chosen = s;
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    // restore the state and the parity it was in
    e = launch_copy(b->pop[cur0], backup, (bytes + 15) / 16 * 16, b->stream);
    if (e != hipSuccess) return fail_hip(e, "state restore");
    b->cur = cur0;
    rc = apply_schedule(b, chosen);
    if (rc) return rc;
    if (best) *best = chosen;
    if (best_ms) *best_ms = best_t;
    return LBM_OK;
}

int lbm_batch_moments(lbm_batch *b, double *rho, double *s, double *totals)
{
    if (!b) return fail(LBM_ERR_ARG, "batch is NULL");
    int rc = check_status(b);
    if (rc) return rc;
    const Plan &pl = b->pl;
    hipError_t e = launch_batch_moments(pl.lattice, pl.storage, (uint32_t)pl.tiles.size(), b->dtiles, b->ddom,
                                        b->dk64, b->pop[b->cur], rho, s, (uint64_t)pl.cells, b->dpart,
                                        (uint32_t)pl.dom.size(), b->dtot, b->stream);
    if (e != hipSuccess) return fail_hip(e, "batch moments launch");
    if (!totals) return LBM_OK;
    std::vector<double> h(pl.dom.size() * 4);
    e = hipMemcpyAsync(h.data(), b->dtot, h.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return fail_hip(e, "totals copy");
    for (size_t d = 0; d < pl.dom.size(); ++d) {
        totals[4 * d + 0] = (double)pl.dom[d].cells * pl.rho0 + h[4 * d + 0];
        for (int a = 1; a < 4; ++a) totals[4 * d + a] = h[4 * d + a];
        for (int a = 0; a < 4; ++a)
            if (!std::isfinite(totals[4 * d + a]))
                return fail(LBM_ERR_NONFINITE, "domain %zu: a conservation total is not finite", d);
    }
    return LBM_OK;
}

int lbm_batch_get_f64(lbm_batch *b, double *out)
{
    if (!b || !out) return fail(LBM_ERR_ARG, "NULL argument");
    int rc = check_status(b);
    if (rc) return rc;
    const Plan &pl = b->pl;
    const hipError_t e = launch_batch_export(pl.lattice, pl.storage, (uint32_t)pl.tiles.size(), b->dtiles, b->ddom,
                                             b->dk64, b->pop[b->cur], out, b->stream);
    return e == hipSuccess ? LBM_OK : fail_hip(e, "batch export launch");
}

int64_t lbm_batch_time(const lbm_batch *b) { return b ? b->t : -1; }

int lbm_batch_set_spin_limit(lbm_batch *b, uint32_t polls)
{
    if (!b) return fail(LBM_ERR_ARG, "batch is NULL");
    b->spin_limit = polls;
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch *b) { delete b; }

}  // extern "C"
