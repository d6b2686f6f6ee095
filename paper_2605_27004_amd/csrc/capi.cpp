// capi.cpp -- host side of the C ABI declared in include/lbm.h: parameter validation and
// preparation, context bookkeeping and kernel launches. No device memory is allocated here.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>
#include <string>

#include "../../include/lbm.h"
#include "common.hpp"
#include "host.hpp"

using namespace lbm;

namespace lbm {
namespace host {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int fail_hip(hipError_t e, const char *what)
{
    return fail(LBM_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

// ---- lattice tables in canonical order -------------------------------------------------


template <int LAT> void fill_table(LatticeTable &t)
{
    using L = Lattice<LAT>;
    t.q = L::Q;
    t.d = L::D;
    t.np = L::NP;
    t.c[0][0] = t.c[0][1] = t.c[0][2] = 0;
    t.w[0] = (double)L::w_rest / kWeightDen;
    t.opp[0] = 0;
    for (int p = 0; p < L::NP; ++p) {
        const PairRow v = L::pair(p);
        const int ip = 2 * p + 1, im = 2 * p + 2;
        t.c[ip][0] = v.cx;
        t.c[ip][1] = v.cy;
        t.c[ip][2] = v.cz;
        t.c[im][0] = -v.cx;
        t.c[im][1] = -v.cy;
        t.c[im][2] = -v.cz;
        t.w[ip] = t.w[im] = (double)L::w_pair(p) / kWeightDen;
        t.opp[ip] = im;
        t.opp[im] = ip;
    }
}

bool table_of(int lattice, LatticeTable &t)
{
    switch (lattice) {
    case LBM_D2Q9: fill_table<kD2Q9>(t); return true;
    case LBM_D3Q19: fill_table<kD3Q19>(t); return true;
    case LBM_D3Q27: fill_table<kD3Q27>(t); return true;
    default: return false;
    }
}

int storage_bytes(int storage)
{
    switch (storage) {
    case LBM_F64: return 8;
    case LBM_F32: return 4;
    case LBM_F16:
    case LBM_BF16: return 2;
    default: return 0;
    }
}

// ---- small dense linear algebra (d <= 3) ----------------------------------------------------

// Cholesky factor L (lower) of a symmetric d x d matrix; false unless positive definite.
bool cholesky(int d, const double *m, double *l)
{
    std::memset(l, 0, sizeof(double) * 9);
    for (int j = 0; j < d; ++j) {
        double s = m[j * d + j];
        for (int k = 0; k < j; ++k) s -= l[j * 3 + k] * l[j * 3 + k];
        if (!(s > 0.0)) return false;
        l[j * 3 + j] = std::sqrt(s);
        for (int i = j + 1; i < d; ++i) {
            double t = m[i * d + j];
            for (int k = 0; k < j; ++k) t -= l[i * 3 + k] * l[j * 3 + k];
            l[i * 3 + j] = t / l[j * 3 + j];
        }
    }
    return true;
}

// Inverse of an SPD matrix from its Cholesky factor: M^-1 = L^-T L^-1 (d x d, stride d).
void spd_inverse(int d, const double *l, double *inv)
{
    double li[9] = {0};  // L^-1, lower, stride 3
    for (int j = 0; j < d; ++j) {
        li[j * 3 + j] = 1.0 / l[j * 3 + j];
        for (int i = j + 1; i < d; ++i) {
            double t = 0.0;
            for (int k = j; k < i; ++k) t -= l[i * 3 + k] * li[k * 3 + j];
            li[i * 3 + j] = t / l[i * 3 + i];
        }
    }
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            double t = 0.0;
            for (int k = 0; k < d; ++k) t += li[k * 3 + a] * li[k * 3 + b];
            inv[a * d + b] = t;
        }
}

double det_from_cholesky(int d, const double *l)
{
    double p = 1.0;
    for (int j = 0; j < d; ++j) p *= l[j * 3 + j];
    return p * p;
}


Grid grid_of(int64_t nx, int64_t ny, int64_t nz, int q, int bytes)
{
    Grid g{};
    g.nx = (int32_t)nx;
    g.ny = (int32_t)ny;
    g.nz = (int32_t)nz;
    g.n = (uint32_t)(nx * ny * nz);
    int64_t rows = 1;
    for (int64_t r = ny; r >= 1; --r)
        if (ny % r == 0 && r * nx * bytes <= block_bytes(bytes)) {
            rows = r;
            break;
        }
    g.rows = (uint32_t)rows;
    g.mr = rows == 1 ? 0xffffffffu : (uint32_t)(4294967296.0 / (double)rows);
    // floor(2^32 / rows) exactly (the double quotient can round up at the last bit)
    if (rows > 1 && (uint64_t)g.mr * (uint64_t)rows > 4294967296ull) --g.mr;
    g.bc = (uint32_t)(rows * nx);
    g.bq = (uint32_t)(q * rows * nx);
    g.zs = (uint32_t)(q * nx * ny);
    return g;
}

int prepare(const lbm_params *p, Prepared &out)
{
    if (!p) return fail(LBM_ERR_ARG, "params is NULL");
    if (!table_of(p->lattice, out.lat)) return fail(LBM_ERR_ARG, "unknown lattice %d", p->lattice);
    const int d = out.lat.d, q = out.lat.q;
    out.d = d;
    out.q = q;
    out.bytes = storage_bytes(p->storage);
    if (!out.bytes) return fail(LBM_ERR_ARG, "unknown storage %d", p->storage);
    if (p->order != 2 && p->order != 3) return fail(LBM_ERR_ARG, "order must be 2 or 3 (got %d)", p->order);
    if (p->tensor_kind < LBM_TENSOR_THETA || p->tensor_kind > LBM_TENSOR_ATILDE)
        return fail(LBM_ERR_ARG, "unknown tensor kind %d", p->tensor_kind);
    if (p->shift_kind != LBM_SHIFT_REST && p->shift_kind != LBM_SHIFT_WEIGHT)
        return fail(LBM_ERR_ARG, "unknown shift kind %d", p->shift_kind);
    if (p->flags & ~(LBM_FLAG_MASK | LBM_FLAG_GRAY)) return fail(LBM_ERR_ARG, "unknown flags 0x%x", p->flags);
    if ((p->flags & LBM_FLAG_MASK) && (p->flags & LBM_FLAG_GRAY))
        return fail(LBM_ERR_ARG, "LBM_FLAG_MASK and LBM_FLAG_GRAY are exclusive");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->force[a])) return fail(LBM_ERR_ARG, "force has a non-finite entry");
    if (d == 2 && p->force[2] != 0.0) return fail(LBM_ERR_ARG, "D2Q9 needs force[2] == 0");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1)
        return fail(LBM_ERR_ARG, "grid extents must be >= 1 (got %lld x %lld x %lld)", (long long)p->nx,
                    (long long)p->ny, (long long)p->nz);
    if (d == 2 && p->nz != 1) return fail(LBM_ERR_ARG, "D2Q9 needs nz == 1 (got %lld)", (long long)p->nz);
    const double nd = (double)p->nx * (double)p->ny * (double)p->nz;
    // 32-bit cell indices and 32-bit byte offsets inside each population plane
    if (nd >= 2147483648.0 || nd * out.bytes >= 4294967296.0)
        return fail(LBM_ERR_SIZE, "grid of %.0f cells exceeds the 2^31-cell / 4 GiB-per-plane limit", nd);
    // the population layout indexes one z-plane with 32-bit byte offsets
    if ((double)q * (double)p->nx * (double)p->ny * out.bytes >= 4294967296.0)
        return fail(LBM_ERR_SIZE, "one z-plane of %lld x %lld cells holds 4 GiB or more of populations",
                    (long long)p->nx, (long long)p->ny);
    out.n = (uint32_t)(p->nx * p->ny * p->nz);
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(LBM_ERR_TAU, "tau must be > 1/2 (got %g)", p->tau);
    if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return fail(LBM_ERR_ARG, "rho0 must be > 0 (got %g)", p->rho0);

    // tensor -> A^-1
    double t[9], tmax = 0.0;
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            t[a * d + b] = p->tensor[a * 3 + b];
            if (!std::isfinite(t[a * d + b])) return fail(LBM_ERR_ARG, "tensor has a non-finite entry");
            tmax = std::fmax(tmax, std::fabs(t[a * d + b]));
        }
    for (int a = 0; a < d; ++a)
        for (int b = a + 1; b < d; ++b)
            if (std::fabs(t[a * d + b] - t[b * d + a]) > 1e-12 * tmax)
                return fail(LBM_ERR_NOT_SPD, "tensor is not symmetric (T[%d][%d] != T[%d][%d])", a, b, b, a);
    // the tensor enters as its symmetric part (T + T^T) / 2 (equal to T within the check above),
    // so the update, and every derivative of it, depends on T_ab and T_ba alike
    for (int a = 0; a < d; ++a)
        for (int b = a + 1; b < d; ++b) t[a * d + b] = t[b * d + a] = 0.5 * (t[a * d + b] + t[b * d + a]);
    double l[9], ainv[9];
    if (!cholesky(d, t, l)) return fail(LBM_ERR_NOT_SPD, "tensor is not positive definite");
    if (p->tensor_kind == LBM_TENSOR_THETA) {
        for (int k = 0; k < d * d; ++k) ainv[k] = t[k] / kCs2;  // tensor = cs^2 A^-1
    } else {
        double scale = 1.0;
        if (p->tensor_kind == LBM_TENSOR_ATILDE) scale = std::pow(det_from_cholesky(d, l), 1.0 / d);
        double inv[9];
        spd_inverse(d, l, inv);  // (A~)^-1 or A^-1
        for (int k = 0; k < d * d; ++k) ainv[k] = inv[k] * scale;  // A^-1 = det^(1/d) A~^-1
    }
    // symmetrise exactly (the inverse is symmetric up to round-off)
    for (int a = 0; a < d; ++a)
        for (int b = a + 1; b < d; ++b) ainv[a * d + b] = ainv[b * d + a] = 0.5 * (ainv[a * d + b] + ainv[b * d + a]);

    lbm_derived &dv = out.dv;
    std::memset(&dv, 0, sizeof dv);
    dv.q = q;
    dv.d = d;
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            dv.ainv[a * 3 + b] = ainv[a * d + b];
            dv.k[a * 3 + b] = ainv[a * d + b] - (a == b ? 1.0 : 0.0);  // K = A^-1 - I
        }
    dv.omega = 1.0 / p->tau;
    dv.nu = kCs2 * (p->tau - 0.5);
    const double trk = dv.k[0] + dv.k[4] + dv.k[8];
    dv.min_rest_ratio = 1e300;
    for (int i = 0; i < q; ++i) {
        double ckc = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) ckc += out.lat.c[i][a] * dv.k[a * 3 + b] * out.lat.c[i][b];
        // r_i = f^eq_i(1, 0) = w_i (1 + H2_i:K / (2 cs^2)),  H2_i:K = c.K.c - cs^2 tr K
        const double r = out.lat.w[i] * (1.0 + (ckc - kCs2 * trk) / (2.0 * kCs2));
        dv.rest[i] = r;
        dv.shift[i] = p->rho0 * (p->shift_kind == LBM_SHIFT_REST ? r : out.lat.w[i]);
        dv.min_rest_ratio = std::fmin(dv.min_rest_ratio, r / out.lat.w[i]);
    }
    return LBM_OK;
}

template <typename C> StepConsts<C> consts_for(const lbm_params &p, const Prepared &pr)
{
    StepConsts<C> k;
    std::memset(&k, 0, sizeof k);
    const lbm_derived &dv = pr.dv;
    k.omega = (C)dv.omega;
    k.keep = (C)(1.0 - dv.omega);
    k.rho0 = (C)p.rho0;
    k.k[0] = (C)dv.k[0];
    k.k[1] = (C)dv.k[4];
    k.k[2] = (C)dv.k[8];
    k.k[3] = (C)dv.k[1];
    k.k[4] = (C)dv.k[2];
    k.k[5] = (C)dv.k[5];
    const int kidx[6] = {0, 4, 8, 1, 2, 5};
    for (int e = 0; e < 6; ++e) k.km3[e] = (C)(-3.0 * dv.k[kidx[e]]);
    const double trk = dv.k[0] + dv.k[4] + dv.k[8];
    for (int pp = 0; pp <= pr.lat.np; ++pp) {
        const int i = pp == 0 ? 0 : 2 * pp - 1;  // the + member of pair pp (or the rest)
        double ckc = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) ckc += pr.lat.c[i][a] * dv.k[a * 3 + b] * pr.lat.c[i][b];
        k.w[pp] = (C)pr.lat.w[i];
        k.rest[pp] = (C)dv.rest[i];
        k.eoff[pp] = (C)(p.rho0 * dv.rest[i] - dv.shift[i]);
        k.ow[pp] = (C)(dv.omega * pr.lat.w[i]);
        k.orest[pp] = (C)(dv.omega * dv.rest[i]);
        k.oeoff[pp] = (C)(dv.omega * (p.rho0 * dv.rest[i] - dv.shift[i]));
        k.a[pp] = (C)(3.0 + 4.5 * ckc - 1.5 * trk);
        k.sigma[pp] = (C)dv.shift[i];
    }
    k.forced = 0;
    for (int a = 0; a < 3; ++a) {
        k.force[a] = (C)p.force[a];
        if (p.force[a] != 0.0) k.forced = 1;
    }
    return k;
}

// Scratch layout: [link words, 4 bytes per cell, when masked][partials][totals], 256-byte
// aligned pieces.
int64_t links_bytes(const lbm_params &p, uint32_t n)
{
    return (p.flags & (LBM_FLAG_MASK | LBM_FLAG_GRAY)) ? ((int64_t)n * 4 + 255) / 256 * 256 : 0;
}

int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

bool aligned256(const void *ptr) { return ((uintptr_t)ptr & 255u) == 0; }

template StepConsts<float> consts_for<float>(const lbm_params &, const Prepared &);
template StepConsts<double> consts_for<double>(const lbm_params &, const Prepared &);

}  // namespace host
}  // namespace lbm

using namespace lbm::host;

extern "C" {

int lbm_lattice_info(int32_t lattice, int32_t *q, int32_t *d, int32_t *c, double *w, int32_t *opp)
{
    LatticeTable t;
    if (!table_of(lattice, t)) return fail(LBM_ERR_ARG, "unknown lattice %d", lattice);
    if (q) *q = t.q;
    if (d) *d = t.d;
    for (int i = 0; i < t.q; ++i) {
        if (c)
            for (int a = 0; a < 3; ++a) c[3 * i + a] = t.c[i][a];
        if (w) w[i] = t.w[i];
        if (opp) opp[i] = t.opp[i];
    }
    return LBM_OK;
}

int lbm_prepare(const lbm_params *p, lbm_derived *out)
{
    Prepared pr;
    const int rc = prepare(p, pr);
    if (rc) return rc;
    if (out) *out = pr.dv;
    return LBM_OK;
}

int64_t lbm_pop_bytes(const lbm_params *p)
{
    Prepared pr;
    if (prepare(p, pr)) return -1;
    return (int64_t)pr.q * (int64_t)pr.n * pr.bytes;
}

int64_t lbm_rows_per_block(const lbm_params *p)
{
    Prepared pr;
    if (prepare(p, pr)) return -1;
    return grid_of(p->nx, p->ny, p->nz, pr.q, pr.bytes).rows;
}

int64_t lbm_scratch_bytes(const lbm_params *p)
{
    Prepared pr;
    if (prepare(p, pr)) return -1;
    const Grid g = grid_of(p->nx, p->ny, p->nz, pr.q, pr.bytes);
    // kPartials sums per work-group of the moments launch, then kPartials totals, rounded up
    // to 256 bytes
    const int64_t bytes = 8 * (kPartials * (int64_t)moments_groups(g) + kPartials);
    return links_bytes(*p, pr.n) + (bytes + 255) / 256 * 256;
}

int lbm_init(lbm_ctx **out, const lbm_params *p, void *pop_a, void *pop_b, void *scratch, const double *rho0,
             const double *s0, const void *mask, void *stream)
{
    if (!out) return fail(LBM_ERR_ARG, "out is NULL");
    *out = nullptr;
    Prepared pr;
    int rc = prepare(p, pr);
    if (rc) return rc;
    const bool masked = p->flags & LBM_FLAG_MASK;
    const bool grayed = p->flags & LBM_FLAG_GRAY;
    if ((masked || grayed) && !mask) return fail(LBM_ERR_ARG, "LBM_FLAG_MASK / LBM_FLAG_GRAY is set but mask is NULL");
    if (!masked && !grayed && mask) return fail(LBM_ERR_ARG, "a mask was passed without LBM_FLAG_MASK / LBM_FLAG_GRAY");
    if (!pop_a || !pop_b || !scratch || !rho0 || !s0) return fail(LBM_ERR_ARG, "a device pointer is NULL");
    if (pop_a == pop_b) return fail(LBM_ERR_ARG, "pop_a and pop_b must be distinct buffers");
    if (!aligned256(pop_a) || !aligned256(pop_b) || !aligned256(scratch))
        return fail(LBM_ERR_ALIGN, "population and scratch buffers must be 256-byte aligned");
    lbm_ctx *c = new (std::nothrow) lbm_ctx;
    if (!c) return fail(LBM_ERR_ARG, "out of host memory");
    c->p = *p;
    c->pr = pr;
    c->grid = grid_of(p->nx, p->ny, p->nz, pr.q, pr.bytes);
    c->k64 = consts_for<double>(*p, pr);
    c->k32 = consts_for<float>(*p, pr);
    c->pop[0] = pop_a;
    c->pop[1] = pop_b;
    c->cur = 0;
    c->links = masked ? (uint32_t *)scratch : nullptr;
    c->gray = grayed ? (float *)scratch : nullptr;
    c->partials = (double *)((char *)scratch + links_bytes(*p, pr.n));
    c->stream = (hipStream_t)stream;
    c->t = 0;
    // Work-groups span whole x rows where they fit (up to 256 cells), so the boundary cache
    // line of every x-shifted pull is shared by waves of the same work-group; the rest of the
    // 256 lanes stack rows in y. Hardware round-robin order measured best for such tiles.
    // Longer rows take the width of 256, 128 or 64 that pads the row least, the widest on a tie
    // (D3Q19 FP32, fraction of 8 TB/s: 320^3 at 64 x 4 76% against 58% at 256 wide, 384^3 at
    // 128 x 2 74% against 69% at 192 wide, 512^3 at 256 wide 75% against 69% at 128 wide).
    if (p->nx <= 256) {
        c->block_x = (int)((p->nx + 63) / 64) * 64;
    } else {
        int64_t best = INT64_MAX;
        for (int bx : {256, 128, 64}) {
            const int64_t padded = (p->nx + bx - 1) / bx * bx;
            if (padded < best) {
                best = padded;
                c->block_x = bx;
            }
        }
    }
    c->block_y = 256 / c->block_x;
    c->launch_flags = 0;
    hipError_t e = hipSuccess;
    if (masked) e = launch_links(p->lattice, c->grid, (const uint8_t *)mask, c->links, c->stream);
    if (grayed) e = hipMemcpyAsync(c->gray, mask, (size_t)pr.n * 4, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
        e = launch_init(p->lattice, p->storage, p->order, c->grid, c->k64, rho0, s0, c->links, c->pop[0], c->stream);
    if (e != hipSuccess) {
        delete c;
        return fail_hip(e, "init kernel launch");
    }
    *out = c;
    return LBM_OK;
}

int lbm_stream_floor(lbm_ctx *c, int64_t nsteps)
{
    if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
    if (nsteps < 0) return fail(LBM_ERR_ARG, "nsteps must be >= 0");
    if (c->links || c->gray) return fail(LBM_ERR_UNSUPPORTED, "the streaming floor is defined for periodic grids only");
    for (int64_t s = 0; s < nsteps; ++s) {
        hipError_t e = launch_step(c->p.lattice, c->p.storage, c->p.order, c->grid, c->k64, c->k32, nullptr, nullptr,
                                   c->pop[c->cur], c->pop[c->cur ^ 1], c->block_x, c->block_y,
                                   c->launch_flags | kLaunchStreamOnly, c->stream);
        if (e != hipSuccess) return fail_hip(e, "streaming kernel launch");
        c->cur ^= 1;
    }
    return LBM_OK;
}

int lbm_step(lbm_ctx *c, int64_t nsteps)
{
    if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
    if (nsteps < 0) return fail(LBM_ERR_ARG, "nsteps must be >= 0");
    for (int64_t s = 0; s < nsteps; ++s) {
        hipError_t e = launch_step(c->p.lattice, c->p.storage, c->p.order, c->grid, c->k64, c->k32, c->links,
                                   c->gray, c->pop[c->cur], c->pop[c->cur ^ 1], c->block_x, c->block_y,
                                   c->launch_flags, c->stream);
        if (e != hipSuccess) return fail_hip(e, "step kernel launch");
        c->cur ^= 1;
        ++c->t;
    }
    return LBM_OK;
}

int lbm_moments(lbm_ctx *c, double *rho, double *s, double *totals)
{
    if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
    const uint32_t nb = moments_groups(c->grid);
    return moments_with(c, rho, s, totals, c->partials, c->partials + kPartials * (size_t)nb);
}

}  // extern "C"

namespace lbm {
namespace host {

int moments_with(lbm_ctx *c, double *rho, double *s, double *totals, double *partials, double *dtot)
{
    hipError_t e = launch_moments(c->p.lattice, c->p.storage, c->grid, c->k64, c->links, c->pop[c->cur], rho, s,
                                  partials, dtot, c->stream);
    if (e != hipSuccess) return fail_hip(e, "moments kernel launch");
    if (!totals) return LBM_OK;
    double h[kPartials];
    e = hipMemcpyAsync(h, dtot, sizeof h, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail_hip(e, "moments read-back");
    // sum over fluid cells of rho = (fluid cells) rho0 + sum (rho - rho0); the device sums
    // the deviations and counts the fluid cells
    totals[0] = h[4] * c->p.rho0 + h[0];
    totals[1] = h[1];
    totals[2] = h[2];
    totals[3] = c->pr.d == 3 ? h[3] : 0.0;
    for (int m = 0; m < 4; ++m)
        if (!std::isfinite(totals[m])) return fail(LBM_ERR_NONFINITE, "conservation total %d is not finite", m);
    return LBM_OK;
}

}  // namespace host
}  // namespace lbm

extern "C" {

int lbm_get_populations(lbm_ctx *c, void *out)
{
    if (!c || !out) return fail(LBM_ERR_ARG, "NULL argument");
    hipError_t e =
        launch_permute(c->p.lattice, c->p.storage, 0, c->grid, c->k64, c->links, c->pop[c->cur], out, c->stream);
    return e == hipSuccess ? LBM_OK : fail_hip(e, "export kernel launch");
}

int lbm_set_populations(lbm_ctx *c, const void *in)
{
    if (!c || !in) return fail(LBM_ERR_ARG, "NULL argument");
    hipError_t e =
        launch_permute(c->p.lattice, c->p.storage, 1, c->grid, c->k64, c->links, in, c->pop[c->cur], c->stream);
    return e == hipSuccess ? LBM_OK : fail_hip(e, "import kernel launch");
}

int lbm_get_f64(lbm_ctx *c, double *out)
{
    if (!c || !out) return fail(LBM_ERR_ARG, "NULL argument");
    hipError_t e =
        launch_permute(c->p.lattice, c->p.storage, 2, c->grid, c->k64, c->links, c->pop[c->cur], out, c->stream);
    return e == hipSuccess ? LBM_OK : fail_hip(e, "export kernel launch");
}

int64_t lbm_time(const lbm_ctx *c) { return c ? c->t : -1; }

int lbm_set_launch(lbm_ctx *c, int32_t block_x, int32_t block_y, int32_t flags)
{
    if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
    if (flags & ~(LBM_LAUNCH_XCD_SLABS | LBM_LAUNCH_SHIFTED_PULL))
        return fail(LBM_ERR_ARG, "unknown launch flags 0x%x", flags);
    if (block_x < 64 || block_x % 64 != 0 || block_y < 1 || block_x * block_y > 256)
        return fail(LBM_ERR_ARG, "block shape %d x %d: need block_x a multiple of 64 and block_x*block_y <= 256",
                    block_x, block_y);
    c->block_x = block_x;
    c->block_y = block_y;
    c->launch_flags = flags;
    return LBM_OK;
}

namespace {

struct GradLayout {
    int64_t nseg, seglen;
    int64_t ckpt, seg, lam_a, lam_b, gpart, jpart, sums, total;  // byte offsets / size
};

int grad_layout(const lbm_ctx *c, const lbm_grad_spec *spec, GradLayout &l)
{
    if (!c || !spec) return fail(LBM_ERR_ARG, "NULL argument");
    if (spec->reserved != 0) return fail(LBM_ERR_ARG, "spec->reserved must be 0");
    if (spec->objective != 0 && spec->objective != 1) return fail(LBM_ERR_ARG, "objective must be 0 or 1");
    if (spec->nsteps < 0 || spec->checkpoint_every < 1)
        return fail(LBM_ERR_ARG, "need nsteps >= 0 and checkpoint_every >= 1");
    if (spec->objective == 0 && (spec->outlet_plane < 0 || spec->outlet_plane >= c->p.nx))
        return fail(LBM_ERR_ARG, "outlet_plane %lld outside 0..%lld", (long long)spec->outlet_plane,
                    (long long)(c->p.nx - 1));
    const int64_t popb = (int64_t)c->pr.q * c->grid.n * c->pr.bytes;
    const int lam_bytes = c->p.storage == LBM_F64 ? 8 : 4;
    const int64_t lamb = (int64_t)c->pr.q * c->grid.n * lam_bytes;
    // the adjoint populations use the state's layout in the arithmetic precision (FP32 for
    // half storage), and one z-plane of them must stay below 4 GiB as well
    if ((double)c->pr.q * (double)c->p.nx * (double)c->p.ny * lam_bytes >= 4294967296.0)
        return fail(LBM_ERR_SIZE, "one z-plane of the adjoint populations would hold 4 GiB or more");
    const int64_t nb = moments_groups(c->grid), na = adjoint_blocks(c->grid);
    l.seglen = std::min<int64_t>(spec->checkpoint_every, std::max<int64_t>(spec->nsteps, 1));
    l.nseg = (spec->nsteps + spec->checkpoint_every - 1) / spec->checkpoint_every;
    int64_t off = 0;
    l.ckpt = off;
    off += align256(popb) * l.nseg;
    l.seg = off;
    off += align256(popb) * (l.seglen - 1);
    l.lam_a = off;
    off += align256(lamb);
    l.lam_b = off;
    off += align256(lamb);
    l.gpart = off;
    off += align256(8 * kGradPartialsHost * na);
    l.jpart = off;
    off += align256(8 * nb);
    l.sums = off;
    off += 256;
    l.total = off;
    return LBM_OK;
}

}  // namespace

int64_t lbm_grad_workspace_bytes(const lbm_ctx *c, const lbm_grad_spec *spec)
{
    GradLayout l;
    const int rc = grad_layout(c, spec, l);
    return rc ? rc : l.total;
}

int lbm_grad(lbm_ctx *c, const lbm_grad_spec *spec, void *workspace, double *objective, double *dtensor,
             double *dtau, double *dmask)
{
    GradLayout l;
    int rc = grad_layout(c, spec, l);
    if (rc) return rc;
    if (!workspace || !objective) return fail(LBM_ERR_ARG, "workspace and objective must not be NULL");
    if (!aligned256(workspace)) return fail(LBM_ERR_ALIGN, "workspace must be 256-byte aligned");
    char *ws = (char *)workspace;
    const int64_t popb = (int64_t)c->pr.q * c->grid.n * c->pr.bytes;
    const int64_t pstride = align256(popb);
    const uint32_t nb = moments_groups(c->grid), na = adjoint_blocks(c->grid);
    hipStream_t st = c->stream;
    hipError_t e = hipSuccess;
    auto ckpt = [&](int64_t s) { return (void *)(ws + l.ckpt + s * pstride); };
    auto segst = [&](int64_t t) { return (void *)(ws + l.seg + (t - 1) * pstride); };  // t >= 1

    // forward pass. Each step runs from one buffer into another, as in lbm_step, but the step
    // that ends a segment writes straight into the next segment's checkpoint, and the steps of
    // the last segment write straight into the segment buffer, from which the reverse sweep then
    // takes that segment without recomputing it (the step is deterministic, so these are bitwise
    // the states a recompute gives). Only the initial state is copied.
    if (l.nseg > 0) {
        e = hipMemcpyAsync(ckpt(0), c->pop[c->cur], popb, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return fail_hip(e, "checkpoint copy");
        const void *src = ckpt(0);
        for (int64_t sgi = 0; sgi < l.nseg; ++sgi) {
            const int64_t len = std::min(spec->checkpoint_every, spec->nsteps - sgi * spec->checkpoint_every);
            const bool last = sgi == l.nseg - 1;
            for (int64_t t = 1; t <= len; ++t) {
                void *dst = t == len ? (last ? c->pop[0] : ckpt(sgi + 1)) : (last ? segst(t) : c->pop[t & 1]);
                e = launch_step(c->p.lattice, c->p.storage, c->p.order, c->grid, c->k64, c->k32, c->links, c->gray,
                                src, dst, c->block_x, c->block_y, c->launch_flags, st);
                if (e != hipSuccess) return fail_hip(e, "forward step");
                src = dst;
            }
        }
        c->cur = 0;
        c->t += spec->nsteps;
    }
    // seed the reverse sweep with dJ/df at the final state
    void *lam_in = ws + l.lam_a, *lam_out = ws + l.lam_b;
    double *gpart = (double *)(ws + l.gpart), *jpart = (double *)(ws + l.jpart), *sums = (double *)(ws + l.sums);
    e = launch_seed(c->p.lattice, c->p.storage, c->grid, c->k64, c->k32, c->pop[c->cur], lam_in, jpart,
                    spec->objective, (int)spec->outlet_plane, c->links, st);
    if (e == hipSuccess) e = launch_sum(jpart, nb, 1, sums, st);
    if (e == hipSuccess) e = launch_zero(gpart, (uint64_t)kGradPartialsHost * na, st);
    if (e == hipSuccess && dmask) e = launch_zero(dmask, c->grid.n, st);
    if (e != hipSuccess) return fail_hip(e, "reverse-sweep set-up");
    // reverse sweep, one recomputed segment at a time
    for (int64_t sgi = l.nseg - 1; sgi >= 0; --sgi) {
        const int64_t len = std::min(spec->checkpoint_every, spec->nsteps - sgi * spec->checkpoint_every);
        auto state = [&](int64_t t) { return t == 0 ? ckpt(sgi) : segst(t); };
        // the last segment's states are already there from the forward pass
        for (int64_t t = 1; t < len && sgi < l.nseg - 1; ++t) {
            e = launch_step(c->p.lattice, c->p.storage, c->p.order, c->grid, c->k64, c->k32, c->links, c->gray,
                            state(t - 1), state(t), c->block_x, c->block_y, c->launch_flags, st);
            if (e != hipSuccess) return fail_hip(e, "segment recompute");
        }
        for (int64_t t = len - 1; t >= 0; --t) {
            e = launch_adjoint(c->p.lattice, c->p.storage, c->p.order, c->grid, c->k64, c->k32, state(t), lam_in,
                               lam_out, c->gray, c->links, dmask, gpart, st);
            if (e != hipSuccess) return fail_hip(e, "adjoint step");
            std::swap(lam_in, lam_out);
        }
    }
    e = launch_sum(gpart, na, kGradPartialsHost, sums + 1, st);
    double h[1 + kGradPartialsHost];
    if (e == hipSuccess) e = hipMemcpyAsync(h, sums, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail_hip(e, "gradient read-back");
    *objective = h[0];
    if (dtau) *dtau = h[7];
    if (dtensor) {
        const int d = c->pr.d;
        // dJ/dK: the symmetric part, which is all that the derivatives below depend on (K and
        // the caller's tensor are symmetric)
        const double G[9] = {h[1], h[4], h[5], h[4], h[2], h[6], h[5], h[6], h[3]};
        double D[9] = {0};  // dJ/dT as a general matrix
        if (c->p.tensor_kind == LBM_TENSOR_THETA) {
            for (int i = 0; i < 9; ++i) D[i] = G[i] / kCs2;  // K = T / cs^2 - I
        } else {
            // T = A, K = A^-1 - I: dJ/dA = -A^-1 G A^-1. T = A~ with A^-1 = s A~^-1 and
            // s = det(A~)^(1/d): dA^-1 = s [tr(A~^-1 dA~) A~^-1 / d - A~^-1 dA~ A~^-1], so
            // dJ/dA~ = [tr(G^T A^-1) A^-1 / d - A^-1 G A^-1] / s (A^-1 is symmetric).
            const double *ai = c->pr.dv.ainv;  // zero outside the d x d block
            double t[9] = {0};
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    for (int k2 = 0; k2 < 3; ++k2) t[a * 3 + b] += ai[a * 3 + k2] * G[k2 * 3 + b];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double v = 0.0;
                    for (int k2 = 0; k2 < 3; ++k2) v += t[a * 3 + k2] * ai[k2 * 3 + b];
                    D[a * 3 + b] = -v;
                }
            if (c->p.tensor_kind == LBM_TENSOR_ATILDE) {
                double T[9];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) T[a * 3 + b] = 0.5 * (c->p.tensor[a * 3 + b] + c->p.tensor[b * 3 + a]);
                const double det = d == 2 ? T[0] * T[4] - T[1] * T[3]
                                          : T[0] * (T[4] * T[8] - T[5] * T[7]) - T[1] * (T[3] * T[8] - T[5] * T[6]) +
                                                T[2] * (T[3] * T[7] - T[4] * T[6]);
                const double sc = std::pow(det, 1.0 / d);
                double tr = 0.0;
                for (int i = 0; i < 9; ++i) tr += G[i] * ai[i];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) D[a * 3 + b] = (D[a * 3 + b] + tr * ai[a * 3 + b] / d) / sc;
            }
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double v = 0.0;
                if (a < d && b < d) v = (a == b) ? D[a * 3 + a] : D[a * 3 + b] + D[b * 3 + a];
                dtensor[a * 3 + b] = v;
            }
    }
    return LBM_OK;
}

int lbm_objective(lbm_ctx *c, int32_t objective, int64_t outlet_plane, double *value)
{
    if (!c || !value) return fail(LBM_ERR_ARG, "NULL argument");
    if (objective != 0 && objective != 1) return fail(LBM_ERR_ARG, "objective must be 0 or 1");
    if (objective == 0 && (outlet_plane < 0 || outlet_plane >= c->p.nx))
        return fail(LBM_ERR_ARG, "outlet_plane %lld outside 0..%lld", (long long)outlet_plane,
                    (long long)(c->p.nx - 1));
    // the moments partials hold one double per seed work-group, the totals slot the sum
    double *jpart = c->partials;
    double *sum = c->partials + kPartials * (size_t)moments_groups(c->grid);
    hipError_t e = launch_seed(c->p.lattice, c->p.storage, c->grid, c->k64, c->k32, c->pop[c->cur], nullptr, jpart,
                               objective, (int)outlet_plane, c->links, c->stream);
    if (e == hipSuccess) e = launch_sum(jpart, moments_groups(c->grid), 1, sum, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(value, sum, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? LBM_OK : fail_hip(e, "objective evaluation");
}

void lbm_destroy(lbm_ctx *c) { delete c; }

const char *lbm_last_error(void) { return g_last_error.c_str(); }

int lbm_stream_copy(void *dst, const void *src, int64_t nbytes, void *stream)
{
    if (!dst || !src || nbytes < 0 || nbytes % 16 != 0)
        return fail(LBM_ERR_ARG, "copy needs non-NULL buffers and a byte count that is a multiple of 16");
    hipError_t e = launch_copy(dst, src, nbytes, (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : fail_hip(e, "copy kernel launch");
}

}  // extern "C"
