// cell.hpp -- per-cell device building blocks of the BGK update shared by every kernel file:
// storage conversions, the periodic neighbourhood of a cell, population addressing, the
// folded anisotropic equilibrium, its moments and one collision.
//
// The arithmetic contract (eq:3rd_order_equilibrium with cs^2 = 1/3, per opposite pair
// c / -c):
//   f^eq = rho r + w rho P'(s),  r = w (1 + 1.5 c.K.c - 0.5 tr K),
//   P'   = 4.5 u^2 - 1.5 |s|^2  +/-  [u (A - 4.5 |s|^2 + 4.5 u^2) - 3 c.(K s)]   (order 3)
//   P'   = 4.5 u^2 - 1.5 |s|^2  +/-  3 u                                         (order 2)
// with u = c.s and A = 3 + 4.5 c.K.c - 1.5 tr K, evaluated on stored deviations g = f - sigma.
// Contraction is off and every fused multiply-add is explicit, so a cell's result is fixed by
// this source and identical in every kernel that calls these functions.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.hpp"

#pragma clang fp contract(off)

namespace lbm {
namespace cell {

__device__ inline float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---- storage conversions ---------------------------------------------------------------

template <typename S> struct Conv;
template <> struct Conv<double> {
    using C = double;
    __device__ static double ld(double v) { return v; }
    __device__ static double st(double v) { return v; }
};
template <> struct Conv<float> {
    using C = float;
    __device__ static float ld(float v) { return v; }
    __device__ static float st(float v) { return v; }
};
template <> struct Conv<_Float16> {
    using C = float;
    __device__ static float ld(_Float16 v) { return (float)v; }
    __device__ static _Float16 st(float v) { return (_Float16)v; }  // round to nearest even
};
template <> struct Conv<__bf16> {
    using C = float;
    __device__ static float ld(__bf16 v) { return (float)v; }
    __device__ static __bf16 st(float v) { return (__bf16)v; }  // round to nearest even
};

// The moment closure runs for FP32 storage only (see collide_cell).
template <typename S> constexpr bool kClose = std::is_same<S, float>::value;

// ---- neighbourhood and population addressing ----------------------------------------
//
// Population arrays use the blocked layout of Grid. Because `rows` divides ny, the storage
// offset from a cell to a neighbour is a sum of one term per axis -- the x-term depends on x
// only, the y-term on y only, the z-term on z only -- so a neighbour costs the same few adds
// as in a plain plane-per-direction layout, with the periodic wrap folded into the terms.

// floor(n / d) and n mod d from m = floor(2^32 / d) (0xffffffff for d = 1): the estimate
// umulhi(n, m) is exact or one too small for every 32-bit n, so one correction suffices
// (division by invariant integers using multiplication, Granlund and Montgomery).
__device__ inline uint32_t div_by(uint32_t n, uint32_t m, uint32_t d, uint32_t &rem)
{
    uint32_t q = __umulhi(n, m);
    uint32_t r = n - q * d;
    if (r >= d) {
        r -= d;
        ++q;
    }
    rem = r;
    return q;
}

// Offsets (in elements, modulo 2^32) from a cell to its periodic neighbours at coordinate -1
// and +1 along one axis.
struct AxisOff {
    uint32_t m1, p1;
};

__device__ inline AxisOff axis_off(uint32_t v, uint32_t n, uint32_t stride)
{
    AxisOff o;
    o.m1 = (v == 0) ? (n - 1u) * stride : 0u - stride;
    o.p1 = (v == n - 1u) ? 0u - (n - 1u) * stride : stride;
    return o;
}

// Offset to the cell x - c for one velocity component c in {-1, 0, 1} (a constant after
// unrolling).
__device__ inline uint32_t back(const AxisOff &o, int c) { return c > 0 ? o.m1 : (c < 0 ? o.p1 : 0u); }

// Storage offset of row y within its z-plane, and the offsets to rows y - 1 and y + 1.
__device__ inline uint32_t row_off(const Grid &g, uint32_t y, AxisOff &oy)
{
    uint32_t yr;
    const uint32_t yb = div_by(y, g.mr, g.rows, yr);
    const uint32_t last = g.zs - g.bq + (g.rows - 1u) * (uint32_t)g.nx;  // row ny - 1
    const uint32_t cross = g.bq - (g.rows - 1u) * (uint32_t)g.nx;        // row to the next block's first
    oy.m1 = (y == 0u) ? last : (yr == 0u ? 0u - cross : 0u - (uint32_t)g.nx);
    oy.p1 = (y == (uint32_t)g.ny - 1u) ? 0u - last : (yr == g.rows - 1u ? cross : (uint32_t)g.nx);
    return yb * g.bq + yr * (uint32_t)g.nx;
}

// Location of one population: an element offset that is the same for the whole work-group
// (the z-plane) plus a per-lane 32-bit index.
struct Ref {
    uint64_t zo;
    uint32_t idx;
};

// A cell of a single grid. Every kernel over a single grid runs work-groups inside one
// z-plane, so the z-plane offsets are work-group uniform (scalar registers) and the per-lane
// index stays within one z-plane, whatever the size of the grid.
struct Cell {
    uint32_t own;         // canonical index x + nx (y + ny z)
    uint32_t at;          // storage index within the z-plane
    AxisOff ox, oy;
    uint64_t z0, zm, zp;  // element offsets of the z-planes z, z - 1 and z + 1 (periodic)
};

__device__ inline Cell cell_of(const Grid &g, int32_t x, int32_t y, int32_t z)
{
    Cell c;
    c.own = (uint32_t)((z * g.ny + y) * g.nx + x);
    c.ox = axis_off((uint32_t)x, (uint32_t)g.nx, 1u);
    c.at = row_off(g, (uint32_t)y, c.oy) + (uint32_t)x;
    c.z0 = (uint64_t)z * g.zs;
    c.zm = (uint64_t)(z == 0 ? g.nz - 1 : z - 1) * g.zs;
    c.zp = (uint64_t)(z == g.nz - 1 ? 0 : z + 1) * g.zs;
    return c;
}

// A cell of a batched domain, addressed with one 32-bit index over the domain (whose
// populations stay below 4 GiB). Batched domains use linear blocks instead of row blocks:
// block b holds cells [b B, (b + 1) B) of the canonical order (B = 2^lb, a multiple of the
// 256-cell tile), its q direction planes back to back, so canonical cell n of direction i is
//     (n >> lb) q B + i B + (n mod B).
// A tile then stores whole cache lines in every plane however short the domain's rows are.
// With lb = 31 and bq = 0 the same cell addresses canonical order (canon_cell_of).
struct FlatCell {
    uint32_t own;  // canonical index
    uint32_t lb;   // log2 of the cells per block
    uint32_t bq;   // q B: elements per block
    AxisOff ox, oy, oz;
};

__device__ inline uint32_t lin_at(const FlatCell &c, uint32_t n) { return (n >> c.lb) * c.bq + (n & ((1u << c.lb) - 1u)); }

__device__ inline FlatCell flat_cell_of(const Grid &g, uint32_t x, uint32_t y, uint32_t z)
{
    FlatCell c;
    c.own = (z * (uint32_t)g.ny + y) * (uint32_t)g.nx + x;
    c.lb = g.lb;
    c.bq = g.bq;
    c.ox = axis_off(x, (uint32_t)g.nx, 1u);
    c.oy = axis_off(y, (uint32_t)g.ny, (uint32_t)g.nx);
    c.oz = axis_off(z, (uint32_t)g.nz, (uint32_t)g.nx * (uint32_t)g.ny);
    return c;
}

__device__ inline FlatCell canon_cell_of(const Grid &g, uint32_t x, uint32_t y, uint32_t z)
{
    FlatCell c = flat_cell_of(g, x, y, z);
    c.lb = 31u;
    c.bq = 0u;
    return c;
}

__device__ inline Ref own_ref(const Cell &c) { return Ref{c.z0, c.at}; }
__device__ inline Ref own_ref(const FlatCell &c) { return Ref{0u, lin_at(c, c.own)}; }

// The cell x - (cx, cy, cz), periodic (src_plus passes the pair's c, src_minus its -c).
__device__ inline Ref nbr(const Cell &c, int cx, int cy, int cz)
{
    return Ref{cz > 0 ? c.zm : (cz < 0 ? c.zp : c.z0), c.at + back(c.ox, cx) + back(c.oy, cy)};
}
__device__ inline Ref nbr(const FlatCell &c, int cx, int cy, int cz)
{
    return Ref{0u, lin_at(c, c.own + back(c.ox, cx) + back(c.oy, cy) + back(c.oz, cz))};
}

// x - c and x + c for the velocity c of pair p.
template <int LAT, typename CellT> __device__ inline Ref src_plus(const CellT &c, int p)
{
    const PairRow v = Lattice<LAT>::pair(p);
    return nbr(c, v.cx, v.cy, v.cz);
}
template <int LAT, typename CellT> __device__ inline Ref src_minus(const CellT &c, int p)
{
    const PairRow v = Lattice<LAT>::pair(p);
    return nbr(c, -v.cx, -v.cy, -v.cz);
}

// Element of direction i at r in a population array (plane bases and the z-plane offset are
// work-group uniform; the per-lane offset stays a 32-bit byte offset).
template <typename S> __device__ inline const S *pop_base(const S *base, const Grid &g, int i, const Ref &r)
{
    return base + r.zo + (uint64_t)i * g.bc;
}
template <typename S> __device__ inline S *pop_base(S *base, const Grid &g, int i, const Ref &r)
{
    return base + r.zo + (uint64_t)i * g.bc;
}

// Element `idx` of canonical plane i of a [q][n] array.
template <typename S> __device__ inline const S *plane(const S *base, int i, uint32_t n)
{
    return base + (size_t)i * n;
}
template <typename S> __device__ inline S *plane(S *base, int i, uint32_t n) { return base + (size_t)i * n; }

template <typename S> __device__ inline S ld_at(const S *p, uint32_t idx)
{
    return *reinterpret_cast<const S *>(reinterpret_cast<const char *>(p) + (uint32_t)(idx * (uint32_t)sizeof(S)));
}
template <typename S> __device__ inline void st_at(S *p, uint32_t idx, S v)
{
    *reinterpret_cast<S *>(reinterpret_cast<char *>(p) + (uint32_t)(idx * (uint32_t)sizeof(S))) = v;
}
// Streaming stores of one cell's q populations through a buffer resource based at the cell's
// z-plane: all q stores share the lane's byte offset and differ by a work-group-uniform offset
// (direction i at i blocks-per-direction), so they need no per-lane address arithmetic. Offsets
// stay below 4 GiB because one z-plane of populations does. Cache policy: non-temporal. A step's
// output is not read again within the step, and keeping it out of the caches leaves them to the
// lines the shifted pulls share (measured faster; those loads stay cached for that reason).
struct PlaneStores {
    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t lane_off;    // bytes from the z-plane base to direction 0 of the cell
    uint32_t plane_step;  // bytes between consecutive direction planes of a block
};

template <typename S> __device__ inline PlaneStores plane_stores(S *base, const Grid &g, const Ref &r)
{
    PlaneStores ps;
    // raw buffer: stride 0, the largest record count, the data format word of gfx9 raw buffers.
    // The base is the z-plane's, the same for the whole work-group; readfirstlane keeps it in
    // scalar registers even where the compiler cannot prove that (otherwise every buffer access
    // becomes a loop over the distinct descriptors of the wave)
    const uint64_t a = reinterpret_cast<uint64_t>(base + r.zo);
    const uint64_t u = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32)) << 32) |
                       (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
    ps.rsrc = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<S *>(u), (short)0, -1, 0x00020000);
    ps.lane_off = r.idx * (uint32_t)sizeof(S);
    ps.plane_step = g.bc * (uint32_t)sizeof(S);
    return ps;
}

// Store of direction i through a PlaneStores; AUX is the cache policy (2: non-temporal, 0: the
// default, for data read again soon).
template <int AUX, typename S> __device__ inline void st_plane_aux(const PlaneStores &ps, int i, S v)
{
    // the scalar offset is uniform; readfirstlane says so where control flow has hidden it from
    // the compiler (a value merged after a divergent branch), which would otherwise wrap the
    // store in a loop over the distinct values
    const int soff = __builtin_amdgcn_readfirstlane((int)((uint32_t)i * ps.plane_step));
    if constexpr (sizeof(S) == 2)
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), ps.rsrc, (int)ps.lane_off, soff, AUX);
    else if constexpr (sizeof(S) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), ps.rsrc, (int)ps.lane_off, soff, AUX);
    else
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) uint32_t, v),
                                              ps.rsrc, (int)ps.lane_off, soff, AUX);
}
template <typename S> __device__ inline void st_plane(const PlaneStores &ps, int i, S v) { st_plane_aux<2>(ps, i, v); }

// Non-temporal load of one element (16-bit types go through their bit pattern).
template <typename S> __device__ inline S ld_nt_at(const S *p, uint32_t idx)
{
    const char *a = reinterpret_cast<const char *>(p) + (uint32_t)(idx * (uint32_t)sizeof(S));
    if constexpr (sizeof(S) == 2) {
        return __builtin_bit_cast(S, __builtin_nontemporal_load(reinterpret_cast<const uint16_t *>(a)));
    } else {
        return __builtin_nontemporal_load(reinterpret_cast<const S *>(a));
    }
}

template <typename S> __device__ inline S ld_pop(const S *base, const Grid &g, int i, const Ref &r)
{
    return ld_at(pop_base(base, g, i, r), r.idx);
}

// ---- one-lane shifts across a 64-lane wave ----------------------------------------------
//
// DPP wave shifts: kFromLeft gives lane l the value of lane l - 1 (wave_shr:1) and kFromRight
// the value of lane l + 1 (wave_shl:1); the lane with no source in the wave (0, resp. 63)
// receives `edge`. They need all 64 lanes active.
constexpr int kFromLeft = 0x138;
constexpr int kFromRight = 0x130;

template <int CTRL> __device__ inline float wave_shift(float edge, float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                                 __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ inline double wave_shift(double edge, double v)
{
    const uint64_t e = __builtin_bit_cast(uint64_t, edge), w = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)e, (int)(uint32_t)w, CTRL, 0xF, 0xF, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(e >> 32), (int)(uint32_t)(w >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <typename S> __device__ inline void st_pop(S *base, const Grid &g, int i, const Ref &r, S v)
{
    st_at(pop_base(base, g, i, r), r.idx, v);
}

// Issue order of a cell's q pulls: by source z-plane (z - 1, z, z + 1), then by direction
// index, which is ascending address order in the population layouts. Direction 2p+1 (+c of
// pair p) is pulled from x - c and 2p+2 (-c) from x + c. On the bare D3Q19 pattern this order
// measured 2% faster than pair order (the loads of one wave then walk memory upwards).
template <int LAT> struct PullOrder {
    int dir[Lattice<LAT>::Q];
    __host__ __device__ constexpr PullOrder() : dir()
    {
        int k = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int i = 0; i < Lattice<LAT>::Q; ++i) {
                const int cz = i == 0 ? 0 : Lattice<LAT>::pair((i - 1) / 2).cz;
                const int src = i == 0 ? 0 : ((i & 1) ? -cz : cz);
                if (src == dz) dir[k++] = i;
            }
    }
};

// ---- the collision -----------------------------------------------------------------------

// Per-cell quantities of the folded equilibrium that every velocity pair shares.
template <typename C> struct EqCell {
    C rho, drho, sx, sy, sz, k3x, k3y, k3z, even0, bq;  // k3 = -3 K s
};

template <typename C>
__device__ inline EqCell<C> eq_cell(const StepConsts<C> &k, C drho, C rho, C sx, C sy, C sz)
{
    EqCell<C> e;
    e.rho = rho;
    e.drho = drho;
    e.sx = sx;
    e.sy = sy;
    e.sz = sz;
    const C usq = fmad(sx, sx, fmad(sy, sy, sz * sz));
    e.k3x = fmad(k.km3[0], sx, fmad(k.km3[3], sy, k.km3[4] * sz));
    e.k3y = fmad(k.km3[3], sx, fmad(k.km3[1], sy, k.km3[5] * sz));
    e.k3z = fmad(k.km3[4], sx, fmad(k.km3[5], sy, k.km3[2] * sz));
    e.even0 = C(-1.5) * usq;
    e.bq = C(-4.5) * usq;
    return e;
}

// c . (ax, ay, az) for c in {-1, 0, 1}^3 (c != 0), summed in x, y, z order from the first
// non-zero term: no leading 0 + term, which IEEE arithmetic keeps as an instruction.
template <typename C> __device__ inline C c_dot(int cx, int cy, int cz, C ax, C ay, C az)
{
    C r = cx != 0 ? (cx > 0 ? ax : -ax) : (cy != 0 ? (cy > 0 ? ay : -ay) : (cz > 0 ? az : -az));
    if (cx != 0 && cy != 0) r = cy > 0 ? r + ay : r - ay;
    if ((cx != 0 || cy != 0) && cz != 0) r = cz > 0 ? r + az : r - az;
    return r;
}

// g^eq of the rest velocity.
template <typename C> __device__ inline C eq_rest(const StepConsts<C> &k, const EqCell<C> &e)
{
    return fmad(k.w[0] * e.rho, e.even0, fmad(k.rest[0], e.drho, k.eoff[0]));
}

// Even and odd s-dependent parts of pair p's equilibrium: g^eq(+-c) = w rho (even +- odd) + base.
template <int LAT, int ORDER, typename C>
__device__ inline void eq_parts(const StepConsts<C> &k, const EqCell<C> &e, int p, C &even, C &odd)
{
    const PairRow v = Lattice<LAT>::pair(p);
    // u = c.s and -3 kc = c.(-3 K s) for c in {-1, 0, 1}^3
    const C u = c_dot(v.cx, v.cy, v.cz, e.sx, e.sy, e.sz);
    const C u2 = u * u;
    even = fmad(C(4.5), u2, e.even0);
    if constexpr (ORDER == 3) {
        const C k3c = c_dot(v.cx, v.cy, v.cz, e.k3x, e.k3y, e.k3z);
        odd = fmad(u, fmad(C(4.5), u2, k.a[p + 1] + e.bq), k3c);
    } else {
        odd = C(3) * u;
    }
}

// g^eq of the +c / -c members of pair p.
template <int LAT, int ORDER, typename C>
__device__ inline void eq_pair(const StepConsts<C> &k, const EqCell<C> &e, int p, C &ep, C &em)
{
    C even, odd;
    eq_parts<LAT, ORDER, C>(k, e, p, even, odd);
    const C wr = k.w[p + 1] * e.rho;
    const C base = fmad(k.rest[p + 1], e.drho, k.eoff[p + 1]);
    ep = fmad(wr, even + odd, base);
    em = fmad(wr, even - odd, base);
}

// Equilibrium deviations g^eq = f^eq - sigma of every direction for one cell with density
// rho = rho0 + drho and lattice velocity s: eqp[0] is the rest velocity, eqp[p+1] / eqm[p+1]
// are the +c / -c members of pair p.
template <int LAT, int ORDER, typename C>
__device__ inline void equilibrium_pairs(const StepConsts<C> &k, C drho, C rho, C sx, C sy, C sz, C *eqp, C *eqm)
{
    const EqCell<C> e = eq_cell(k, drho, rho, sx, sy, sz);
    eqp[0] = eq_rest(k, e);
#pragma unroll
    for (int p = 0; p < Lattice<LAT>::NP; ++p) eq_pair<LAT, ORDER, C>(k, e, p, eqp[p + 1], eqm[p + 1]);
}

// BGK relaxation g* = g + omega (g^eq - g) written as (1 - omega) g + omega g^eq, with
// omega g^eq assembled from constants that carry the factor omega (the equilibrium's own
// constants times omega): one operation per direction fewer than forming g^eq first.
template <int LAT, int ORDER, typename C>
__device__ inline void relax_pairs(const StepConsts<C> &k, C drho, C rho, C sx, C sy, C sz, C *gp, C *gm)
{
    const EqCell<C> e = eq_cell(k, drho, rho, sx, sy, sz);
    gp[0] = fmad(k.keep, gp[0], fmad(k.ow[0] * e.rho, e.even0, fmad(k.orest[0], e.drho, k.oeoff[0])));
#pragma unroll
    for (int p = 0; p < Lattice<LAT>::NP; ++p) {
        C even, odd;
        eq_parts<LAT, ORDER, C>(k, e, p, even, odd);
        const C owr = k.ow[p + 1] * e.rho;
        const C obase = fmad(k.orest[p + 1], e.drho, k.oeoff[p + 1]);
        gp[p + 1] = fmad(k.keep, gp[p + 1], fmad(owr, even + odd, obase));
        gm[p + 1] = fmad(k.keep, gm[p + 1], fmad(owr, even - odd, obase));
    }
}

// BGK with the exact-difference force, g* = (1 - omega) (g - g^eq(s)) + g^eq(s + F/rho). The
// two equilibria share w rho and the constant part, so with E, O the even and odd parts at s
// and E', O' at s + F/rho each pair member is
// g*+- = (1 - omega) g+- + w rho [(E' - (1 - omega) E) +- (O' - (1 - omega) O)] + omega base:
// the pair's two differences are formed once and neither equilibrium is assembled. With F = 0
// this is plain BGK.
// CLOSE (FP32 storage) then closes the conserved moments of g* itself: the axis pairs take the
// difference between j + F and the momentum of g*, and the rest population takes drho minus
// the other populations, so sum_i g*_i = drho and sum_i g*_i c_i = j + F hold up to
// per-operation rounding. In exact arithmetic these are the corrections that closing each
// equilibrium on its own momentum (close_moments) carries into g*: the FP32 constants' rounding
// is removed the same way, without assembling and closing two equilibria.
template <int LAT, int ORDER, bool CLOSE, typename C>
__device__ inline void relax_forced_pairs(const StepConsts<C> &k, C drho, C rho, C inv, C jx, C jy, C jz, C *gp,
                                          C *gm)
{
    using L = Lattice<LAT>;
    const C fjx = jx + k.force[0], fjy = jy + k.force[1], fjz = jz + k.force[2];
    const EqCell<C> e = eq_cell(k, drho, rho, jx * inv, jy * inv, jz * inv);
    const EqCell<C> f = eq_cell(k, drho, rho, fjx * inv, fjy * inv, fjz * inv);
    const C keep = k.keep;
    if constexpr (!CLOSE)
        gp[0] = fmad(keep, gp[0],
                     fmad(k.w[0] * rho, fmad(-keep, e.even0, f.even0), fmad(k.orest[0], drho, k.oeoff[0])));
    C mass = C(0), mx = C(0), my = C(0), mz = C(0);
    bool bx = false, by = false, bz = false;
#pragma unroll
    for (int p = 0; p < L::NP; ++p) {
        C even, odd, feven, fodd;
        eq_parts<LAT, ORDER, C>(k, e, p, even, odd);
        eq_parts<LAT, ORDER, C>(k, f, p, feven, fodd);
        const C de = fmad(-keep, even, feven), dd = fmad(-keep, odd, fodd);
        const C wr = k.w[p + 1] * rho;
        const C obase = fmad(k.orest[p + 1], drho, k.oeoff[p + 1]);
        gp[p + 1] = fmad(keep, gp[p + 1], fmad(wr, de + dd, obase));
        gm[p + 1] = fmad(keep, gm[p + 1], fmad(wr, de - dd, obase));
        if constexpr (CLOSE) {
            // mass and momentum of g*, each from its first term
            const PairRow v = L::pair(p);
            const C sum = gp[p + 1] + gm[p + 1], dif = gp[p + 1] - gm[p + 1];
            mass = p == 0 ? sum : mass + sum;
            if (v.cx != 0) mx = bx ? (v.cx > 0 ? mx + dif : mx - dif) : (v.cx > 0 ? dif : -dif), bx = true;
            if (v.cy != 0) my = by ? (v.cy > 0 ? my + dif : my - dif) : (v.cy > 0 ? dif : -dif), by = true;
            if (v.cz != 0) mz = bz ? (v.cz > 0 ? mz + dif : mz - dif) : (v.cz > 0 ? dif : -dif), bz = true;
        }
    }
    if constexpr (CLOSE) {
        static_assert(L::pair(0).cx == 1 && L::pair(1).cy == 1, "axis pairs come first");
        const C hx = C(0.5) * (fjx - mx);
        const C hy = C(0.5) * (fjy - my);
        gp[1] += hx;
        gm[1] -= hx;
        gp[2] += hy;
        gm[2] -= hy;
        if constexpr (L::D == 3) {
            static_assert(L::D == 2 || L::pair(2).cz == 1, "axis pairs come first");
            const C hz = C(0.5) * (fjz - mz);
            gp[3] += hz;
            gm[3] -= hz;
        }
        gp[0] = drho - mass;
    }
}

template <int LAT, typename C> __device__ inline void moments_of(const C *gp, const C *gm, C &drho, C &jx, C &jy, C &jz)
{
    using L = Lattice<LAT>;
    drho = gp[0];
    // each momentum component starts from its first contribution (no leading 0 + term)
    bool bx = false, by = false, bz = false;
    jx = jy = jz = C(0);
#pragma unroll
    for (int p = 0; p < L::NP; ++p) {
        const PairRow v = L::pair(p);
        drho += gp[p + 1] + gm[p + 1];
        const C dif = gp[p + 1] - gm[p + 1];
        if (v.cx != 0) jx = bx ? (v.cx > 0 ? jx + dif : jx - dif) : (v.cx > 0 ? dif : -dif), bx = true;
        if (v.cy != 0) jy = by ? (v.cy > 0 ? jy + dif : jy - dif) : (v.cy > 0 ? dif : -dif), by = true;
        if (v.cz != 0) jz = bz ? (v.cz > 0 ? jz + dif : jz - dif) : (v.cz > 0 ? dif : -dif), bz = true;
    }
}

// Single-precision closure of the equilibrium's conserved moments. The FP32 constants of
// the equilibrium (w_i, the per-pair K terms) are rounded, and their rounding is the same in
// every cell and every step, so the computed g^eq carries a tiny but systematic excess of
// momentum (fl(1/18) alone is 7.5e-9 too large) that BGK injects into the flow each step.
// Here the momentum of the computed g^eq is measured and its deficit against j is put on the
// axis pairs (which carry no other correction), and the rest population takes the mass
// balance, so sum_i g^eq_i = drho and sum_i g^eq_i c_i = j hold up to per-operation
// rounding -- the discrete identities eq:a0discrete / eq:a1discrete require exactly that.
template <int LAT, typename C>
__device__ inline void close_moments(C *eqp, C *eqm, C drho, C jx, C jy, C jz)
{
    using L = Lattice<LAT>;
    C mx = C(0), my = C(0), mz = C(0), mass = C(0);
#pragma unroll
    for (int p = 0; p < L::NP; ++p) {
        const PairRow v = L::pair(p);
        mass += eqp[p + 1] + eqm[p + 1];
        const C dif = eqp[p + 1] - eqm[p + 1];
        if (v.cx > 0) mx += dif;
        if (v.cx < 0) mx -= dif;
        if (v.cy > 0) my += dif;
        if (v.cy < 0) my -= dif;
        if (v.cz > 0) mz += dif;
        if (v.cz < 0) mz -= dif;
    }
    static_assert(L::pair(0).cx == 1 && L::pair(1).cy == 1, "axis pairs come first");
    const C hx = C(0.5) * (jx - mx);
    const C hy = C(0.5) * (jy - my);
    eqp[1] += hx;
    eqm[1] -= hx;
    eqp[2] += hy;
    eqm[2] -= hy;
    if constexpr (L::D == 3) {
        static_assert(L::D == 2 || L::pair(2).cz == 1, "axis pairs come first");
        const C hz = C(0.5) * (jz - mz);
        eqp[3] += hz;
        eqm[3] -= hz;
    }
    eqp[0] = drho - mass;
}

// One BGK collision of eq:LBE_BGK on the pre-collision deviations of a cell (rest in gp[0],
// pair p in gp[p+1] / gm[p+1]); the arrays receive the post-collision deviations. With FORCE
// the body force is added by the exact-difference method,
// g* = g + w (g^eq(rho, s) - g) + [g^eq(rho, s + F/rho) - g^eq(rho, s)]
//    = (1 - w) (g - g^eq(rho, s)) + g^eq(rho, s + F/rho),
// which relax_forced_pairs evaluates from the two equilibria's even and odd parts, whether or
// not a force is set (F = 0 then gives plain BGK): one code path keeps the register count of
// these kernels down. CLOSE closes the conserved moments (close_moments on the equilibrium, or
// on g* in relax_forced_pairs); it
// matters where the stored deviations keep FP32 resolution (FP32 storage). With 16-bit storage
// each step's rounding of the deviations is about four orders above the drift the closure
// removes, so those kernels skip it (measured: FP16 e(s) 2.23e-3 with, 2.25e-3 without, after
// 1000 steps of the 256^3 vortex, and 3% less time).
template <int LAT, int ORDER, bool FORCE, typename C, bool CLOSE = (sizeof(C) == 4)>
__device__ inline void collide_cell(const StepConsts<C> &k, C *gp, C *gm)
{
    constexpr int NP = Lattice<LAT>::NP;
    C drho, jx, jy, jz;
    moments_of<LAT>(gp, gm, drho, jx, jy, jz);
    const C rho = k.rho0 + drho;
    const C inv = C(1) / rho;
    if constexpr (!CLOSE && !FORCE) {
        // without the closure g^eq itself is not needed: relax against omega g^eq directly
        relax_pairs<LAT, ORDER, C>(k, drho, rho, jx * inv, jy * inv, jz * inv, gp, gm);
        return;
    }
    if constexpr (FORCE) {
        // one form whether or not a force is set: a runtime branch between two forms took the
        // D3Q27 FP64 masked step from 208 to 255 VGPRs
        relax_forced_pairs<LAT, ORDER, CLOSE, C>(k, drho, rho, inv, jx, jy, jz, gp, gm);
        return;
    }
    C eqp[NP + 1], eqm[NP + 1];
    equilibrium_pairs<LAT, ORDER, C>(k, drho, rho, jx * inv, jy * inv, jz * inv, eqp, eqm);
    if constexpr (CLOSE) close_moments<LAT>(eqp, eqm, drho, jx, jy, jz);
    gp[0] = fmad(k.omega, eqp[0] - gp[0], gp[0]);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        gp[p + 1] = fmad(k.omega, eqp[p + 1] - gp[p + 1], gp[p + 1]);
        gm[p + 1] = fmad(k.omega, eqm[p + 1] - gm[p + 1], gm[p + 1]);
    }
}

// Where the canonical pre-collision population i of a cell lives in the state: normally the
// post-collision value of the upstream cell x - c_i (pull streaming); when that cell is solid,
// the cell's own post-collision value of the opposite direction (halfway bounce-back). The
// link word has bit i set in the second case. A slot keeps both candidates. When they lie in
// the same z-plane (c_z = 0, or a flat cell), both are offsets from one work-group-uniform
// plane base and resolving the slot selects a 32-bit index; otherwise it selects between two
// uniform plane bases.
struct Slot {
    bool bounce;
    bool same_z;  // a constant after unrolling
    int own_plane, src_plane;
    Ref own, src;
};

__device__ inline bool same_z(const Cell &, int cz) { return cz == 0; }
__device__ inline bool same_z(const FlatCell &, int) { return true; }

template <int LAT, typename CellT> __device__ inline Slot slot_plus(const CellT &c, int p, uint32_t links)
{
    const bool bounce = (links >> (2 * p + 1) & 1u) != 0u;
    return Slot{bounce, same_z(c, Lattice<LAT>::pair(p).cz), 2 * p + 2, 2 * p + 1, own_ref(c), src_plus<LAT>(c, p)};
}

template <int LAT, typename CellT> __device__ inline Slot slot_minus(const CellT &c, int p, uint32_t links)
{
    const bool bounce = (links >> (2 * p + 2) & 1u) != 0u;
    return Slot{bounce, same_z(c, Lattice<LAT>::pair(p).cz), 2 * p + 1, 2 * p + 2, own_ref(c), src_minus<LAT>(c, p)};
}

// A slot that is always the given plane at r (no bounce-back alternative).
__device__ inline Slot fixed_slot(int plane, const Ref &r) { return Slot{false, true, plane, plane, r, r}; }

// Plane base and per-lane index of a slot.
template <typename S> __device__ inline void slot_at(S *base, const Grid &g, const Slot &s, S *&p, uint32_t &idx)
{
    if (s.same_z) {
        const int lo = s.own_plane < s.src_plane ? s.own_plane : s.src_plane;
        p = pop_base(base, g, lo, s.src);
        const uint32_t io = s.own.idx + (uint32_t)(s.own_plane - lo) * g.bc;
        const uint32_t is = s.src.idx + (uint32_t)(s.src_plane - lo) * g.bc;
        idx = s.bounce ? io : is;
    } else {
        S *a = pop_base(base, g, s.own_plane, s.own), *b = pop_base(base, g, s.src_plane, s.src);
        p = s.bounce ? a : b;
        idx = s.bounce ? s.own.idx : s.src.idx;
    }
}

template <typename S> __device__ inline S ld_slot(const S *base, const Grid &g, const Slot &s)
{
    const S *p;
    uint32_t idx;
    slot_at(base, g, s, p, idx);
    return ld_at(p, idx);
}
// The same through a non-temporal load (data read once per launch).
template <typename S> __device__ inline S ld_slot_nt(const S *base, const Grid &g, const Slot &s)
{
    const S *p;
    uint32_t idx;
    slot_at(base, g, s, p, idx);
    return ld_nt_at(p, idx);
}
template <typename S> __device__ inline void st_slot(S *base, const Grid &g, const Slot &s, S v)
{
    S *p;
    uint32_t idx;
    slot_at(base, g, s, p, idx);
    st_at(p, idx, v);
}

}  // namespace cell
}  // namespace lbm
