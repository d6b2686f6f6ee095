// host.hpp -- host-side helpers shared by the single-grid (capi.cpp) and batched (batch.cpp)
// parts of the C ABI: error reporting, parameter preparation and per-step constants.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <string>

#include "../../include/lbm.h"
#include "common.hpp"

namespace lbm {
namespace host {

constexpr double kCs2 = 1.0 / 3.0;

// Velocity set in the library's canonical order (rest, then +c / -c of each pair).
struct LatticeTable {
    int q, d, np;
    int c[kMaxQ][3];
    double w[kMaxQ];
    int opp[kMaxQ];
};

// Validated parameters with everything derived from them on the host.
struct Prepared {
    lbm_derived dv;
    LatticeTable lat;
    int d, q, bytes;
    uint32_t n;
};

// Message of the last failing call on this thread (lbm_last_error).
extern thread_local std::string g_last_error;

// Record a message for lbm_last_error and return `code`.
int fail(int code, const char *fmt, ...);
int fail_hip(hipError_t e, const char *what);

bool table_of(int lattice, LatticeTable &t);
int storage_bytes(int storage);

// Validate p and derive A^-1, K, omega, r_i and the shift; LBM_OK or a negative code.
int prepare(const lbm_params *p, Prepared &out);

// Kernel constants of one parameter set in arithmetic precision C.
template <typename C> StepConsts<C> consts_for(const lbm_params &p, const Prepared &pr);

// Target bytes of one direction plane of one block in the population layout (Grid): rows per
// block is the largest divisor of ny with rows * nx * bytes <= block_bytes(bytes), at least 1.
// Blocks of about this size keep a work-group's 2q population streams within one compact
// stretch of memory; measured on the D3Q19 256^3 step, 8 KiB was best for FP32 and FP16,
// 32 KiB for FP64.
constexpr int64_t block_bytes(int bytes) { return bytes == 8 ? 32768 : 8192; }

// Extents and population layout of an nx x ny x nz grid of q directions in `bytes`-byte
// storage (the caller has validated the sizes).
Grid grid_of(int64_t nx, int64_t ny, int64_t nz, int q, int bytes);

int64_t align256(int64_t b);
bool aligned256(const void *ptr);

}  // namespace host
}  // namespace lbm

// The context behind the opaque lbm_ctx handle (host memory only; the device buffers belong to
// the caller).
struct lbm_ctx {
    lbm_params p;
    lbm::host::Prepared pr;
    lbm::Grid grid;
    lbm::StepConsts<double> k64;
    lbm::StepConsts<float> k32;
    void *pop[2];
    int cur;                 // index of the buffer that holds the current state
    double *partials;        // reduction partials, then the totals (in the caller's scratch)
    uint32_t *links;         // null without a solid mask
    float *gray;             // null without a gray field
    hipStream_t stream;
    int64_t t;
    int block_x, block_y;
    int launch_flags;
};

namespace lbm {
namespace host {

// lbm_moments with the reduction partials (kPartials * moments_groups doubles) and the totals
// (kPartials doubles) at the given device addresses.
int moments_with(lbm_ctx *c, double *rho, double *s, double *totals, double *partials, double *dtot);

}  // namespace host
}  // namespace lbm
