// noalloc.hip -- lbm_moments_static: the moments read-out of lbm_moments for callers that cannot
// allocate device memory. Its reduction partials and totals live in one file-scope device array
// of fixed size instead of the context's scratch buffer; nothing is allocated by the call.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lbm.h"
#include "common.hpp"
#include "host.hpp"

namespace {

// The partial sums of every work-group of a moments launch (at most kMomentGroups, whatever the
// grid) followed by the totals: (kMomentGroups + 1) kPartials doubles, in whole 256-byte units.
constexpr size_t kScratchBytes =
    ((size_t)(lbm::kMomentGroups + 1) * lbm::kPartials * sizeof(double) + 255) / 256 * 256;

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void *g_scratch_at[kMaxDevices];  // device address of `scratch` on each device (0: not looked up)

}  // namespace

// One copy per device, held until the process ends. Host code must not pass this name to a
// kernel or a copy: it is a host-side stand-in. scratch_on() gives the device's address.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// The address of `scratch` on `device`, looked up once per device with that device current.
hipError_t scratch_on(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(g_lock);
    if (!g_scratch_at[device]) {
        int current = 0;
        hipError_t e = hipGetDevice(&current);
        if (e != hipSuccess) return e;
        if (current != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t back = current != device ? hipSetDevice(current) : hipSuccess;
        if (e != hipSuccess) return e;
        if (back != hipSuccess) return back;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_at[device] = p;
    }
    *out = g_scratch_at[device];
    return hipSuccess;
}

}  // namespace

extern "C" int lbm_moments_static(lbm_ctx *c, double *rho, double *s, double *totals)
{
    using namespace lbm;
    using namespace lbm::host;
    if (!c) return fail(LBM_ERR_ARG, "ctx is NULL");
    const uint32_t groups = moments_groups(c->grid);
    const size_t need = ((size_t)groups + 1) * kPartials * sizeof(double);
    if (need > kScratchBytes)
        return fail(LBM_ERR_SIZE, "the moments reduction needs %zu bytes of scratch; the static array holds %zu",
                    need, kScratchBytes);
    int device = 0;
    hipError_t e = c->stream ? hipStreamGetDevice(c->stream, &device) : hipGetDevice(&device);
    if (e != hipSuccess) return fail_hip(e, "device of the context's stream");
    void *base = nullptr;
    e = scratch_on(device, &base);
    if (e != hipSuccess) return fail_hip(e, "address of the static scratch array");
    double *partials = (double *)base;
    return moments_with(c, rho, s, totals, partials, partials + kPartials * (size_t)groups);
}
