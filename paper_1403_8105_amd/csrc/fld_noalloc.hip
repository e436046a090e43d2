// fld_noalloc.hip -- the nonlinear residual of a device fluence without any
// device allocation, for callers that cannot allocate (code under stream
// capture, serving loops, harnesses that forbid hipMalloc).
//
// Its temporaries (the limiter's D, the right-hand-side copy of r and the
// problem descriptor) live in `scratch`, a fixed array this file reserves on
// every GPU the library runs on, held until the process ends.  Calls on one
// GPU share that GPU's array: calls that overlap in time on one GPU race.
// Every call overwrites all of the scratch it reads, so nothing has to be
// cleared between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fld_internal.h"

namespace {

constexpr long long kMaxCells = FLD_NOALLOC_MAX_CELLS;
// D at 0, the copy of r after it, the descriptor on the next 256-byte boundary
constexpr size_t kFineOffset = ((size_t)2 * kMaxCells * sizeof(double) + 255) / 256 * 256;
constexpr size_t kScratchBytes = kFineOffset + (sizeof(fld::Fine) + 255) / 256 * 256;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
unsigned char *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up once per device with that
// device current.  The array's name in host code is only a host-side handle,
// so every use goes through this address.
hipError_t scratch_on(int device, unsigned char **out)
{
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess)
            return e;
        e = hipSetDevice(device);
        if (e != hipSuccess)
            return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        hipError_t e2 = hipSetDevice(prev);
        if (e != hipSuccess)
            return e;
        if (e2 != hipSuccess)
            return e2;
        if (!p)
            return hipErrorInvalidSymbol;
        g_scratch[device] = (unsigned char *)p;
    }
    *out = g_scratch[device];
    return hipSuccess;
}

}  // namespace

extern "C" fld_status fld_residual_device_noalloc(fld_context *c, const double *d_phi,
                                                  double *d_r_out, double *rel_out)
{
    if (!c || !rel_out)
        return FLD_ERR_INVALID_ARGUMENT;
    unsigned char *base = nullptr;
    if (scratch_on(fld::context_device(c), &base) != hipSuccess)
        return FLD_ERR_DEVICE;
    const fld::ResidualWork ws{(double *)base, (double *)base + kMaxCells,
                               (fld::Fine *)(base + kFineOffset), kMaxCells};
    return fld::residual_with_workspace(c, d_phi, d_r_out, rel_out, &ws);
}
