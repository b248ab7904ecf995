// ec_static.hip -- the allocation-free PCG solve (ec_solve_static): its
// iteration vectors, control records and partial sums live in a file-scope
// device array instead of a caller workspace, so a caller that cannot
// allocate device memory (code under graph capture, serving loops) only
// passes b and x.  Each GPU the library runs on holds its own copy of the
// array until the process ends; its device address is looked up once per
// device (the name of the array is a host-side stand-in in host code).
#include <hip/hip_runtime.h>

#include <mutex>

#include "ec.h"
#include "ec_internal.h"

static __device__ __align__(256) unsigned char scratch[EC_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char *g_scratch[kMaxDevices] = {};

// Device address of this GPU's scratch array (hipGetSymbolAddress with the
// device current, once per device).
hipError_t scratch_ptr(hipStream_t st, char **out)
{
    int dev = 0;
    hipError_t e = st ? hipStreamGetDevice(st, &dev) : hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        int cur = 0;
        e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = (char *)p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" int32_t ec_solve_static(ec_handle h, int32_t method, const double *b, double *x,
                                   const ec_solve_opts *opts, ec_solve_info *dev_info)
{
    char *p = nullptr;
    const hipError_t e = h ? scratch_ptr(ec::bound_stream(h), &p) : hipSuccess;
    return ec::solve_scratch(h, method, b, x, opts, dev_info, p, (int64_t)EC_STATIC_SCRATCH_BYTES,
                             e);
}
