// noalloc.hip -- device scratch of the allocation-free entry points, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops).
//
// The scratch is one file-scope device array of kNoAllocDoubles doubles (about 96 KiB).  Every
// GPU the library runs on holds its own copy until the process ends, at its own address: in host
// code the array's name is not a device address, so the address is looked up once per device
// with hipGetSymbolAddress (that device current) and kept per device; kernels receive it as an
// argument.  Calls that overlap on one GPU share the array and race; each call writes every
// scratch value it later reads (nothing has to start at zero).
#include <mutex>

#include "noalloc.h"

namespace lbm {

static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
std::mutex g_mu;
double *g_ptr[kNoAllocMaxDevices] = {};
hipError_t g_status[kNoAllocMaxDevices] = {};
bool g_done[kNoAllocMaxDevices] = {};
}  // namespace

hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_done[device]) return g_status[device];
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    void *p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) (void)hipGetLastError();
    g_done[device] = true;
    g_status[device] = e;
    g_ptr[device] = e == hipSuccess ? static_cast<double *>(p) : nullptr;
    return e;
}

hipError_t noalloc_scratch(int device, double **ptr) {
    if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_done[device] || !g_ptr[device]) return hipErrorNotInitialized;
    *ptr = g_ptr[device];
    return hipSuccess;
}

__global__ __launch_bounds__(64) void k_scale2(const double *sums, double scale, double *out) {
    if (threadIdx.x < 2) out[threadIdx.x] = scale * sums[threadIdx.x];
}

hipError_t noalloc_scale2(const double *sums, double scale, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_scale2, dim3(1), dim3(64), 0, s, sums, scale, out);
    return hipGetLastError();
}

}  // namespace lbm
