// Kernel registry storage and the fixed-order final stage of the diagnostic reductions.
#include "kernels.h"

namespace lbm {

std::vector<KernelSet> &registry() {
    static std::vector<KernelSet> r;
    return r;
}

// One block of 64 threads: thread k < width adds partials[b][k] for b = 0..nblocks-1 in order.
__global__ __launch_bounds__(64) void k_diag_final(const double *partials, uint32_t nblocks, int width,
                                                   double *out) {
    const int k = threadIdx.x;
    if (k >= width) return;
    double s = 0.0;
    for (uint32_t b = 0; b < nblocks; ++b) s += partials[(size_t)b * width + k];
    out[k] = s;
}

hipError_t diag_final(const double *partials, uint32_t nblocks, int width, double *out, hipStream_t s) {
    if (width < 1 || width > 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, s, partials, nblocks, width, out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_zero(int *p, uint32_t n) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t fill_zero(int *p, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_zero, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace lbm
