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

// Grid-stride copy of n 16-byte words: aligned vector loads, non-temporal vector stores.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy16(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(src[i], dst + i);
}

hipError_t copy16(const void *src, void *dst, uint64_t words, uint32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_copy16, dim3(blocks), dim3(256), 0, s, static_cast<const u32x4 *>(src),
                       static_cast<u32x4 *>(dst), words);
    return hipGetLastError();
}

}  // namespace lbm
