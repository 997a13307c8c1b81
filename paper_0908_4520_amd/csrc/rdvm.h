// rdvm.h -- device descriptors of the reduced discrete-velocity model of the forced standing
// shear wave (section 4, Eqs. ga and gb): per instance, M Gauss-Hermite velocities xi_k in the
// wave direction times N_w cells, state G~[k * N_w + j] in FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int kRdvmMaxNodes = 64;    // velocities per instance
constexpr int kRdvmMaxCells = 256;   // N_w per instance
constexpr int kRdvmBlock = 512;      // threads per workgroup
constexpr int kRdvmMaxValues = 16384; // M * N_w: the state lives in LDS (128 KiB)

// Threads per cell P (a power of two, P * N_w <= kRdvmBlock, P <= 64 so a cell's threads sit in
// one wave); thread t serves cell t / P and the velocities k = t % P + q P.
inline int rdvm_threads_per_cell(int nw) {
    int P = 64;
    while (P > 1 && P * nw > kRdvmBlock) P >>= 1;
    return P;
}
// Velocity slots per thread of the kernel variants (those up to 8 keep their coefficients in
// registers and read every slot; padded slots cost LDS reads, hence the close spacing).
constexpr int kRdvmVariants = 6;
constexpr int kRdvmK[kRdvmVariants] = {4, 5, 6, 8, 16, 32};
// Velocities per thread, rounded up to a kernel variant (P >= 2 and M <= 64, so at most 32).
inline int rdvm_variant(int M, int nw) {
    const int P = rdvm_threads_per_cell(nw), k = (M + P - 1) / P;
    for (int g = 0; g < kRdvmVariants; ++g)
        if (k <= kRdvmK[g]) return kRdvmK[g];
    return kRdvmK[kRdvmVariants - 1];
}

struct RdvmInst {
    int32_t M, nw, P;     // velocities, cells, threads per cell
    double dt, omega, amp, freq;
    uint32_t node_off;    // nodes: xi[M], w[M], alpha[M], beta[M] (Beam-Warming coefficients)
    uint32_t tab_off;     // tabs: cos(2 pi j / nw)[nw], then sin[nw]
    uint64_t state_off;   // G~[k * nw + j] in the state pool
    uint64_t log_off;     // velocity record [nrec], then stress record [nrec]
};

struct RdvmArgs {
    const RdvmInst *inst;
    const double *nodes;
    const double *tabs;
    double *state;
    double *log;
    int64_t step0;        // steps taken before this launch (time origin of the force)
    int64_t steps;
    int32_t record;       // record after every `record` steps of this launch (0 = never)
    int32_t nrec;         // records per instance in this launch
    int32_t two;          // two state buffers in LDS (rdvm_two_buffers of the largest instance)
};

constexpr size_t kRdvmMaxLds = 160 * 1024;   // LDS per workgroup (gfx950)
constexpr int kRdvmTf = kRdvmBlock;           // force time factors tabulated at once (one per thread)

// One workgroup per instance of the list `index` (count entries), all of kernel variant K;
// lds_bytes = rdvm_lds_bytes(largest M * N_w, largest M, a.two).
// LDS: the state (two buffers when they fit, so that a step needs one barrier), the
// coefficients, two sums per wave and the force time factors of the next kRdvmTf steps.
inline size_t rdvm_lds_bytes(size_t values, int M, bool two) {
    return sizeof(double) * ((two ? 2 : 1) * values + 4 * (size_t)M + 2 * (kRdvmBlock / 64) + kRdvmTf);
}
inline bool rdvm_two_buffers(size_t values, int M) { return rdvm_lds_bytes(values, M, true) <= kRdvmMaxLds; }
hipError_t launch_rdvm(int K, const RdvmArgs &a, const int32_t *index, uint32_t count, size_t lds_bytes,
                       hipStream_t s);
hipError_t rdvm_allow_lds(size_t lds_bytes);

}  // namespace lbm
