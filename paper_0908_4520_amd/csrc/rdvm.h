// rdvm.h -- device descriptors of the reduced discrete-velocity model of the forced standing
// shear wave (section 4, Eqs. ga and gb): per instance, M Gauss-Hermite velocities xi_k in the
// wave direction times N_w cells, state G~[k * N_w + j] in FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int kRdvmMaxNodes = 64;    // velocities per instance
constexpr int kRdvmBlock = 256;      // threads per workgroup = the largest N_w (one cell each)
constexpr int kRdvmMaxValues = 16384; // M * N_w: the state lives in LDS (128 KiB)

struct RdvmInst {
    int32_t M, nw;
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
};

// One workgroup per instance; lds_bytes = 8 * (max M * N_w + 4).
hipError_t launch_rdvm(const RdvmArgs &a, uint32_t count, size_t lds_bytes, hipStream_t s);
hipError_t rdvm_allow_lds(size_t lds_bytes);

}  // namespace lbm
