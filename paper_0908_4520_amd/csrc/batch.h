// batch.h -- device descriptors of the batched (persistent, many-instance) step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

struct BatchInst {
    int32_t lattice, order;     // velocity set id and Hermite order N
    int32_t nx, ny;
    uint32_t ncell, pstride;    // cells, elements between population planes
    uint64_t off;               // element offset of buffer 0 in the pool (buffer 1 follows)
    uint32_t sin_off;           // offset of this instance's sin(2 pi j / ny) table
    uint64_t amp_off;           // offset of this instance's amplitude series in the log
    uint32_t bw_off;            // offset of alpha_x, beta_x, alpha_y, beta_y (4 x kMaxQ) in bw
    double omega;
};

struct BatchArgs {
    const BatchInst *inst;
    const int32_t *order;       // workgroup b runs instance order[b]
    void *pool;
    const double *sin_tab;
    const double *bw;
    double *amp;                // amplitude log
    int32_t *cur;               // per instance: buffer holding the state (read at start, written at end)
    int64_t steps;
    int32_t record;             // record every this many steps (0 = never)
    int32_t record_first;       // also record before the first step
};

hipError_t launch_batch(int storage, int block, const BatchArgs &a, uint32_t count, hipStream_t s);
bool batch_supports(int lattice, int order, int storage);

}  // namespace lbm
