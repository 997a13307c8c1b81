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

// A run of consecutive cells of one instance, updated by one workgroup (one cell per thread).
struct BatchChunk {
    int32_t inst;
    uint32_t start, count;
};

struct BatchArgs {
    const BatchInst *inst;
    const int32_t *order;       // per-instance form: workgroup b runs instance order[b]
    void *pool;
    const double *sin_tab;
    const double *bw;
    const float *bwf;           // the same rounded to FP32, per population one 16-byte record
                                // alpha_x, beta_x, alpha_y, beta_y at bwf[bw_off + 4 a]
    double *amp;                // amplitude log
    const int32_t *cur;         // per instance: buffer holding the state when the launch starts
    int64_t steps;
    int32_t record;             // record every this many steps (0 = never)
    int32_t record_first;       // also record before the first step
    // grid form
    const BatchChunk *chunks;   // chunks, grouped by instance
    const uint32_t *inst_first; // chunks of instance i: [inst_first[i], inst_first[i+1])
    const uint32_t *wg_first;   // chunks of workgroup b: wg_chunks[wg_first[b] .. wg_first[b+1])
    const uint32_t *wg_chunks;
    uint32_t nwg;               // workgroups of the grid form
    uint32_t nrec;              // amplitudes per instance in this run
    uint64_t *barrier;          // device-wide barrier arrivals (zeroed before the launch); 64 bits, so
                                // steps x workgroups never wraps it
    int32_t *abort;             // 1: a barrier wait exceeded its bound; 2: XCD placement differs from the plan
    uint32_t spin_limit;        // sleeps a barrier wait may take before it aborts the run
    double *partials;           // per chunk and record: FP64 sums
    // XCD-local grid form: workgroup slot s on XCD x runs the chunks of plan entry x * wg_per_xcd + s
    uint32_t *sync;             // per-XCD counters, see kSyncWords (zeroed before the launch)
    uint32_t nxcd, wg_per_xcd;
    // step profile of the grid forms (null = off; non-null launches the profiling kernel): for
    // steps ts_first .. ts_first + ts_count - 1 every workgroup stores three 100 MHz timestamps,
    // ts[(entry * ts_count + k) * 3 + {0,1,2}] = step start, its chunks done, the step's barrier
    // passed (entry = plan entry of the workgroup)
    uint64_t *ts;
    int64_t ts_first;
    int32_t ts_count;
};

// Per-XCD counters of the XCD-local form, one 128-byte line each: sync[x * kSyncStride] counts
// the slots taken on XCD x, the 64-bit word at sync + (kMaxXcd + x) * kSyncStride its barrier
// arrivals.
constexpr uint32_t kMaxXcd = 16, kSyncStride = 32, kSyncWords = 2 * kMaxXcd * kSyncStride;
// Default bound of a barrier wait, in sleeps of ~50 ns: seconds, far beyond any real step.
constexpr uint32_t kSpinLimit = 1u << 26;

// form 0: one workgroup per instance; form 1: chunks over a resident grid with a device-wide
// barrier per step; form 2: the same with every instance's chunks on one XCD and a barrier per XCD.
hipError_t launch_batch(int storage, int form, int block, const BatchArgs &a, uint32_t count, hipStream_t s);
int batch_grid_resident_per_cu(int storage, int form, int block);
// XCD (accelerator complex die) of every one of n workgroups of a small probe launch: out[b].
hipError_t probe_xcd(uint32_t *out, uint32_t n, hipStream_t s);
bool batch_supports(int lattice, int order, int storage);

}  // namespace lbm
