// batch.hip -- many independent shear-wave instances advanced in one persistent launch.
//
// Three persistent forms, chosen by timing (lbm_batch_autotune):
//  * per-instance: each workgroup owns one whole instance for the run and loops over the
//    steps with a workgroup barrier between them; nothing synchronises across CUs, but the
//    run lasts as long as the largest instance takes on one CU;
//  * grid: every instance is cut into chunks of one cell per thread, the chunks are spread
//    over a grid that is small enough to be resident at once (largest-cost-first onto the
//    least-loaded workgroup), and all workgroups meet at a device-wide barrier after every
//    step.  The barrier spins on an agent-scope counter with a bounded number of sleeps; if
//    the bound is hit (workgroups not resident together) it raises an abort flag that every
//    workgroup checks, so all of them leave the loop and the host reports the failure.
//    Each XCD has its own L2 and the L2s are not coherent with each other, so every arrival
//    writes back and every departure invalidates the workgroup's whole L2: on a full grid that
//    is hundreds of L2 flushes per step, which stall the loads of every workgroup still working;
//  * XCD-local grid: the same chunks, but all chunks of an instance go to workgroups of one
//    XCD, so no data crosses an L2 and a step ends at a barrier of that XCD's workgroups only.
//    Stores are visible to the XCD once they reach its L2, so the barrier needs only a wait
//    for the stores and an L1 invalidate, no L2 writeback.  A workgroup reads which XCD it runs
//    on and takes the next slot there; one device-wide barrier at the start checks that every
//    XCD received the planned number of workgroups, and if not, every workgroup leaves before
//    touching the state and the host falls back to the device-wide form.
// Amplitudes: the sine projection of u_x is summed in FP64 per chunk (fixed order) and the
// per-instance sums are formed by a second kernel in a fixed order, so runs are bitwise
// reproducible.
#include "batch.h"
#include "kernels_impl.h"

namespace lbm {

// Lane moves within a quad (4 consecutive lanes): with nx = 4 a quad holds one whole periodic
// row, so quad rotations are the x-shifts.  quad_perm [p0,p1,p2,p3]: lane i takes lane p_i.
template <int CTRL>
__device__ __forceinline__ float quad_move(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double quad_move(double v) {
    const int2v x = __builtin_bit_cast(int2v, v);
    return __builtin_bit_cast(double, int2v{__builtin_amdgcn_mov_dpp(x.x, CTRL, 0xf, 0xf, false),
                                            __builtin_amdgcn_mov_dpp(x.y, CTRL, 0xf, 0xf, false)});
}
constexpr int kQuadXm1 = 3 | (0 << 2) | (1 << 4) | (2 << 6);   // lane i <- i-1 (mod 4): value at x-1
constexpr int kQuadXp1 = 1 | (2 << 2) | (3 << 4) | (0 << 6);   // lane i <- i+1 (mod 4): value at x+1
constexpr int kQuadX2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);    // lane i <- i+2 (mod 4): value at x+-2

template <class L, int S>
__device__ __forceinline__ typename Codec<S>::raw *inst_buffer(const BatchInst &in, const BatchArgs &a, int which) {
    return static_cast<typename Codec<S>::raw *>(a.pool) + in.off + (size_t)which * L::Q * in.pstride;
}

// Beam-Warming coefficients (alpha_x, beta_x, alpha_y, beta_y) of population i, in the
// collision's precision: the FP32 table holds the FP64 values rounded to nearest, one 16-byte
// record per population, so FP32 kernels take one load and no conversion per population.
template <class T>
__device__ __forceinline__ void bw_coefs(const BatchArgs &a, uint32_t off, int i, T &ax, T &bx, T &ay, T &by) {
    if constexpr (sizeof(T) == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 c = *reinterpret_cast<const f4 *>(a.bwf + off + 4 * i);
        ax = c.x, bx = c.y, ay = c.z, by = c.w;
    } else {
        ax = a.bw[off + 0 * kMaxQ + i], bx = a.bw[off + 1 * kMaxQ + i];
        ay = a.bw[off + 2 * kMaxQ + i], by = a.bw[off + 3 * kMaxQ + i];
    }
}

// Largest |c| over the velocity set's components.
template <class L>
constexpr int max_c() {
    int m = 0;
    for (int i = 0; i < L::Q; ++i)
        for (int d = 0; d < L::D; ++d) m = L::c[i][d] > m ? L::c[i][d] : (-L::c[i][d] > m ? -L::c[i][d] : m);
    return m;
}

// One step for cells [start, start + count) of an instance, one cell per thread (count <= the
// block size; with nx = 4 the start is a multiple of 4, so quads are whole rows).
// Addresses: a 64-bit base per population plane, the same for every lane (scalar registers), plus
// a 32-bit byte offset per lane that the load and store instructions add themselves.  The offsets
// are built from per-row and per-column parts shared by every population moving along that row
// or column, so a population costs at most one vector add for its address.  An instance holds at
// most 2^26 cells (checked by the host), so an offset within a plane stays below 2^31.
template <class L, int N, int S, bool BW, bool QUAD>
__device__ __forceinline__ void step_cells(const BatchInst &in, const BatchArgs &a, int cur, uint32_t start,
                                           uint32_t count) {
    using C = Codec<S>;
    using raw = typename C::raw;
    using T = typename C::T;
    constexpr uint32_t E = sizeof(raw);
    if (threadIdx.x >= count) return;
    const char *__restrict__ src = reinterpret_cast<const char *>(inst_buffer<L, S>(in, a, cur));
    char *__restrict__ dst = reinterpret_cast<char *>(inst_buffer<L, S>(in, a, cur ^ 1));
    const size_t psb = (size_t)in.pstride * E;   // bytes between population planes
    const int nx = in.nx, ny = in.ny;
    const uint32_t cell = start + threadIdx.x;
    const int x = (int)(cell % (uint32_t)nx), y = (int)(cell / (uint32_t)nx);
    auto load = [&](int i, uint32_t off) -> raw { return *reinterpret_cast<const raw *>(src + (size_t)i * psb + off); };
    T v[L::Q];
    if constexpr (!BW) {
        // grids at least max|c| wide and high (a uniform condition, so a scalar branch): one
        // conditional add or subtract wraps an index; smaller ones take the true modulo
        if (nx >= max_c<L>() && ny >= max_c<L>()) {
            static_for<L::Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const uint32_t rb = (uint32_t)(wrap_once(y - L::c[i][1], ny) * nx) * E;
                const uint32_t cb = (uint32_t)wrap_once(x - L::c[i][0], nx) * E;
                v[i] = C::dec(load(i, rb + cb));
            });
        } else {
            static_for<L::Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const uint32_t rb = (uint32_t)(imod(y - L::c[i][1], ny) * nx) * E;
                const uint32_t cb = (uint32_t)imod(x - L::c[i][0], nx) * E;
                v[i] = C::dec(load(i, rb + cb));
            });
        }
    } else {
        // byte offsets of the rows y, y -+ 1, y -+ 2 (the upwind side by the sign of xi_y) and of
        // the column x
        const uint32_t rowm[3] = {(uint32_t)(y * nx) * E, (uint32_t)(imod(y - 1, ny) * nx) * E,
                                  (uint32_t)(imod(y - 2, ny) * nx) * E};
        const uint32_t rowp[3] = {rowm[0], (uint32_t)(imod(y + 1, ny) * nx) * E, (uint32_t)(imod(y + 2, ny) * nx) * E};
        const uint32_t colx = (uint32_t)x * E;
        static_for<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr bool px = L::xi[i][0] > 0.0, py = L::xi[i][1] > 0.0;
            T ax, bx, ay, by;
            bw_coefs<T>(a, in.bw_off, i, ax, bx, ay, by);
            const uint32_t *rows = py ? rowm : rowp;
            T xa[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const T f0 = (T)C::dec(load(i, rows[k] + colx));
                T f1, f2;
                if constexpr (QUAD) {
                    f1 = px ? quad_move<kQuadXm1>(f0) : quad_move<kQuadXp1>(f0);
                    f2 = quad_move<kQuadX2>(f0);
                } else {
                    f1 = (T)C::dec(load(i, rows[k] + (uint32_t)imod(px ? x - 1 : x + 1, nx) * E));
                    f2 = (T)C::dec(load(i, rows[k] + (uint32_t)imod(px ? x - 2 : x + 2, nx) * E));
                }
                xa[k] = f0 - ax * (f0 - f1) + bx * (f1 - f2);
            }
            v[i] = xa[0] - ay * (xa[0] - xa[1]) + by * (xa[1] - xa[2]);
        });
    }
    collide<L, N, S, T>(v, (T)in.omega);
    const uint32_t cb = cell * E;
    static_for<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        *reinterpret_cast<raw *>(dst + (size_t)i * psb + cb) = C::template enc<false>(v[i], 0u);
    });
}

// Workgroup sum over cells [start, start + count) of u_x sin(2 pi y / ny), FP64, fixed order.
// Every thread of the block must call it; the result is valid in thread 0.
template <class L, int S, int BLOCK>
__device__ double partial_amp(const BatchInst &in, const BatchArgs &a, int cur, uint32_t start, uint32_t count,
                              double *red) {
    using C = Codec<S>;
    const auto *f = inst_buffer<L, S>(in, a, cur);
    const size_t ps = in.pstride;
    const double *sin_tab = a.sin_tab + in.sin_off;
    double acc = 0.0;
    for (uint32_t t = threadIdx.x; t < count; t += BLOCK) {
        const uint32_t cell = start + t;
        double dsum = 0.0, jx = 0.0;
        static_for<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr double mf = moment_factor<L, S, i>();
            const double g = mf * C::dec64(f[(size_t)i * ps + cell]);
            dsum += g;
            if constexpr (L::xi[i][0] != 0.0) jx += L::xi[i][0] * g;
        });
        const double rho = C::dev ? 1.0 + dsum : dsum;
        acc += (jx / rho) * sin_tab[cell / (uint32_t)in.nx];
    }
    const double s = wave_sum(acc);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < BLOCK / 64; ++w) t += red[w];
    return t;
}

// Kind of an instance: 4 * set + (N - 1), set 0 = D2Q9, 1 = D2Q37, 2 = D2Q16-GH, 3 = D2Q36-GH;
// Beam-Warming kinds with nx = 4 add 16 (quad-rotation path).
__host__ __device__ inline int batch_kind(int lattice, int order, int nx) {
    const int set = lattice == D2Q9::id ? 0 : lattice == D2Q37::id ? 1 : lattice == D2Q16_GH::id ? 2 : 3;
    return 4 * set + (order - 1) + ((set >= 2 && nx == 4) ? 16 : 0);
}

#define LBM_BATCH_KINDS(X)                                                                           \
    X(0, D2Q9, 1, false, false) X(1, D2Q9, 2, false, false) X(2, D2Q9, 3, false, false)              \
    X(3, D2Q9, 4, false, false) X(4, D2Q37, 1, false, false) X(5, D2Q37, 2, false, false)            \
    X(6, D2Q37, 3, false, false) X(7, D2Q37, 4, false, false) X(8, D2Q16_GH, 1, true, false)         \
    X(9, D2Q16_GH, 2, true, false) X(10, D2Q16_GH, 3, true, false) X(11, D2Q16_GH, 4, true, false)   \
    X(12, D2Q36_GH, 1, true, false) X(13, D2Q36_GH, 2, true, false) X(14, D2Q36_GH, 3, true, false)  \
    X(15, D2Q36_GH, 4, true, false) X(24, D2Q16_GH, 1, true, true) X(25, D2Q16_GH, 2, true, true)    \
    X(26, D2Q16_GH, 3, true, true) X(27, D2Q16_GH, 4, true, true) X(28, D2Q36_GH, 1, true, true)     \
    X(29, D2Q36_GH, 2, true, true) X(30, D2Q36_GH, 3, true, true) X(31, D2Q36_GH, 4, true, true)

template <int S>
__device__ __forceinline__ void step_chunk(const BatchInst &in, const BatchArgs &a, int cur, uint32_t start,
                                           uint32_t count) {
    switch (batch_kind(in.lattice, in.order, in.nx)) {
#define LBM_STEP_CASE(K, L, N, BW, QUAD) \
    case K: step_cells<L, N, S, BW, QUAD>(in, a, cur, start, count); break;
        LBM_BATCH_KINDS(LBM_STEP_CASE)
#undef LBM_STEP_CASE
        default: break;
    }
}

template <int S, int BLOCK>
__device__ __forceinline__ double amp_chunk(const BatchInst &in, const BatchArgs &a, int cur, uint32_t start,
                                            uint32_t count, double *red) {
    switch (in.lattice) {
        case D2Q9::id: return partial_amp<D2Q9, S, BLOCK>(in, a, cur, start, count, red);
        case D2Q37::id: return partial_amp<D2Q37, S, BLOCK>(in, a, cur, start, count, red);
        case D2Q16_GH::id: return partial_amp<D2Q16_GH, S, BLOCK>(in, a, cur, start, count, red);
        default: return partial_amp<D2Q36_GH, S, BLOCK>(in, a, cur, start, count, red);
    }
}

// ---------------------------------------------------------------- per-instance form
template <int S, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_batch(BatchArgs a) {
    __shared__ double red[BLOCK / 64];
    const int32_t idx = a.order[blockIdx.x];
    const BatchInst in = a.inst[idx];
    int cur = a.cur[idx];
    auto record = [&](int k) {
        const double s = amp_chunk<S, BLOCK>(in, a, cur, 0, in.ncell, red);
        if (threadIdx.x == 0) a.amp[in.amp_off + (size_t)k] = 2.0 * s / (double)in.ncell;
    };
    if (a.record_first) record(0);
    for (int64_t step = 0; step < a.steps; ++step) {
        for (uint32_t base = 0; base < in.ncell; base += BLOCK)
            step_chunk<S>(in, a, cur, base, min((uint32_t)BLOCK, in.ncell - base));
        __syncthreads();
        cur ^= 1;
        if (a.record > 0 && (step + 1) % a.record == 0) record((int)((step + 1) / a.record));
    }
}

// ---------------------------------------------------------------- grid form
// Device-wide barrier number `gen` (1, 2, ...).  The arrival count is 64-bit: gen * nwg stays
// exact for any step count.  Returns false if the run was aborted.
__device__ bool grid_barrier(const BatchArgs &a, uint64_t gen, int *flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();   // release this workgroup's stores to every CU
        __hip_atomic_fetch_add(a.barrier, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t target = gen * (uint64_t)a.nwg;
        uint32_t spins = 0;
        int ab = 0;
        while (__hip_atomic_load(a.barrier, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            ab = __hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ab) break;
            __builtin_amdgcn_s_sleep(2);
            if (++spins >= a.spin_limit) {
                __hip_atomic_store(a.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ab = 1;
                break;
            }
        }
        __threadfence();   // acquire: later loads see every workgroup's stores
        *flag = ab;
    }
    __syncthreads();
    return *flag == 0;
}

// XCD the calling wave runs on (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ uint32_t xcd_id() { return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15u; }

// Barrier number `gen` (1, 2, ...) of the workgroups on XCD x.  They share that XCD's L2: each
// wave waits until its stores have reached the L2, thread 0 counts the workgroup in and waits
// for the others, and then every wave invalidates its CU's L1 (buffer_inv at group scope, the
// invalidate the compiler itself issues for a workgroup acquire when a workgroup may span CUs)
// so that its later loads are served from the L2.  An agent-scope acquire would do as well but
// also invalidates the XCD's L2, which the other workgroups are still reading from.  Returns
// false if the run was aborted.
__device__ bool xcd_barrier(const BatchArgs &a, uint32_t x, uint64_t gen, int *flag) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);   // vmcnt(0): this wave's stores are acknowledged by the L2
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t *ctr = reinterpret_cast<uint64_t *>(a.sync + (kMaxXcd + x) * kSyncStride);   // 128-byte aligned
        __hip_atomic_fetch_add(ctr, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t target = gen * (uint64_t)a.wg_per_xcd;
        uint32_t spins = 0;
        int ab = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            ab = __hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ab) break;
            __builtin_amdgcn_s_sleep(1);
            if (++spins >= 2u * a.spin_limit) {   // half-length sleeps: twice the count
                __hip_atomic_store(a.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ab = 1;
                break;
            }
        }
        *flag = ab;
    }
    __syncthreads();
    asm volatile("buffer_inv sc0" ::: "memory");
    return *flag == 0;
}

// XCD: false for the device-wide form (plan entry = blockIdx.x), true for the XCD-local form.
// PROF: the step-profile instantiation (timestamps into a.ts); the plain one has none of that code.
template <int S, int BLOCK, bool XCD, bool PROF = false>
__global__ __launch_bounds__(BLOCK) void k_batch_grid(BatchArgs a) {
    __shared__ double red[BLOCK / 64];
    __shared__ int flag;
    __shared__ uint32_t place[2];   // XCD, plan entry
    if constexpr (XCD) {
        if (threadIdx.x == 0) {
            const uint32_t x = xcd_id();
            uint32_t p = ~0u;
            if (x < a.nxcd) {
                const uint32_t slot = __hip_atomic_fetch_add(a.sync + x * kSyncStride, 1u, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                if (slot < a.wg_per_xcd) p = x * a.wg_per_xcd + slot;
            }
            if (p == ~0u) __hip_atomic_store(a.abort, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            place[0] = x;
            place[1] = p;
        }
        // every workgroup has its slot; a placement that differs from the plan is seen by all
        if (!grid_barrier(a, 1, &flag)) return;
        if (threadIdx.x == 0) flag = __hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        if (flag) return;
    } else {
        if (threadIdx.x == 0) {
            place[0] = 0;
            place[1] = blockIdx.x;
        }
        __syncthreads();
    }
    // the same for every lane: read into scalar registers, so the descriptors below are loaded once
    // per wave by the scalar unit and the coefficients enter the arithmetic as scalar operands
    const uint32_t xcd = __builtin_amdgcn_readfirstlane(place[0]), entry = __builtin_amdgcn_readfirstlane(place[1]);
    const uint32_t c0 = a.wg_first[entry], c1 = a.wg_first[entry + 1];
    auto record = [&](int k, int64_t done) {
        for (uint32_t c = c0; c < c1; ++c) {
            const BatchChunk ch = a.chunks[a.wg_chunks[c]];
            const BatchInst in = a.inst[ch.inst];
            const int cur = a.cur[ch.inst] ^ (int)(done & 1);
            const double s = amp_chunk<S, BLOCK>(in, a, cur, ch.start, ch.count, red);
            if (threadIdx.x == 0) a.partials[(size_t)a.wg_chunks[c] * a.nrec + k] = s;
        }
    };
    if (a.record_first) record(0, 0);
    uint64_t gen = 0;
    for (int64_t step = 0; step < a.steps; ++step) {
        // step profile: thread 0 stores each timestamp as it is taken (nothing held across the step)
        const bool prof = PROF && step >= a.ts_first && step < a.ts_first + a.ts_count;
        auto stamp = [&](int j) {
            a.ts[((size_t)entry * (size_t)a.ts_count + (size_t)(step - a.ts_first)) * 3 + j] =
                __builtin_amdgcn_s_memrealtime();
        };
        if (prof && threadIdx.x == 0) stamp(0);
        for (uint32_t c = c0; c < c1; ++c) {
            const BatchChunk ch = a.chunks[a.wg_chunks[c]];
            const BatchInst in = a.inst[ch.inst];
            step_chunk<S>(in, a, a.cur[ch.inst] ^ (int)(step & 1), ch.start, ch.count);
        }
        if (prof) {
            __syncthreads();
            if (threadIdx.x == 0) stamp(1);
        }
        if constexpr (XCD) {
            if (!xcd_barrier(a, xcd, ++gen, &flag)) return;
        } else {
            if (!grid_barrier(a, ++gen, &flag)) return;
        }
        if (prof && threadIdx.x == 0) stamp(2);
        if (a.record > 0 && (step + 1) % a.record == 0) record((int)((step + 1) / a.record), step + 1);
    }
}

// amp[i][k] = 2 / ncell_i * sum over the chunks of instance i (in order) of partials[c][k].
__global__ __launch_bounds__(256) void k_batch_amp(BatchArgs a, uint32_t count) {
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (uint64_t)count * a.nrec) return;
    const uint32_t i = (uint32_t)(t / a.nrec), k = (uint32_t)(t % a.nrec);
    double s = 0.0;
    for (uint32_t c = a.inst_first[i]; c < a.inst_first[i + 1]; ++c) s += a.partials[(size_t)c * a.nrec + k];
    a.amp[a.inst[i].amp_off + k] = 2.0 * s / (double)a.inst[i].ncell;
}

__global__ __launch_bounds__(256) void k_batch_reset(BatchArgs a) {
    if (threadIdx.x == 0) {
        *a.barrier = 0ull;
        *a.abort = 0;
    }
    if (a.sync)
        for (uint32_t i = threadIdx.x; i < kSyncWords; i += 256) a.sync[i] = 0u;
}

__global__ __launch_bounds__(64) void k_probe_xcd(uint32_t *out) {
    if (threadIdx.x == 0) out[blockIdx.x] = xcd_id();
}

hipError_t probe_xcd(uint32_t *out, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_probe_xcd, dim3(n), dim3(64), 0, s, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- host launchers
template <int S, int BLOCK>
hipError_t launch_t(int form, const BatchArgs &a, uint32_t count, hipStream_t s) {
    if (form == 0) {
        hipLaunchKernelGGL((k_batch<S, BLOCK>), dim3(count), dim3(BLOCK), 0, s, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.ts) {
        // the profile instantiation must fit as many workgroups per CU as the plan assumed
        int n0 = 0, n1 = 0;
        const void *k0 = form == 2 ? (const void *)k_batch_grid<S, BLOCK, true> : (const void *)k_batch_grid<S, BLOCK, false>;
        const void *k1 = form == 2 ? (const void *)k_batch_grid<S, BLOCK, true, true>
                                   : (const void *)k_batch_grid<S, BLOCK, false, true>;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n0, k0, BLOCK, 0)) != hipSuccess) return e;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n1, k1, BLOCK, 0)) != hipSuccess) return e;
        if (n1 < n0) return hipErrorLaunchOutOfResources;
        if (form == 2)
            hipLaunchKernelGGL((k_batch_grid<S, BLOCK, true, true>), dim3(a.nwg), dim3(BLOCK), 0, s, a);
        else
            hipLaunchKernelGGL((k_batch_grid<S, BLOCK, false, true>), dim3(a.nwg), dim3(BLOCK), 0, s, a);
    } else if (form == 2) {
        hipLaunchKernelGGL((k_batch_grid<S, BLOCK, true>), dim3(a.nwg), dim3(BLOCK), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_batch_grid<S, BLOCK, false>), dim3(a.nwg), dim3(BLOCK), 0, s, a);
    }
    e = hipGetLastError();
    if (e != hipSuccess || (a.record <= 0 && !a.record_first)) return e;
    const uint64_t n = (uint64_t)count * a.nrec;
    hipLaunchKernelGGL(k_batch_amp, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, a, count);
    return hipGetLastError();
}

template <int S>
hipError_t launch_s(int form, int block, const BatchArgs &a, uint32_t count, hipStream_t s) {
    if (block == 256) return launch_t<S, 256>(form, a, count, s);
    if (block == 512) return launch_t<S, 512>(form, a, count, s);
    if (block == 1024) return launch_t<S, 1024>(form, a, count, s);
    return hipErrorInvalidValue;
}

hipError_t launch_batch(int storage, int form, int block, const BatchArgs &a, uint32_t count, hipStream_t s) {
    if (storage == ST_FP32_DEV) return launch_s<ST_FP32_DEV>(form, block, a, count, s);
    if (storage == ST_FP64) return launch_s<ST_FP64>(form, block, a, count, s);
    return hipErrorInvalidValue;
}

template <int S, int BLOCK, bool XCD>
int resident_t() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_grid<S, BLOCK, XCD>, BLOCK, 0) != hipSuccess) return 0;
    return n;
}

template <int S, bool XCD>
int resident_b(int block) {
    return block == 256 ? resident_t<S, 256, XCD>() : block == 512 ? resident_t<S, 512, XCD>() : resident_t<S, 1024, XCD>();
}

int batch_grid_resident_per_cu(int storage, int form, int block) {
    if (storage == ST_FP32_DEV) return form == 2 ? resident_b<ST_FP32_DEV, true>(block) : resident_b<ST_FP32_DEV, false>(block);
    return form == 2 ? resident_b<ST_FP64, true>(block) : resident_b<ST_FP64, false>(block);
}

bool batch_supports(int lattice, int order, int storage) {
    const bool lat = lattice == D2Q9::id || lattice == D2Q37::id || lattice == D2Q16_GH::id || lattice == D2Q36_GH::id;
    return lat && order >= 1 && order <= 4 && (storage == ST_FP32_DEV || storage == ST_FP64);
}

}  // namespace lbm
