// batch.hip -- many independent shear-wave instances advanced in one persistent launch.
//
// Each workgroup owns one instance (2-D velocity set, nx x ny periodic grid, its own tau and
// Hermite order) for the whole run: it loops over the steps on the device, pulling from one
// of the instance's two buffers and writing the other, with a workgroup barrier between
// steps.  An instance never spans two workgroups, so no synchronisation leaves the CU.  Every
// `record` steps the workgroup reduces the sine projection of u_x over its cells in FP64 and
// stores it in the amplitude log.  Instances are handed to workgroups largest first.
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

// QUAD: nx == 4, x-neighbours by quad rotation; otherwise by loads.
template <class L, int N, int S, bool BW, bool QUAD, int BLOCK>
__device__ __forceinline__ void run_instance(const BatchInst &in, const BatchArgs &a, double *red) {
    using C = Codec<S>;
    using raw = typename C::raw;
    using T = typename C::T;
    const int nx = in.nx, ny = in.ny;
    const uint32_t ncell = in.ncell;
    const size_t ps = in.pstride;
    raw *buf[2] = {static_cast<raw *>(a.pool) + in.off, static_cast<raw *>(a.pool) + in.off + (size_t)L::Q * ps};
    const int32_t idx = a.order[blockIdx.x];
    int cur = a.cur[idx];
    const T om = (T)in.omega;
    const double *sin_tab = a.sin_tab + in.sin_off;
    const int tid = threadIdx.x;

    auto record = [&](int k) {
        const raw *f = buf[cur];
        double acc = 0.0;
        for (uint32_t cell = tid; cell < ncell; cell += BLOCK) {
            double dsum = 0.0, jx = 0.0;
            static_for<L::Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr double mf = moment_factor<L, S, i>();
                const double g = mf * C::dec64(f[(size_t)i * ps + cell]);
                dsum += g;
                if constexpr (L::xi[i][0] != 0.0) jx += L::xi[i][0] * g;
            });
            const double rho = C::dev ? 1.0 + dsum : dsum;
            acc += (jx / rho) * sin_tab[cell / (uint32_t)nx];
        }
        const double s = wave_sum(acc);
        if ((tid & 63) == 0) red[tid >> 6] = s;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < BLOCK / 64; ++w) t += red[w];
            a.amp[in.amp_off + (size_t)k] = 2.0 * t / (double)ncell;
        }
        __syncthreads();
    };

    if (a.record_first) record(0);
    for (int64_t step = 0; step < a.steps; ++step) {
        const raw *__restrict__ src = buf[cur];
        raw *__restrict__ dst = buf[cur ^ 1];
        for (uint32_t base = 0; base < ncell; base += BLOCK) {
            const uint32_t cell = base + (uint32_t)tid;
            // nx = 4 and BLOCK % 4 == 0: quads are whole rows, active or inactive together
            if (cell >= ncell) continue;
            const int x = (int)(cell % (uint32_t)nx), y = (int)(cell / (uint32_t)nx);
            T v[L::Q];
            if constexpr (!BW) {
                static_for<L::Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    const int xs = imod(x - L::c[i][0], nx), ys = imod(y - L::c[i][1], ny);
                    v[i] = C::dec(src[(size_t)i * ps + (size_t)ys * nx + xs]);
                });
            } else {
                static_for<L::Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    constexpr bool px = L::xi[i][0] > 0.0, py = L::xi[i][1] > 0.0;
                    const T ax = (T)a.bw[in.bw_off + 0 * kMaxQ + i], bx = (T)a.bw[in.bw_off + 1 * kMaxQ + i];
                    const T ay = (T)a.bw[in.bw_off + 2 * kMaxQ + i], by = (T)a.bw[in.bw_off + 3 * kMaxQ + i];
                    const int r0 = y, r1 = imod(py ? y - 1 : y + 1, ny), r2 = imod(py ? y - 2 : y + 2, ny);
                    const raw *p = src + (size_t)i * ps;
                    T xa[3];
                    const int rows[3] = {r0, r1, r2};
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const raw *pr = p + (size_t)rows[k] * nx;
                        const T f0 = (T)C::dec(pr[x]);
                        T f1, f2;
                        if constexpr (QUAD) {
                            f1 = px ? quad_move<kQuadXm1>(f0) : quad_move<kQuadXp1>(f0);
                            f2 = quad_move<kQuadX2>(f0);
                        } else {
                            f1 = (T)C::dec(pr[imod(px ? x - 1 : x + 1, nx)]);
                            f2 = (T)C::dec(pr[imod(px ? x - 2 : x + 2, nx)]);
                        }
                        xa[k] = f0 - ax * (f0 - f1) + bx * (f1 - f2);
                    }
                    v[i] = xa[0] - ay * (xa[0] - xa[1]) + by * (xa[1] - xa[2]);
                });
            }
            collide<L, N, S, T>(v, om);
            static_for<L::Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                dst[(size_t)i * ps + cell] = C::template enc<false>(v[i], 0u);
            });
        }
        __syncthreads();
        cur ^= 1;
        if (a.record > 0 && (step + 1) % a.record == 0) record((int)((step + 1) / a.record));
    }
    if (tid == 0) a.cur[idx] = cur;
}

// Kind of an instance: 4 * set + (N - 1), set 0 = D2Q9, 1 = D2Q37, 2 = D2Q16-GH, 3 = D2Q36-GH;
// Beam-Warming kinds with nx = 4 add 16 (quad-rotation path).
__host__ __device__ inline int batch_kind(int lattice, int order, int nx) {
    const int set = lattice == D2Q9::id ? 0 : lattice == D2Q37::id ? 1 : lattice == D2Q16_GH::id ? 2 : 3;
    return 4 * set + (order - 1) + ((set >= 2 && nx == 4) ? 16 : 0);
}

template <int S, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_batch(BatchArgs a) {
    __shared__ double red[BLOCK / 64];
    const BatchInst in = a.inst[a.order[blockIdx.x]];
    switch (batch_kind(in.lattice, in.order, in.nx)) {
#define LBM_CASE(K, L, N, BW, QUAD) \
    case K: run_instance<L, N, S, BW, QUAD, BLOCK>(in, a, red); break;
        LBM_CASE(0, D2Q9, 1, false, false)
        LBM_CASE(1, D2Q9, 2, false, false)
        LBM_CASE(2, D2Q9, 3, false, false)
        LBM_CASE(3, D2Q9, 4, false, false)
        LBM_CASE(4, D2Q37, 1, false, false)
        LBM_CASE(5, D2Q37, 2, false, false)
        LBM_CASE(6, D2Q37, 3, false, false)
        LBM_CASE(7, D2Q37, 4, false, false)
        LBM_CASE(8, D2Q16_GH, 1, true, false)
        LBM_CASE(9, D2Q16_GH, 2, true, false)
        LBM_CASE(10, D2Q16_GH, 3, true, false)
        LBM_CASE(11, D2Q16_GH, 4, true, false)
        LBM_CASE(12, D2Q36_GH, 1, true, false)
        LBM_CASE(13, D2Q36_GH, 2, true, false)
        LBM_CASE(14, D2Q36_GH, 3, true, false)
        LBM_CASE(15, D2Q36_GH, 4, true, false)
        LBM_CASE(24, D2Q16_GH, 1, true, true)
        LBM_CASE(25, D2Q16_GH, 2, true, true)
        LBM_CASE(26, D2Q16_GH, 3, true, true)
        LBM_CASE(27, D2Q16_GH, 4, true, true)
        LBM_CASE(28, D2Q36_GH, 1, true, true)
        LBM_CASE(29, D2Q36_GH, 2, true, true)
        LBM_CASE(30, D2Q36_GH, 3, true, true)
        LBM_CASE(31, D2Q36_GH, 4, true, true)
#undef LBM_CASE
        default: break;
    }
}

template <int S, int BLOCK>
hipError_t launch_batch_t(const BatchArgs &a, uint32_t count, hipStream_t s) {
    hipLaunchKernelGGL((k_batch<S, BLOCK>), dim3(count), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_batch(int storage, int block, const BatchArgs &a, uint32_t count, hipStream_t s) {
    if (storage == ST_FP32_DEV) {
        if (block == 256) return launch_batch_t<ST_FP32_DEV, 256>(a, count, s);
        if (block == 512) return launch_batch_t<ST_FP32_DEV, 512>(a, count, s);
        if (block == 1024) return launch_batch_t<ST_FP32_DEV, 1024>(a, count, s);
    } else if (storage == ST_FP64) {
        if (block == 256) return launch_batch_t<ST_FP64, 256>(a, count, s);
        if (block == 512) return launch_batch_t<ST_FP64, 512>(a, count, s);
        if (block == 1024) return launch_batch_t<ST_FP64, 1024>(a, count, s);
    }
    return hipErrorInvalidValue;
}

bool batch_supports(int lattice, int order, int storage) {
    const bool lat = lattice == D2Q9::id || lattice == D2Q37::id || lattice == D2Q16_GH::id || lattice == D2Q36_GH::id;
    return lat && order >= 1 && order <= 4 && (storage == ST_FP32_DEV || storage == ST_FP64);
}

}  // namespace lbm
