// kernels_impl.h -- kernel templates, included by the per-lattice units only.
#pragma once

#include <math.h>

#include "bgk_device.h"
#include "kernels.h"

namespace lbm {

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD b mod 8).  When
// the grid divides evenly, give each XCD a contiguous range of logical tiles so that the
// tiles sharing halo cache lines meet in the same L2.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t bid, uint32_t nblocks) {
    return (nblocks & 7u) == 0u ? (bid & 7u) * (nblocks >> 3) + (bid >> 3) : bid;
}

// Stochastic-rounding bits.  A conversion reads a window of at most 16 of its 32 random bits
// (the low 16 bits: the 16 bits BF16 drops from FP32, the 13 FP16 drops).  Each cell hashes its
// index with the step's key twice (h1, h2: two multiply-xorshift finalisers, the only
// quarter-rate work); population pair k takes the word w_k = rotl(h1, r1_k) ^ rotl(h2, r2_k),
// population 2k its low half and 2k + 1 its high half (w_k rotated by 16).  The rotation pairs
// below were chosen so that, for (h1, h2) uniform, the 16-bit windows of any two of the first 39
// populations are jointly uniform (the 32 x 64 bit matrix mapping (h1, h2) to the two windows
// has full rank over GF(2)): every population's rounding is unbiased and any two populations
// of a cell round independently, at three full-rate operations per pair instead of one hash.
// A CPU test re-derives the rank condition from this table.
struct CellBits {
    uint32_t h1, h2;
};
constexpr int kSrRot[20][2] = {{24, 22}, {26, 14}, {21, 1}, {17, 10}, {20, 6}, {13, 17}, {18, 7},
                               {4, 30},  {30, 5},  {22, 4}, {26, 9},  {1, 18}, {27, 26}, {7, 2},
                               {2, 24},  {21, 17}, {15, 2}, {19, 0},  {4, 6},  {2, 12}};
__device__ __forceinline__ CellBits cell_bits(uint32_t cell, uint32_t key) {
    return CellBits{mix32(cell ^ key), mix32((cell ^ key) + 0x9e3779b9u)};
}
template <int A>
__device__ __forceinline__ uint32_t pop_bits(const CellBits &c) {
    static_assert(A < 40, "rotation table covers 40 populations");
    constexpr int k = A >> 1;
    const uint32_t w = __builtin_rotateleft32(c.h1, kSrRot[k][0]) ^ __builtin_rotateleft32(c.h2, kSrRot[k][1]);
    return (A & 1) ? __builtin_rotateleft32(w, 16) : w;
}
__device__ __forceinline__ uint32_t pop_bits_rt(const CellBits &c, int a) {   // runtime population index
    const int k = a >> 1;
    uint32_t r1 = 0, r2 = 0;
#pragma unroll
    for (int j = 0; j < 20; ++j)
        if (j == k) {
            r1 = (uint32_t)kSrRot[j][0];
            r2 = (uint32_t)kSrRot[j][1];
        }
    const uint32_t w = __builtin_rotateleft32(c.h1, r1) ^ __builtin_rotateleft32(c.h2, r2);
    return (a & 1) ? __builtin_rotateleft32(w, 16) : w;
}

__device__ __forceinline__ int wrap_once(int v, int n) {   // |v| < 2n
    v += (v < 0) ? n : 0;
    v -= (v >= n) ? n : 0;
    return v;
}
__device__ __forceinline__ int imod(int v, int n) {
    int r = v % n;
    return r < 0 ? r + n : r;
}

// Sum over the 64 lanes of a wave in a fixed butterfly order (every lane gets the sum).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Forced steps: lane 0 of each wave stores the wave's sums of stress x sin and stress x cos
// in slot blockIdx.x * (BLOCK / 64) + wave; the slots are added in index order afterwards.
template <int BLOCK>
__device__ __forceinline__ void store_stress(double *out, double ss, double sc) {
    ss = wave_sum(ss);
    sc = wave_sum(sc);
    if ((threadIdx.x & 63) == 0) {
        const size_t slot = (size_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
        out[2 * slot] = ss;
        out[2 * slot + 1] = sc;
    }
}

// Cross-lane moves of one wave (DPP row/wave shifts, gfx9 family):
//   shr: lane l takes lane l-1's value, lane 0 takes `old`;
//   shl: lane l takes lane l+1's value, lane 63 takes `old`.
__device__ __forceinline__ int dpp_shr_i(int old, int v) { return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_shl_i(int old, int v) { return __builtin_amdgcn_update_dpp(old, v, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ float dpp_shr(float old, float v) {
    return __builtin_bit_cast(float, dpp_shr_i(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float dpp_shl(float old, float v) {
    return __builtin_bit_cast(float, dpp_shl_i(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v)));
}
typedef int int2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double dpp_shr(double old, double v) {
    const int2v o = __builtin_bit_cast(int2v, old), x = __builtin_bit_cast(int2v, v);
    return __builtin_bit_cast(double, int2v{dpp_shr_i(o.x, x.x), dpp_shr_i(o.y, x.y)});
}
__device__ __forceinline__ double dpp_shl(double old, double v) {
    const int2v o = __builtin_bit_cast(int2v, old), x = __builtin_bit_cast(int2v, v);
    return __builtin_bit_cast(double, int2v{dpp_shl_i(o.x, x.x), dpp_shl_i(o.y, x.y)});
}

// ---------------------------------------------------------------- exact shift, row tiles
// Block = `tile` chunks of BLOCK consecutive cells of one row (y, z).  Thread pulls
// f*_a(x - c_a) for every a, collides, and writes f*(x) to the other buffer.  Loads of one
// population by one wave cover 64 consecutive cells (256 B in FP32); stores are aligned and,
// with NTS, non-temporal: the output is not read again in this step, and streaming it past
// the L2 leaves room for the cache lines that neighbouring chunks share through the x-shifts.
// With F the collision adds the body force of the row and the stress sums are stored.
template <class L, int N, int S, bool SR, int BLOCK, bool NTS, bool F>
__global__ __launch_bounds__(BLOCK) void k_shift_rows(StepArgs a) {
    using C = Codec<S>;
    using raw = typename C::raw;
    using T = typename C::T;
    const uint32_t lb = xcd_tile(blockIdx.x, a.nblocks);
    const uint32_t row = lb / a.per_row;
    const uint32_t xb = lb - row * a.per_row;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int y = (int)(row % (uint32_t)ny), z = (int)(row / (uint32_t)ny);
    // Addresses: a 64-bit scalar base per source row (one per distinct (c_y, c_z), shared by the
    // populations moving along it) plus a 32-bit lane offset, population * (bytes between
    // populations) + x-offset, which the load and store instructions add themselves.  A row of all
    // Q populations is below 2^31 bytes (checked by the host), so the offset cannot wrap.
    const char *__restrict__ fin = static_cast<const char *>(a.fin);
    char *__restrict__ fout = static_cast<char *>(a.fout);
    const uint32_t ps = (uint32_t)a.lay.pop * (uint32_t)sizeof(raw);
    const size_t rs = (size_t)a.lay.row * sizeof(raw);
    const T om = (T)a.omega;
    const int jf = a.force_axis == 1 ? y : z;           // row index along the force axis
    T Gx = T(0);
    if constexpr (F) Gx = (T)(a.force_g * a.force_cos[jf]);
    double sig_sum = 0.0;
    for (uint32_t k = 0; k < a.tile; ++k) {
        int x = (int)((xb * a.tile + k) * BLOCK + threadIdx.x);
        if (x >= nx) break;
        // 16-bit storages: the column is opaque to the optimiser, so the per-population load
        // offsets are formed inside the loop from it (one add each, as they are anyway) instead
        // of being hoisted as 64-bit addresses that hold registers through the collision.  The
        // empty statement emits no instruction.
        if constexpr (C::lowp) asm volatile("" : "+v"(x));
        raw rv[L::Q];
        static_for<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
            int ys = y - cy, zs = z - cz;
            if constexpr (cy > 0) ys += (ys < 0) ? ny : 0;
            if constexpr (cy < 0) ys -= (ys >= ny) ? ny : 0;
            if constexpr (cz > 0) zs += (zs < 0) ? nz : 0;
            if constexpr (cz < 0) zs -= (zs >= nz) ? nz : 0;
            int xs = x - cx;
            if constexpr (cx > 0) xs += (xs < 0) ? nx : 0;
            if constexpr (cx < 0) xs -= (xs >= nx) ? nx : 0;
            const char *rb = fin + (size_t)(ys + ny * zs) * rs;
            const uint32_t off = (uint32_t)i * ps + (uint32_t)xs * (uint32_t)sizeof(raw);
            rv[i] = *reinterpret_cast<const raw *>(rb + off);
        });
        // all Q loads are issued before any is used: left to itself the scheduler may, under
        // register pressure, wait for each load before issuing the next
        __builtin_amdgcn_sched_barrier(0);
        T v[L::Q];
        static_for<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            v[i] = C::dec(rv[i]);
            // FP16: keep only the decoded FP32 value live.  Otherwise the compiler folds the
            // conversion into mixed-precision FMAs that read the half value, and both forms of
            // every population stay in registers through the collision (159 registers, 3 waves
            // per SIMD, against 126 for BF16; the forced kernels keep the folding, which suits
            // their register allocation better).  The empty statement emits no instruction.
            if constexpr (S == ST_FP16_DEV && !F) asm volatile("" : "+v"(v[i]));
        });
        if constexpr (F) {
            T sig[2];
            collide_impl<L, N, S, T, true>(v, om, Gx, sig);
            sig_sum += (double)(a.force_axis == 1 ? sig[0] : sig[1]);
        } else {
            collide<L, N, S, T>(v, om);
        }
        const uint32_t cell = row * (uint32_t)nx + (uint32_t)x;
        char *ob = fout + (size_t)row * rs;
        const uint32_t xo = (uint32_t)x * (uint32_t)sizeof(raw);
        CellBits hb{0u, 0u};
        if constexpr (SR) hb = cell_bits(cell, a.sr_key);
        static_for<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const raw r = C::template enc<SR>(v[i], SR ? pop_bits<i>(hb) : 0u);
            raw *dst = reinterpret_cast<raw *>(ob + ((uint32_t)i * ps + xo));
            if constexpr (NTS)
                __builtin_nontemporal_store(r, dst);
            else
                *dst = r;
        });
    }
    if constexpr (F)
        if (a.stress) store_stress<BLOCK>(a.stress, sig_sum * a.force_sin[jf], sig_sum * a.force_cos[jf]);
}

// ---------------------------------------------------------------- exact shift, 4 cells per thread
// A wave owns 256 consecutive cells of a row, four per lane, loaded and stored as aligned
// 4-element vectors (so every global access of a wave is one 1 KiB segment in FP32).  The
// x-shift of population a by c_a (|c_a| <= 4) takes the missing elements from the neighbouring
// lane by DPP lane moves; the lane at the wave's edge takes them from one 4-element load of the
// neighbouring wave's cells, which every lane issues at the same address.  Needs nx a multiple
// of 256 and rows aligned to 4 elements.  With NTL the loads are non-temporal.
template <class L>
constexpr int max_cx() {
    int m = 0;
    for (int i = 0; i < L::Q; ++i) m = L::c[i][0] > m ? L::c[i][0] : (-L::c[i][0] > m ? -L::c[i][0] : m);
    return m;
}

template <class L, int N, int S, bool SR, bool NTL>
__global__ __launch_bounds__(kBlock) void k_shift_rows4(StepArgs a) {
    static_assert(max_cx<L>() <= 4, "x-shifts beyond one lane");
    using C = Codec<S>;
    using raw = typename C::raw;
    using T = typename C::T;
    typedef raw rv4 __attribute__((ext_vector_type(4)));
    const uint32_t lb = xcd_tile(blockIdx.x, a.nblocks);
    const uint32_t row = lb / a.per_row;
    const uint32_t xb = lb - row * a.per_row;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int y = (int)(row % (uint32_t)ny), z = (int)(row / (uint32_t)ny);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const raw *__restrict__ fin = static_cast<const raw *>(a.fin);
    raw *__restrict__ fout = static_cast<raw *>(a.fout);
    const size_t ps = a.lay.pop, rs = a.lay.row;
    const T om = (T)a.omega;
    for (uint32_t k = 0; k < a.tile; ++k) {
        const int xw = (int)(((xb * a.tile + k) * (kBlock / 64) + wv) * 256);   // the wave's first cell
        if (xw >= nx) break;                                                     // whole wave
        const int x0 = xw + 4 * lane;
        T v[4][L::Q];
        static_for<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
            int ys = y - cy, zs = z - cz;
            if constexpr (cy > 0) ys += (ys < 0) ? ny : 0;
            if constexpr (cy < 0) ys -= (ys >= ny) ? ny : 0;
            if constexpr (cz > 0) zs += (zs < 0) ? nz : 0;
            if constexpr (cz < 0) zs -= (zs >= nz) ? nz : 0;
            const raw *p = fin + (size_t)i * ps + (size_t)(ys + ny * zs) * rs;
            rv4 ar;
            if constexpr (NTL)
                ar = __builtin_nontemporal_load(reinterpret_cast<const rv4 *>(p + x0));
            else
                ar = *reinterpret_cast<const rv4 *>(p + x0);
            const T A[4] = {C::dec(ar.x), C::dec(ar.y), C::dec(ar.z), C::dec(ar.w)};
            if constexpr (cx == 0) {
#pragma unroll
                for (int m = 0; m < 4; ++m) v[m][i] = A[m];
            } else if constexpr (cx > 0) {              // element m comes from cell x0 + m - cx
                int hx = xw - 4;
                hx += hx < 0 ? nx : 0;
                const rv4 hr = *reinterpret_cast<const rv4 *>(p + hx);
                const T H[4] = {C::dec(hr.x), C::dec(hr.y), C::dec(hr.z), C::dec(hr.w)};
                T left[4];
#pragma unroll
                for (int m = 4 - cx; m < 4; ++m) left[m] = dpp_shr(H[m], A[m]);
#pragma unroll
                for (int m = 0; m < 4; ++m) v[m][i] = (m >= cx) ? A[m >= cx ? m - cx : 0] : left[m < cx ? 4 + m - cx : 0];
            } else {
                constexpr int c = -cx;
                int hx = xw + 256;
                hx -= hx >= nx ? nx : 0;
                const rv4 hr = *reinterpret_cast<const rv4 *>(p + hx);
                const T H[4] = {C::dec(hr.x), C::dec(hr.y), C::dec(hr.z), C::dec(hr.w)};
                T right[4];
#pragma unroll
                for (int m = 0; m < c; ++m) right[m] = dpp_shl(H[m], A[m]);
#pragma unroll
                for (int m = 0; m < 4; ++m) v[m][i] = (m + c <= 3) ? A[m + c <= 3 ? m + c : 0] : right[m + c > 3 ? m + c - 4 : 0];
            }
        });
#pragma unroll
        for (int m = 0; m < 4; ++m) collide<L, N, S, T>(v[m], om);
        const uint32_t cell = row * (uint32_t)nx + (uint32_t)x0;
        const size_t o = (size_t)row * rs + (size_t)x0;
        CellBits h[4] = {};
        if constexpr (SR) {
#pragma unroll
            for (int m = 0; m < 4; ++m) h[m] = cell_bits(cell + (uint32_t)m, a.sr_key);
        }
        static_for<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            rv4 r;
            r.x = C::template enc<SR>(v[0][i], SR ? pop_bits<i>(h[0]) : 0u);
            r.y = C::template enc<SR>(v[1][i], SR ? pop_bits<i>(h[1]) : 0u);
            r.z = C::template enc<SR>(v[2][i], SR ? pop_bits<i>(h[2]) : 0u);
            r.w = C::template enc<SR>(v[3][i], SR ? pop_bits<i>(h[3]) : 0u);
            __builtin_nontemporal_store(r, reinterpret_cast<rv4 *>(fout + (size_t)i * ps + o));
        });
    }
}

// ---------------------------------------------------------------- exact shift, any grid
template <class L, int N, int S, bool SR, bool F>
__global__ __launch_bounds__(kBlock) void k_shift_cells(StepArgs a) {
    using C = Codec<S>;
    using raw = typename C::raw;
    using T = typename C::T;
    const uint32_t ncell = (uint32_t)a.nx * (uint32_t)a.ny * (uint32_t)a.nz;
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    double ss = 0.0, sc = 0.0;
    if (cell < ncell) {
        const int nx = a.nx, ny = a.ny, nz = a.nz;
        const int x = (int)(cell % (uint32_t)nx);
        const uint32_t t = cell / (uint32_t)nx;
        const int y = (int)(t % (uint32_t)ny), z = (int)(t / (uint32_t)ny);
        const raw *__restrict__ fin = static_cast<const raw *>(a.fin);
        raw *__restrict__ fout = static_cast<raw *>(a.fout);
        const size_t ps = a.lay.pop, rs = a.lay.row;
        T v[L::Q];
        static_for<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const int xs = imod(x - L::c[i][0], nx), ys = imod(y - L::c[i][1], ny), zs = imod(z - L::c[i][2], nz);
            v[i] = C::dec(fin[(size_t)i * ps + (size_t)xs + rs * ((size_t)ys + (size_t)ny * zs)]);
        });
        if constexpr (F) {
            const int jf = a.force_axis == 1 ? y : z;
            T sig[2];
            collide_impl<L, N, S, T, true>(v, (T)a.omega, (T)(a.force_g * a.force_cos[jf]), sig);
            const double sg = (double)(a.force_axis == 1 ? sig[0] : sig[1]);
            ss = sg * a.force_sin[jf];
            sc = sg * a.force_cos[jf];
        } else {
            collide<L, N, S, T>(v, (T)a.omega);
        }
        CellBits hb{0u, 0u};
        if constexpr (SR) hb = cell_bits(cell, a.sr_key);
        const size_t o = (size_t)t * rs + (size_t)x;
        static_for<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            fout[(size_t)i * ps + o] = C::template enc<SR>(v[i], SR ? pop_bits<i>(hb) : 0u);
        });
    }
    if constexpr (F)
        if (a.stress) store_stress<kBlock>(a.stress, ss, sc);
}

// ---------------------------------------------------------------- Beam-Warming, 2-D
// Thread = one column x walking a strip of `tile` rows; a wave owns 64 consecutive
// (aligned) columns.  For each population it keeps the x-advected values of two rows of its
// three-row upwind stencil in registers (sliding window over y) and loads one new row per
// step.  The x-neighbours x - s, x - 2s come from neighbouring lanes by DPP shifts; the two
// columns left (right) of the wave come from one extra load per population-row that touches a
// single cache line and enter the shift as the value of the vacated lane.  So every
// population-row costs one aligned load, one one-line halo load and three lane shifts; stores
// are whole aligned wave segments (non-temporal with NTS: the output is not read again in this
// step; with NTL the loads of the stencil's own column are non-temporal too, the halo columns'
// loads, which the neighbouring wave re-reads, not).  With ALT the odd strips walk up (decreasing y) and the even ones down, so two strips
// start and end at their shared edges at the same time and the rows there, which both read,
// meet in the L2 instead of being fetched twice; the window slides either way (for a population
// whose stencil points along the walk it holds rows y, y + d and loads y + 2d, otherwise it
// holds y - 2d, y - d and loads y).
// With F the collision adds the body force (force axis y) and the stress sums are stored.
// Raw buffer accesses: a 128-bit resource (base address, size in bytes) in scalar registers, a
// 32-bit lane offset and a 32-bit scalar offset, added by the memory unit.  Out-of-range
// loads return zero and out-of-range stores are dropped (the kernels never issue one).
constexpr int kBufWord3 = 0x00020000;   // gfx9 family: raw (untyped) 32-bit data format
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, kBufWord3);
}
template <class R, bool NT = false>
__device__ __forceinline__ R buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    constexpr int aux = NT ? 2 : 0;   // 2: non-temporal
    if constexpr (sizeof(R) == 2)
        return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, aux));
    else if constexpr (sizeof(R) == 4)
        return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, aux));
    else
        return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, aux));
}
template <bool NT, class R>
__device__ __forceinline__ void buf_store(R v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    constexpr int aux = NT ? 2 : 0;   // 2: non-temporal
    if constexpr (sizeof(R) == 2)
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, voff, soff, aux);
    else if constexpr (sizeof(R) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, aux);
    else
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v),
                                              r, voff, soff, aux);
}

// Beam-Warming coefficients depend on |xi_ad| only: population i reads those of the first
// population with the same |xi_ad|, so a kernel holds one (alpha, beta) per distinct magnitude
// (2 per axis for a 4-point Gauss-Hermite product, 3 for 6 points) instead of one per population.
template <class L>
constexpr int bw_slot(int i, int d) {
    for (int j = 0; j < L::Q; ++j)
        if (L::xi[j][d] == L::xi[i][d] || L::xi[j][d] == -L::xi[i][d]) return j;
    return i;
}

template <class L, int N, int S, bool SR, class T, bool F, bool NTS, bool ALT, bool NTL = false, bool PIPE = false>
__global__ __launch_bounds__(kBlock) void k_bw2(StepArgs a, BWCoef<T> cf) {
    static_assert(L::D == 2, "Beam-Warming kernel is two-dimensional");
    using C = Codec<S>;
    using raw = typename C::raw;
    const uint32_t lb = xcd_tile(blockIdx.x, a.nblocks);
    const uint32_t strip = lb / a.per_row;
    const uint32_t xb = lb - strip * a.per_row;
    const int nx = a.nx, ny = a.ny;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int x0 = (int)(xb * (kBlock / 64) + wv) * 64;
    if (x0 >= nx) {                                    // whole wave leaves together
        if constexpr (F)
            if (a.stress) store_stress<kBlock>(a.stress, 0.0, 0.0);
        return;
    }
    const int xo = x0 + lane;                          // this lane's column (may exceed nx)
    const int xl = xo % nx;                            // column it loads (wrapped)
    const int hl = (x0 - 1 - (lane == 1 ? 1 : 0) + 2 * nx) % nx;   // lane 0: x0-1, lane 1: x0-2
    const int hr = (x0 + 64 + (lane == 62 ? 1 : 0)) % nx;          // lane 63: x0+64, lane 62: x0+65
    const bool owner = xo < nx;
    const int y0 = (int)(strip * a.tile);
    const int y1 = min(y0 + (int)a.tile, ny);
    // addresses: a buffer resource per grid row (all Q populations of the row, below 2^31 bytes:
    // host check), the column's byte offset as the lane offset and population * bytes between
    // populations as the scalar offset, so no per-population address arithmetic runs on the VALU
    const char *__restrict__ fin = static_cast<const char *>(a.fin);
    char *__restrict__ fout = static_cast<char *>(a.fout);
    constexpr uint32_t es = (uint32_t)sizeof(raw);
    const uint32_t ps = (uint32_t)a.lay.pop * es, rowb = (uint32_t)a.lay.row * es;
    const uint32_t xlb = (uint32_t)xl * es, hlb = (uint32_t)hl * es, hrb = (uint32_t)hr * es, xob = (uint32_t)xo * es;
    auto row_of = [&](int r) { return (size_t)wrap_once(wrap_once(r, ny), ny) * rowb; };
    // x-advected value of population i from its column's raw value and its halo column's
    auto xadv_raw = [&](auto I, raw f0r, raw hr) -> T {
        constexpr int i = decltype(I)::value;
        constexpr int kx = bw_slot<L>(i, 0);
        const T f0 = (T)C::dec(f0r), h = (T)C::dec(hr);
        T f1, f2;
        if constexpr (L::xi[i][0] > 0.0) {            // upwind = left: f(x-1), f(x-2)
            f1 = dpp_shr(h, f0);
            f2 = dpp_shr(dpp_shl(h, h), f1);
        } else {                                      // upwind = right: f(x+1), f(x+2)
            f1 = dpp_shl(h, f0);
            f2 = dpp_shl(dpp_shr(h, h), f1);
        }
        return f0 - cf.alpha[0][kx] * (f0 - f1) + cf.beta[0][kx] * (f1 - f2);
    };
    constexpr auto halo_of = [](int i) { return L::xi[i][0] > 0.0; };   // true: the halo is on the left
    auto xadv = [&](auto I, size_t roff) -> T {
        constexpr int i = decltype(I)::value;
        const __amdgpu_buffer_rsrc_t rr = make_rsrc(fin + roff, rowb);
        const raw f0r = buf_load<raw, NTL>(rr, xlb, (uint32_t)i * ps);
        const raw hr = buf_load<raw>(rr, halo_of(i) ? hlb : hrb, (uint32_t)i * ps);
        return xadv_raw(I, f0r, hr);
    };
    const T om = (T)a.omega;
    double ss = 0.0, sc = 0.0;
    // walk the strip in direction D (+1: increasing y from y0, -1: decreasing y from y1 - 1)
    auto walk = [&](auto Dir) {
        constexpr int D = decltype(Dir)::value;
        const int ys = D > 0 ? y0 : y1 - 1;
        T A[L::Q], B[L::Q];
        static_for<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr bool along = (L::xi[i][1] < 0.0) == (D > 0);   // stencil rows y, y+D, y+2D
            if constexpr (along) {
                A[i] = xadv(I, row_of(ys));
                B[i] = xadv(I, row_of(ys + D));
            } else {                                                  // rows y-2D, y-D, y
                A[i] = xadv(I, row_of(ys - 2 * D));
                B[i] = xadv(I, row_of(ys - D));
            }
        });
        // y-advection of population i with the window (A, B) and the new row's x-advected value
        auto yadv = [&](auto I, T Cn) -> T {
            constexpr int i = decltype(I)::value;
            constexpr int ky = bw_slot<L>(i, 1);
            constexpr bool along = (L::xi[i][1] < 0.0) == (D > 0);
            T out;
            if constexpr (along)                   // A = row y, B = row y+D, new row y+2D
                out = A[i] - cf.alpha[1][ky] * (A[i] - B[i]) + cf.beta[1][ky] * (B[i] - Cn);
            else                                   // A = row y-2D, B = row y-D, new row y
                out = Cn - cf.alpha[1][ky] * (Cn - B[i]) + cf.beta[1][ky] * (B[i] - A[i]);
            A[i] = B[i];
            B[i] = Cn;
            return out;
        };
        // collision and store of row y
        auto finish = [&](int y, T (&v)[L::Q]) {
            const size_t r0 = row_of(y);
            if constexpr (F) {
                T sig[2];
                collide_impl<L, N, S, T, true>(v, om, (T)(a.force_g * a.force_cos[y]), sig);
                if (owner) {
                    ss += (double)sig[0] * a.force_sin[y];
                    sc += (double)sig[0] * a.force_cos[y];
                }
            } else {
                collide<L, N, S, T>(v, om);
            }
            if (owner) {
                const __amdgpu_buffer_rsrc_t wr = make_rsrc(fout + r0, rowb);
                CellBits hb{0u, 0u};
                if constexpr (SR) hb = cell_bits((uint32_t)(y * nx + xo), a.sr_key);
                static_for<L::Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    const raw r = C::template enc<SR>(v[i], SR ? pop_bits<i>(hb) : 0u);
                    buf_store<NTS>(r, wr, xob, (uint32_t)i * ps);
                });
            }
        };
        const int n = y1 - y0;
        if constexpr (!PIPE) {
            for (int k = 0; k < n; ++k) {
                const int y = ys + D * k;
                T v[L::Q];
                const size_t r0 = row_of(y), r2 = row_of(y + 2 * D);
                static_for<L::Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    constexpr bool along = (L::xi[i][1] < 0.0) == (D > 0);
                    v[i] = yadv(I, xadv(I, along ? r2 : r0));
                });
                finish(y, v);
            }
        } else {
            // software pipeline: the loads of row k + 1 are issued before row k is computed, so
            // a wave's next loads are in flight while it computes (one row of raw values more
            // in registers)
            raw fn[L::Q], hn[L::Q];
            auto prefetch = [&](int k) {
                const int y = ys + D * k;
                const size_t r0 = row_of(y), r2 = row_of(y + 2 * D);
                static_for<L::Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    constexpr bool along = (L::xi[i][1] < 0.0) == (D > 0);
                    const __amdgpu_buffer_rsrc_t rr = make_rsrc(fin + (along ? r2 : r0), rowb);
                    fn[i] = buf_load<raw, NTL>(rr, xlb, (uint32_t)i * ps);
                    hn[i] = buf_load<raw>(rr, halo_of(i) ? hlb : hrb, (uint32_t)i * ps);
                });
            };
            prefetch(0);
            for (int k = 0; k < n; ++k) {
                raw fc[L::Q], hc[L::Q];
                static_for<L::Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    fc[i] = fn[i];
                    hc[i] = hn[i];
                });
                if (k + 1 < n) prefetch(k + 1);
                __builtin_amdgcn_sched_barrier(0);
                T v[L::Q];
                static_for<L::Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    v[i] = yadv(I, xadv_raw(I, fc[i], hc[i]));
                });
                finish(ys + D * k, v);
            }
        }
    };
    if (ALT && (strip & 1u))
        walk(std::integral_constant<int, -1>{});
    else
        walk(std::integral_constant<int, 1>{});
    if constexpr (F)
        if (a.stress) store_stress<kBlock>(a.stress, ss, sc);
}

// ---------------------------------------------------------------- initial state
// SplitMix64 (Steele, Lea, Flood 2014): output k+1 of the stream started at seed.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <class L, int N, int S>
__global__ __launch_bounds__(kBlock) void k_init_wave(WaveArgs a) {
    using C = Codec<S>;
    using raw = typename C::raw;
    const uint32_t ncell = (uint32_t)a.nx * (uint32_t)a.ny * (uint32_t)a.nz;
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= ncell) return;
    const uint32_t yz = cell / (uint32_t)a.nx;
    const uint32_t j = a.wave_axis == 1 ? yz % (uint32_t)a.ny : yz / (uint32_t)a.ny;
    double rho = 1.0;
    if (a.rho_noise != 0.0) {
        const double U = (double)(splitmix64_at(a.seed, cell) >> 11) * 0x1.0p-53;
        rho = 1.0 + a.rho_noise * (2.0 * U - 1.0);
    }
    const double ux = a.u0 * a.sin_tab[j];
    double v[L::Q];
    equilibrium_v<L, N, S>(rho, ux, 0.0, 0.0, v);
    raw *f = static_cast<raw *>(a.f);
    static_for<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        f[a.lay.at(i, cell)] = C::template enc<false>((typename C::T)v[i], 0u);
    });
}

template <class L, int N, int S>
__global__ __launch_bounds__(kBlock) void k_init_fields(void *fv, Layout lay, uint32_t ncell,
                                                        const double *rho, const double *u) {
    using C = Codec<S>;
    using raw = typename C::raw;
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= ncell) return;
    double v[L::Q];
    equilibrium_v<L, N, S>(rho[cell], u[cell], u[ncell + cell], L::D == 3 ? u[2 * (size_t)ncell + cell] : 0.0, v);
    raw *f = static_cast<raw *>(fv);
    static_for<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        f[lay.at(i, cell)] = C::template enc<false>((typename C::T)v[i], 0u);
    });
}

// ---------------------------------------------------------------- codec kernels
template <int S>
__global__ __launch_bounds__(kBlock) void k_decode(const void *fv, Layout lay, uint32_t ncell, int a,
                                                   double add, double mul, double *out) {
    using C = Codec<S>;
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= ncell) return;
    const auto *f = static_cast<const typename C::raw *>(fv);
    out[cell] = add + mul * C::dec64(f[lay.at(a, cell)]);
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_gather(GatherArgs g) {
    using C = Codec<S>;
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (uint64_t)g.count * (uint64_t)g.Q) return;
    const uint32_t a = (uint32_t)(t / g.count), k = (uint32_t)(t - (uint64_t)a * g.count);
    const auto *f = static_cast<const typename C::raw *>(g.f);
    g.out[t] = g.add[a] + g.mul[a] * C::dec64(f[g.lay.at((int)a, g.cells[k])]);
}

template <int S, bool SR>
__global__ __launch_bounds__(kBlock) void k_encode(void *fv, Layout lay, uint32_t ncell, int a, double add,
                                                   double scale, const double *in, uint32_t key) {
    using C = Codec<S>;
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= ncell) return;
    auto *f = static_cast<typename C::raw *>(fv);
    const double v = (in[cell] - add) * scale;
    f[lay.at(a, cell)] = C::template enc<SR>((typename C::T)v, SR ? pop_bits_rt(cell_bits(cell, key), a) : 0u);
}

// Index of a cell along the force axis.
__device__ __forceinline__ uint32_t force_index(const DiagArgs &a, uint32_t cell) {
    const uint32_t yz = cell / (uint32_t)a.nx;
    return a.force_axis == 1 ? yz % (uint32_t)a.ny : yz / (uint32_t)a.ny;
}

// rho and the physical u in FP64 from the stored state (minus half the latest force).
template <class L, int S>
__global__ __launch_bounds__(kBlock) void k_moments(DiagArgs a, double *rho, double *u) {
    using C = Codec<S>;
    const uint32_t ncell = (uint32_t)a.nx * (uint32_t)a.ny * (uint32_t)a.nz;
    const uint32_t cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= ncell) return;
    const auto *f = static_cast<const typename C::raw *>(a.f);
    double v[L::Q];
    static_for<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        v[i] = C::dec64(f[a.lay.at(i, cell)]);
    });
    const Moments<double> m = project<L, S>(v);
    const double r = C::dev ? 1.0 + m.d : m.d;
    rho[cell] = r;
    double ux = m.jx / r;
    if (a.half_g != 0.0) ux -= a.half_g * a.force_cos[force_index(a, cell)];
    u[cell] = ux;
    u[ncell + cell] = m.jy / r;
    if (L::D == 3) u[2 * (size_t)ncell + cell] = m.jz / r;
}

// Deterministic FP64 reduction, stage 1: fixed grid-stride order per thread, fixed
// butterfly per wave (wave_sum), fixed order over the waves of the block.

template <class L, int S>
__global__ __launch_bounds__(kBlock) void k_diag(DiagArgs a) {
    using C = Codec<S>;
    const uint32_t ncell = (uint32_t)a.nx * (uint32_t)a.ny * (uint32_t)a.nz;
    const auto *f = static_cast<const typename C::raw *>(a.f);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t cell = blockIdx.x * kBlock + threadIdx.x; cell < ncell; cell += gridDim.x * kBlock) {
        double v[L::Q];
        static_for<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            v[i] = C::dec64(f[a.lay.at(i, cell)]);
        });
        const Moments<double> m = project<L, S>(v);
        const double r = C::dev ? 1.0 + m.d : m.d;
        double ux = m.jx / r, jx = m.jx;
        if (a.half_g != 0.0) {           // physical velocity and momentum: minus half the force
            const double hg = a.half_g * a.force_cos[force_index(a, cell)];
            ux -= hg;
            jx -= r * hg;
        }
        const uint32_t yz = cell / (uint32_t)a.nx;
        const uint32_t j = a.wave_axis == 1 ? yz % (uint32_t)a.ny : yz / (uint32_t)a.ny;
        acc[0] += ux * a.sin_tab[j];
        acc[1] += ux * a.cos_tab[j];
        acc[2] += m.d;
        acc[3] += jx;
        acc[4] += m.jy;
        acc[5] += m.jz;
    }
    __shared__ double red[kBlock / 64][6];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) red[wv][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
        a.partials[(size_t)blockIdx.x * 6 + threadIdx.x] = s;
    }
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_finite(const void *fv, Layout lay, uint32_t ncell, int Q,
                                                   int *flag) {
    using C = Codec<S>;
    const auto *f = static_cast<const typename C::raw *>(fv);
    bool bad = false;
    for (uint32_t cell = blockIdx.x * kBlock + threadIdx.x; cell < ncell; cell += gridDim.x * kBlock)
        for (int i = 0; i < Q; ++i) bad |= !isfinite((double)C::dec(f[lay.at(i, cell)]));
    if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------- host launchers
inline uint32_t blocks_for(uint32_t n) { return (n + kBlock - 1) / kBlock; }

template <class L, int N, int S, bool SR, int BLOCK, bool NTS, bool F>
hipError_t launch_shift_rows(const StepArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_shift_rows<L, N, S, SR, BLOCK, NTS, F>), dim3(a.nblocks), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}
template <class L, int N, int S, bool SR, bool NTL>
hipError_t launch_shift_rows4(const StepArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_shift_rows4<L, N, S, SR, NTL>), dim3(a.nblocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}
template <class L, int N, int S, bool SR, bool F>
hipError_t launch_shift_cells(const StepArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_shift_cells<L, N, S, SR, F>), dim3(a.nblocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}
template <class L, int N, int S, bool SR, class T, bool F, bool NTS, bool ALT, bool NTL = false, bool PIPE = false>
hipError_t launch_bw2(const StepArgs &a, const BWCoef<T> &cf, hipStream_t s) {
    hipLaunchKernelGGL((k_bw2<L, N, S, SR, T, F, NTS, ALT, NTL, PIPE>), dim3(a.nblocks), dim3(kBlock), 0, s, a, cf);
    return hipGetLastError();
}
template <class L, int N, int S>
hipError_t launch_init_wave(const WaveArgs &a, hipStream_t s) {
    const uint32_t ncell = (uint32_t)a.nx * (uint32_t)a.ny * (uint32_t)a.nz;
    hipLaunchKernelGGL((k_init_wave<L, N, S>), dim3(blocks_for(ncell)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}
template <class L, int N, int S>
hipError_t launch_init_fields(void *f, const Layout &lay, uint32_t ncell, const double *rho, const double *u,
                              hipStream_t s) {
    hipLaunchKernelGGL((k_init_fields<L, N, S>), dim3(blocks_for(ncell)), dim3(kBlock), 0, s, f, lay, ncell, rho, u);
    return hipGetLastError();
}
template <int S>
hipError_t launch_decode(const void *f, const Layout &lay, uint32_t ncell, int a, double add, double mul, double *out,
                         hipStream_t s) {
    hipLaunchKernelGGL((k_decode<S>), dim3(blocks_for(ncell)), dim3(kBlock), 0, s, f, lay, ncell, a, add, mul, out);
    return hipGetLastError();
}
template <int S, bool SR>
hipError_t launch_encode(void *f, const Layout &lay, uint32_t ncell, int a, double add, double scale, const double *in,
                         uint32_t key, hipStream_t s) {
    hipLaunchKernelGGL((k_encode<S, SR>), dim3(blocks_for(ncell)), dim3(kBlock), 0, s, f, lay, ncell, a, add, scale,
                       in, key);
    return hipGetLastError();
}
template <int S>
hipError_t launch_gather(const GatherArgs &g, hipStream_t s) {
    const uint64_t n = (uint64_t)g.count * (uint64_t)g.Q;
    hipLaunchKernelGGL((k_gather<S>), dim3((uint32_t)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, g);
    return hipGetLastError();
}
template <class L, int S>
hipError_t launch_moments(const DiagArgs &a, double *rho, double *u, hipStream_t s) {
    const uint32_t ncell = (uint32_t)a.nx * (uint32_t)a.ny * (uint32_t)a.nz;
    hipLaunchKernelGGL((k_moments<L, S>), dim3(blocks_for(ncell)), dim3(kBlock), 0, s, a, rho, u);
    return hipGetLastError();
}
template <class L, int S>
hipError_t launch_diag(const DiagArgs &a, uint32_t nblocks, hipStream_t s) {
    hipLaunchKernelGGL((k_diag<L, S>), dim3(nblocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}
template <int S>
hipError_t launch_finite(const void *f, const Layout &lay, uint32_t ncell, int Q, int *flag, hipStream_t s) {
    uint32_t nb = blocks_for(ncell);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL((k_finite<S>), dim3(nb), dim3(kBlock), 0, s, f, lay, ncell, Q, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------- registration
template <class L, int N, int S, bool SR>
KernelSet make_set() {
    KernelSet k{};
    k.lattice = L::id;
    k.order = N;
    k.storage = S;
    k.sr = SR ? 1 : 0;
    if constexpr (L::on_lattice) {
        k.shift_rows[0] = &launch_shift_rows<L, N, S, SR, 256, false, false>;
        k.shift_rows[1] = &launch_shift_rows<L, N, S, SR, 256, true, false>;
        k.shift_rows[2] = &launch_shift_rows<L, N, S, SR, 512, true, false>;
        k.shift_cells = &launch_shift_cells<L, N, S, SR, false>;
        k.shift_rows_forced[0] = &launch_shift_rows<L, N, S, SR, 256, false, true>;
        k.shift_rows_forced[1] = &launch_shift_rows<L, N, S, SR, 512, true, true>;
        if constexpr (max_cx<L>() <= 4 && (S == ST_FP32 || S == ST_FP32_DEV))
            k.shift_rows4 = &launch_shift_rows4<L, N, S, SR, true>;
        k.shift_cells_forced = &launch_shift_cells<L, N, S, SR, true>;
    } else if constexpr (L::D == 2) {
        if constexpr (S == ST_FP64) {
            k.bw2_f64[0] = &launch_bw2<L, N, S, SR, double, false, false, false>;
            k.bw2_f64[1] = &launch_bw2<L, N, S, SR, double, false, true, false>;
            k.bw2_f64[2] = &launch_bw2<L, N, S, SR, double, false, true, true>;
            k.bw2_f64[3] = &launch_bw2<L, N, S, SR, double, false, true, true, true>;
            k.bw2_f64[4] = &launch_bw2<L, N, S, SR, double, false, true, true, false, true>;
            k.bw2_f64_forced = &launch_bw2<L, N, S, SR, double, true, false, false>;
        } else {
            k.bw2_f32[0] = &launch_bw2<L, N, S, SR, float, false, false, false>;
            k.bw2_f32[1] = &launch_bw2<L, N, S, SR, float, false, true, false>;
            k.bw2_f32[2] = &launch_bw2<L, N, S, SR, float, false, true, true>;
            k.bw2_f32[3] = &launch_bw2<L, N, S, SR, float, false, true, true, true>;
            k.bw2_f32[4] = &launch_bw2<L, N, S, SR, float, false, true, true, false, true>;
            k.bw2_f32_forced = &launch_bw2<L, N, S, SR, float, true, false, false>;
        }
    }
    k.init_wave = &launch_init_wave<L, N, S>;
    k.init_fields = &launch_init_fields<L, N, S>;
    k.decode = &launch_decode<S>;
    k.encode = &launch_encode<S, SR>;
    k.moments = &launch_moments<L, S>;
    k.diag = &launch_diag<L, S>;
    k.finite = &launch_finite<S>;
    k.gather = &launch_gather<S>;
    return k;
}

template <class L, int N>
void register_order(std::vector<KernelSet> &r) {
    r.push_back(make_set<L, N, ST_FP64, false>());
    r.push_back(make_set<L, N, ST_FP32, false>());
    r.push_back(make_set<L, N, ST_FP32_DEV, false>());
    r.push_back(make_set<L, N, ST_FP16_DEV, false>());
    r.push_back(make_set<L, N, ST_FP16_DEV, true>());
    r.push_back(make_set<L, N, ST_BF16_DEV, false>());
    r.push_back(make_set<L, N, ST_BF16_DEV, true>());
}

template <class L>
void register_lattice() {
    auto &r = registry();
    register_order<L, 1>(r);
    register_order<L, 2>(r);
    register_order<L, 3>(r);
    register_order<L, 4>(r);
}

}  // namespace lbm
