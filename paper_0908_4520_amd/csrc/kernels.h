// kernels.h -- interface between the host runtime and the per-lattice kernel units.
//
// Each lattice unit (k_<lattice>.hip) instantiates the templates of kernels_impl.h for
// its velocity set and fills a table of host launchers; the runtime (runtime.cpp) picks the
// entry for a simulation's (lattice, Hermite order, storage, rounding).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace lbm {

constexpr int kMaxQ = 40;       // largest Q of any supported set (D3Q39)
constexpr int kBlock = 256;     // threads per workgroup of every step kernel
constexpr int kMaxDiagBlocks = 2048;   // workgroups of the diagnostic reduction (grid-stride)

// Where population i of cell (x, r) lives, r = y + ny z the row index: element
// r * row + i * pop + x of a buffer.  A simulation stores the Q populations of each grid row
// one after another (pop = nx, row = Q nx), so the rows a step reads lie close together in
// memory; a batch instance stores one plane per population (pop = plane size, row = nx).
struct Layout {
    uint32_t nx, pop;
    uint64_t row;
    __host__ __device__ size_t at(int i, uint32_t cell) const {
        const uint32_t r = cell / nx;
        return (size_t)r * row + (size_t)i * pop + (cell - r * nx);
    }
};

// Arguments shared by the step kernels (passed by value as kernel arguments).
struct StepArgs {
    const void *fin;
    void *fout;
    int32_t nx, ny, nz;
    Layout lay;
    uint32_t per_row;      // shift rows kernel: blocks per row; bw2: blocks per strip row
    uint32_t tile;         // shift rows kernel: block-size chunks per block; bw2: rows per strip
    uint32_t nblocks;      // grid size (1-D)
    uint32_t sr_key;       // per-step key of the stochastic-rounding stream
    double omega;          // 1/tau (0 = collisionless)
    // Body force of the standing shear wave, read by the forced kernels only:
    // G_x(cell) = force_g * force_cos[j], j the cell's index along force_axis.
    double force_g;            // force times dt at this step's collision time
    const double *force_cos;   // cos(2 pi j / N_w) along the force axis
    const double *force_sin;   // sin(2 pi j / N_w), weights of the stress projection
    double *stress;            // per-wave sums [nblocks * waves per block][2] of the shear stress
                               // times sin and cos, or null
    int32_t force_axis;        // 1 (y) or 2 (z)
};

// Beam-Warming coefficients per population and axis: g = f - alpha D1 + beta D2 with
// alpha = a + a(1-a)/2, beta = a(1-a)/2, a = |nu| (D1, D2 the one-sided differences).
template <class T>
struct BWCoef {
    T alpha[2][kMaxQ];
    T beta[2][kMaxQ];
};

struct WaveArgs {
    void *f;
    int32_t nx, ny, nz;
    Layout lay;
    int32_t wave_axis;
    double u0, rho_noise;
    uint64_t seed;
    const double *sin_tab;   // sin(2 pi j / N_w), j = 0..N_w-1 (host libm)
};

struct DiagArgs {
    const void *f;
    int32_t nx, ny, nz;
    Layout lay;
    int32_t wave_axis;
    const double *sin_tab, *cos_tab;
    double *partials;        // [nblocks][6]: sum u_x sin, sum u_x cos, sum d, sum j_x, j_y, j_z
    // Half the force times dt of the latest collision (0 if none): the velocity is
    // sum_a xi_a f*_a / rho - G/2 with G_x = 2 half_g force_cos[j] (j along force_axis).
    double half_g;
    const double *force_cos;
    int32_t force_axis;
};

using StepFn = hipError_t (*)(const StepArgs &, hipStream_t);
using StepBW32 = hipError_t (*)(const StepArgs &, const BWCoef<float> &, hipStream_t);
using StepBW64 = hipError_t (*)(const StepArgs &, const BWCoef<double> &, hipStream_t);
using WaveFn = hipError_t (*)(const WaveArgs &, hipStream_t);
using FieldsFn = hipError_t (*)(void *f, const Layout &lay, uint32_t ncell, const double *rho,
                                const double *u, hipStream_t);
using DecodeFn = hipError_t (*)(const void *f, const Layout &lay, uint32_t ncell, int a, double add,
                                double mul, double *out, hipStream_t);
using EncodeFn = hipError_t (*)(void *f, const Layout &lay, uint32_t ncell, int a, double add,
                                double scale, const double *in, uint32_t sr_key, hipStream_t);
using MomentsFn = hipError_t (*)(const DiagArgs &, double *rho, double *u, hipStream_t);
using DiagFn = hipError_t (*)(const DiagArgs &, uint32_t nblocks, hipStream_t);
using FiniteFn = hipError_t (*)(const void *f, const Layout &lay, uint32_t ncell, int Q, int *flag,
                                hipStream_t);

// Decoded populations of listed cells: out[a * count + k] = add[a] + mul[a] * f_a(cells[k]).
struct GatherArgs {
    const void *f;
    Layout lay;
    const uint32_t *cells;
    uint32_t count;
    int32_t Q;
    double *out;
    double add[kMaxQ], mul[kMaxQ];
};
using GatherFn = hipError_t (*)(const GatherArgs &, hipStream_t);

// Everything for one (lattice, N, storage, rounding) combination.
struct KernelSet {
    int lattice, order, storage, sr;
    StepFn shift_rows[3];  // on-lattice shift, row tiles (needs nx, ny, nz >= R): 256 threads,
                           // 256 threads with non-temporal stores, 512 threads non-temporal
    StepFn shift_rows4;    // on-lattice shift, 4 cells per thread, vector loads and stores, non-temporal
                           // loads (FP32 storages, |c_x| <= 4, nx a multiple of 256; else null)
    StepFn shift_cells;    // on-lattice shift, one thread per cell (any grid)
    StepBW32 bw2_f32[5];   // Beam-Warming advection (2-D sets), FP32 collision: plain stores,
                           // non-temporal stores, non-temporal stores with alternating strip walks,
                           // the same with non-temporal loads, the same (plain loads) with the next
                           // row's loads issued before the current row is computed
    StepBW64 bw2_f64[5];   // the same with the FP64 collision
    // The same with the body force (row tiles: 256 threads with plain stores, 512 threads with
    // non-temporal stores)
    StepFn shift_rows_forced[2];
    StepFn shift_cells_forced;
    StepBW32 bw2_f32_forced;
    StepBW64 bw2_f64_forced;
    WaveFn init_wave;
    FieldsFn init_fields;
    DecodeFn decode;
    EncodeFn encode;
    MomentsFn moments;
    DiagFn diag;
    FiniteFn finite;
    GatherFn gather;
};

std::vector<KernelSet> &registry();

void register_D2Q9();
void register_D2Q37();
void register_D3Q39();
void register_D2Q16_GH();
void register_D2Q36_GH();
void register_D2Q16_CK();
void register_D2Q17();
void register_D2Q21();
void register_D2Q25_CK();

// Zero n ints with a kernel (kept out of hipMemsetAsync so the step path can be captured).
hipError_t fill_zero(int *p, uint32_t n, hipStream_t s);

// Grid-stride copy of `words` 16-byte words with `blocks` workgroups of 256 threads.
hipError_t copy16(const void *src, void *dst, uint64_t words, uint32_t blocks, hipStream_t s);

// Fixed-order final reduction of per-block partial sums: out[k] = sum_b partials[b][k],
// k < width <= 8 (width 6 for DiagFn partials, 2 for the stress sums of the forced steps).
hipError_t diag_final(const double *partials, uint32_t nblocks, int width, double *out, hipStream_t s);

}  // namespace lbm
