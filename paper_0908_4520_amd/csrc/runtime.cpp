// runtime.cpp -- host side of the C ABI declared in include/lbm.h: argument validation,
// device buffers, kernel selection, step loop, readbacks and the decay-rate fit.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "batch.h"
#include "host_logic.h"
#include "kernels.h"
#include "lattices.inc"
#include "lbm.h"
#include "noalloc.h"

using namespace lbm;
using host::kBWTiles;
using host::kShiftTiles;
static_assert(host::kCellBlock == (uint32_t)kBlock, "one-thread-per-cell kernels run kBlock threads");

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(e_ == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                   \
    } while (0)

struct LatInfo {
    int id, Q, D, R, degree;
    bool on_lattice;
    double scale, xi_max;
    const int (*c)[3];
    const double (*xi)[3];
    const double *w;
};

template <class L>
LatInfo info_of() {
    return LatInfo{L::id, L::Q, L::D, L::R, L::degree, L::on_lattice, L::scale, L::xi_max, L::c, L::xi, L::w};
}

const LatInfo *lat_info(int id) {
    static const LatInfo table[] = {info_of<D2Q9>(),     info_of<D2Q37>(), info_of<D3Q39>(),
                                    info_of<D2Q16_GH>(), info_of<D2Q36_GH>(), info_of<D2Q16_CK>(),
                                    info_of<D2Q17>(),    info_of<D2Q21>(), info_of<D2Q25_CK>()};
    for (const auto &t : table)
        if (t.id == id) return &t;
    return nullptr;
}

void ensure_registered() {
    static std::once_flag once;
    std::call_once(once, [] {
        register_D2Q9();
        register_D2Q37();
        register_D3Q39();
        register_D2Q16_GH();
        register_D2Q36_GH();
        register_D2Q16_CK();
        register_D2Q17();
        register_D2Q21();
        register_D2Q25_CK();
    });
}

const KernelSet *find_kernels(int lat, int N, int storage, int sr) {
    ensure_registered();
    for (const auto &k : registry())
        if (k.lattice == lat && k.order == N && k.storage == storage && k.sr == sr) return &k;
    return nullptr;
}

int elem_size(lbm_storage s) {
    switch (s) {
        case LBM_FP64: return 8;
        case LBM_FP32:
        case LBM_FP32_DEV: return 4;
        default: return 2;
    }
}
bool is_dev(lbm_storage s) { return s == LBM_FP32_DEV || s == LBM_FP16_DEV || s == LBM_BF16_DEV; }
bool is_scaled(lbm_storage s) { return s == LBM_FP16_DEV; }

uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}


}  // namespace

struct lbm_sim {
    const LatInfo *L = nullptr;
    int N = 0;
    double tau = 0, omega = 0;
    lbm_grid g{};
    size_t ncell = 0;
    Layout lay{};              // row-interleaved: the Q populations of each row one after another
    lbm_opts o{};
    lbm_move move = LBM_MOVE_AUTO;
    int esize = 0;
    hipStream_t stream = nullptr;
    void *buf[2] = {nullptr, nullptr};
    bool own_buf = true;        // false: buf[] came from lbm_opts.dev_buf (the caller frees them)
    int device = 0;             // HIP device current at creation
    int cur = 0;
    int64_t nstep = 0;
    const KernelSet *ks = nullptr;
    bool rows_ok = false;       // row-tiled shift kernel is valid for this grid
    int tile = 0;
    double *d_tab = nullptr;    // sin(2 pi j / ny), cos(2 pi j / ny) for j < ny, then the same along z
                                // (3-D sets), made at creation
    double *d_partials = nullptr;
    double *d_result = nullptr;
    int *d_flag = nullptr;
    uint32_t diag_blocks = 0;
    uint32_t warnings = 0;
    BWCoef<float> bwf{};
    BWCoef<double> bwd{};
    // body force F_x = f_amp cos(f_freq t) cos(2 pi j / N_w) along f_axis (Eq. force)
    bool forced = false;
    double f_amp = 0, f_freq = 0, f_dt = 0;
    int f_axis = 0;
    double *d_ftab = nullptr;       // cos then sin along the force axis
    double *d_stress = nullptr;     // per-wave stress sums of the latest forced step
    uint32_t stress_slots = 0;      // slots written by that step
    uint32_t stress_cap = 0;        // slots allocated
    bool stress_valid = false;
};

namespace {

// Force times dt at the collision of step n (time n dt); zero before the first step.
double force_g_at(const lbm_sim *s, int64_t n) {
    if (!s->forced || n <= 0) return 0.0;
    return s->f_amp * s->f_dt * cos(s->f_freq * (double)n * s->f_dt);
}

// What the tile choice of a simulation depends on.
host::StepShape step_shape(const lbm_sim *s) {
    host::StepShape h{};
    h.bw2 = s->move == LBM_MOVE_BW2;
    h.rows_ok = s->rows_ok;
    h.forced = s->forced;
    h.vector_ok = s->ks->shift_rows4 != nullptr && s->g.nx % 256 == 0;
    h.nx = s->g.nx;
    h.ny = s->g.ny;
    h.nz = s->g.nz;
    return h;
}

StepArgs step_args(const lbm_sim *s, const void *fin, void *fout, int tile_index) {
    StepArgs a{};
    a.fin = fin;
    a.fout = fout;
    a.nx = s->g.nx;
    a.ny = s->g.ny;
    a.nz = s->g.nz;
    a.lay = s->lay;
    a.omega = s->omega;
    a.sr_key = (uint32_t)splitmix64(s->o.sr_seed ^ (0x5851F42D4C957F2Dull * (uint64_t)(s->nstep + 1)));
    const host::StepGeom g = host::step_geometry(step_shape(s), tile_index);
    a.tile = g.tile;
    a.per_row = g.per_row;
    a.nblocks = g.nblocks;
    return a;
}

// Per-wave stress sums a forced step with tile tile_index stores.
uint32_t stress_slots(const lbm_sim *s, int tile_index) {
    const uint32_t waves = (s->move != LBM_MOVE_BW2 && s->rows_ok) ? (uint32_t)kShiftTiles[tile_index].block / 64u
                                                                   : (uint32_t)(kBlock / 64);
    return step_args(s, s->buf[0], s->buf[1], tile_index).nblocks * waves;
}

// One step from fin to fout with tile tile_index.  A forced simulation runs the forced
// kernels; with record_stress they also store the per-wave stress sums.
hipError_t launch_step(lbm_sim *s, const void *fin, void *fout, int tile_index, bool record_stress) {
    StepArgs a = step_args(s, fin, fout, tile_index);
    const KernelSet *k = s->ks;
    if (s->forced) {
        a.force_g = force_g_at(s, s->nstep + 1);
        a.force_cos = s->d_ftab;
        a.force_sin = s->d_ftab + (s->f_axis == 1 ? s->g.ny : s->g.nz);
        a.force_axis = s->f_axis;
        if (record_stress) {
            const uint32_t slots = stress_slots(s, tile_index);
            if (slots > s->stress_cap) return hipErrorInvalidValue;
            a.stress = s->d_stress;
            s->stress_slots = slots;
        }
        if (s->move == LBM_MOVE_BW2)
            return s->o.storage == LBM_FP64 ? k->bw2_f64_forced(a, s->bwd, s->stream)
                                            : k->bw2_f32_forced(a, s->bwf, s->stream);
        if (!s->rows_ok) return k->shift_cells_forced(a, s->stream);
        return k->shift_rows_forced[kShiftTiles[tile_index].variant == 2 ? 1 : 0](a, s->stream);
    }
    if (s->move == LBM_MOVE_BW2) {
        const int v = kBWTiles[tile_index].variant;
        return s->o.storage == LBM_FP64 ? k->bw2_f64[v](a, s->bwd, s->stream) : k->bw2_f32[v](a, s->bwf, s->stream);
    }
    if (!s->rows_ok) return k->shift_cells(a, s->stream);
    const int v = kShiftTiles[tile_index].variant;
    return v == 3 ? k->shift_rows4(a, s->stream) : k->shift_rows[v](a, s->stream);
}

int tile_count(const lbm_sim *s) { return host::tile_count(step_shape(s)); }

// Host values of the wave tables (host libm): for each wave axis (y, then z for 3-D sets)
// sin(2 pi j / N_w) then cos(2 pi j / N_w), j < N_w.
std::vector<double> wave_tables(const lbm_sim *s) {
    std::vector<double> h;
    for (int axis = 1; axis <= (s->L->D == 3 ? 2 : 1); ++axis) {
        const int nw = axis == 1 ? s->g.ny : s->g.nz;
        const size_t o = h.size();
        h.resize(o + 2 * (size_t)nw);
        for (int j = 0; j < nw; ++j) {
            const double ph = 2.0 * M_PI * (double)j / (double)nw;
            h[o + j] = sin(ph);
            h[o + nw + j] = cos(ph);
        }
    }
    return h;
}
const double *sin_table(const lbm_sim *s, int axis) { return s->d_tab + (axis == 1 ? 0 : 2 * (size_t)s->g.ny); }
const double *cos_table(const lbm_sim *s, int axis) { return sin_table(s, axis) + (axis == 1 ? s->g.ny : s->g.nz); }

lbm_status check_axis(const lbm_sim *s, int axis) {
    if (axis == 1) return LBM_OK;
    if (axis == 2 && s->L->D == 3) return LBM_OK;
    return fail(LBM_EINVAL, "wave_axis must be 1 (y) or, for 3-D sets, 2 (z); got %d", axis);
}

// Arguments of the diagnostic reduction of the current state along `axis` into `partials`.
DiagArgs diag_args(const lbm_sim *s, int axis, double *partials) {
    DiagArgs a{};
    a.f = s->buf[s->cur];
    a.nx = s->g.nx;
    a.ny = s->g.ny;
    a.nz = s->g.nz;
    a.lay = s->lay;
    a.wave_axis = axis;
    a.sin_tab = sin_table(s, axis);
    a.cos_tab = cos_table(s, axis);
    a.partials = partials;
    a.half_g = 0.5 * force_g_at(s, s->nstep);
    a.force_cos = s->d_ftab;
    a.force_axis = s->f_axis;
    return a;
}

// Runs the diagnostic reduction and copies the 6 sums to host.
lbm_status run_diag(lbm_sim *s, int axis, double out[6]) {
    const DiagArgs a = diag_args(s, axis, s->d_partials);
    HIP_TRY(s->ks->diag(a, s->diag_blocks, s->stream));
    HIP_TRY(diag_final(s->d_partials, s->diag_blocks, 6, s->d_result, s->stream));
    HIP_TRY(hipMemcpyAsync(out, s->d_result, 6 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return LBM_OK;
}

// Caller-owned population buffers (lbm_opts.dev_buf): both given, large enough, aligned for
// the 16-byte vector accesses, disjoint, and device memory of the current device.
lbm_status check_dev_buffers(const lbm_opts &o, size_t need) {
    std::string msg;
    if (host::check_dev_buf_shape(o, need, &msg) != LBM_OK) return fail(LBM_EINVAL, "%s", msg.c_str());
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LBM_EDEVICE, "dev_buf: no HIP device");
    }
    for (int k = 0; k < 2; ++k) {
        hipPointerAttribute_t at{};
        const hipError_t e = hipPointerGetAttributes(&at, o.dev_buf[k]);
        if (e != hipSuccess) (void)hipGetLastError();
        if (e != hipSuccess || at.type != hipMemoryTypeDevice || at.device != dev)
            return fail(LBM_EINVAL, "dev_buf[%d] is not device memory of the current device %d", k, dev);
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

void lbm_opts_default(lbm_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->storage = LBM_FP64;
    o->move = LBM_MOVE_AUTO;
    o->cfl = 0.5;
}

const char *lbm_last_error(void) { return g_err.c_str(); }

lbm_status lbm_lattice_info(lbm_lattice lat, int32_t *Q, int32_t *D, int32_t *c, double *xi, double *w) {
    const LatInfo *L = lat_info((int)lat);
    if (!L) return fail(LBM_EINVAL, "unknown lattice %d", (int)lat);
    if (Q) *Q = L->Q;
    if (D) *D = L->D;
    for (int a = 0; a < L->Q; ++a) {
        for (int d = 0; d < 3; ++d) {
            if (c) c[3 * a + d] = L->c[a][d];
            if (xi) xi[3 * a + d] = L->xi[a][d];
        }
        if (w) w[a] = L->w[a];
    }
    return LBM_OK;
}

double lbm_time_step(lbm_lattice lat, lbm_move move, int32_t wavelength_cells, double cfl) {
    const LatInfo *L = lat_info((int)lat);
    if (!L || wavelength_cells < 1) return NAN;
    if (move == LBM_MOVE_AUTO) move = L->on_lattice ? LBM_MOVE_SHIFT : LBM_MOVE_BW2;
    const double dx = 2.0 * M_PI / (double)wavelength_cells;
    if (move == LBM_MOVE_SHIFT) return L->on_lattice ? dx / L->scale : NAN;
    if (move != LBM_MOVE_BW2 || !(cfl > 0.0 && cfl <= 1.0)) return NAN;
    return cfl * dx / L->xi_max;
}

double lbm_tau_from_kn(lbm_lattice lat, lbm_move move, double kn, int32_t wavelength_cells, double cfl) {
    if (!(kn >= 0.0)) return NAN;
    const double dt = lbm_time_step(lat, move, wavelength_cells, cfl);
    return isnan(dt) ? NAN : kn / dt + 0.5;
}

lbm_status lbm_init(lbm_sim **out, lbm_lattice lat, int32_t eq_order, double tau, lbm_grid g) {
    return lbm_init_ex(out, lat, eq_order, tau, g, nullptr);
}

lbm_status lbm_init_ex(lbm_sim **out, lbm_lattice lat, int32_t eq_order, double tau, lbm_grid g,
                       const lbm_opts *opts) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    const LatInfo *L = lat_info((int)lat);
    if (!L) return fail(LBM_EINVAL, "unknown lattice %d", (int)lat);
    lbm_opts o;
    lbm_opts_default(&o);
    if (opts) o = *opts;
    const host::LatShape shape{L->Q, L->D, L->R, L->on_lattice};
    lbm_move move = LBM_MOVE_AUTO;
    std::string msg;
    if (host::check_init(&shape, eq_order, tau, g, o, host::storage_bytes(o), &move, &msg) != LBM_OK)
        return fail(LBM_EINVAL, "%s", msg.c_str());
    const unsigned long long ncell = (unsigned long long)g.nx * g.ny * g.nz;
    const size_t state_bytes = (size_t)L->Q * (size_t)ncell * (size_t)elem_size(o.storage);
    const bool given = o.dev_buf[0] != nullptr || o.dev_buf[1] != nullptr;
    if (given) {
        lbm_status st = check_dev_buffers(o, state_bytes);
        if (st != LBM_OK) return st;
    }
    const int sr = (o.stochastic_round && (o.storage == LBM_FP16_DEV || o.storage == LBM_BF16_DEV)) ? 1 : 0;
    const KernelSet *ks = find_kernels((int)lat, eq_order, (int)o.storage, sr);
    if (!ks) return fail(LBM_EINVAL, "no kernels for lattice %d order %d storage %d", (int)lat, eq_order, (int)o.storage);

    lbm_sim *s = new lbm_sim();
    s->L = L;
    s->N = eq_order;
    s->tau = tau;
    s->omega = isinf(tau) ? 0.0 : 1.0 / tau;
    s->g = g;
    s->ncell = (size_t)ncell;
    s->lay = Layout{(uint32_t)g.nx, (uint32_t)g.nx, (uint64_t)L->Q * (uint64_t)g.nx};
    s->o = o;
    s->move = move;
    s->esize = elem_size(o.storage);
    s->stream = (hipStream_t)o.hip_stream;
    s->ks = ks;
    // the row-tiled and Beam-Warming kernels address a grid row (all Q populations) with 32-bit offsets
    s->rows_ok = host::row_tiles_ok(move == LBM_MOVE_SHIFT, L->Q, L->D, L->R, g, elem_size(o.storage));
    s->tile = (o.tile > 0 && o.tile < tile_count(s)) ? o.tile : 0;
    if (L->degree < 2 * eq_order) s->warnings |= LBM_WARN_QUADRATURE;
    if (move == LBM_MOVE_BW2) {
        const double lam = o.cfl / L->xi_max;
        for (int a = 0; a < L->Q; ++a)
            for (int d = 0; d < 2; ++d) {
                const double A = fabs(L->xi[a][d] * lam);
                const double b = 0.5 * A * (1.0 - A);
                s->bwd.alpha[d][a] = A + b;
                s->bwd.beta[d][a] = b;
                s->bwf.alpha[d][a] = (float)(A + b);
                s->bwf.beta[d][a] = (float)b;
            }
    }
    s->diag_blocks = (uint32_t)std::min<size_t>((s->ncell + kBlock - 1) / kBlock, kMaxDiagBlocks);
    const size_t bytes = state_bytes;
    hipError_t e = hipGetDevice(&s->device);
    if (given) {
        s->own_buf = false;
        s->buf[0] = o.dev_buf[0];
        s->buf[1] = o.dev_buf[1];
    } else {
        if (e == hipSuccess) e = hipMalloc(&s->buf[0], bytes);
        if (e == hipSuccess) e = hipMalloc(&s->buf[1], bytes);
    }
    const std::vector<double> tabs = wave_tables(s);
    if (e == hipSuccess) e = hipMalloc(&s->d_tab, sizeof(double) * tabs.size());
    if (e == hipSuccess) e = hipMemcpyAsync(s->d_tab, tabs.data(), sizeof(double) * tabs.size(), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMalloc(&s->d_partials, sizeof(double) * 6 * s->diag_blocks);
    if (e == hipSuccess) e = hipMalloc(&s->d_result, sizeof(double) * 8);
    if (e == hipSuccess) e = hipMalloc(&s->d_flag, sizeof(int) * 4);
    if (e == hipSuccess) e = hipMemsetAsync(s->buf[0], 0, bytes, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->buf[1], 0, bytes, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        lbm_status st = fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE,
                             "allocating %zu bytes of populations: %s", 2 * bytes, hipGetErrorString(e));
        lbm_free(s);
        (void)hipGetLastError();
        return st;
    }
    // address of this device's scratch array for lbm_shear_amplitude_noalloc (once per device);
    // a failure here is reported by that entry point, not by the creation
    (void)noalloc_setup(s->device);
    *out = s;
    return LBM_OK;
}

void lbm_free(lbm_sim *s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    if (s->own_buf)
        for (void *p : {s->buf[0], s->buf[1]})
            if (p) (void)hipFree(p);
    for (void *p : {(void *)s->d_tab, (void *)s->d_partials, (void *)s->d_result, (void *)s->d_flag,
                    (void *)s->d_ftab, (void *)s->d_stress})
        if (p) (void)hipFree(p);
    delete s;
}

uint32_t lbm_warnings(const lbm_sim *s) { return s ? s->warnings : 0u; }

int64_t lbm_step_count(const lbm_sim *s) { return s ? s->nstep : -1; }

lbm_status lbm_sizes(const lbm_sim *s, int64_t *ncell, int32_t *Q, int32_t *D, int64_t *bytes_per_step) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (ncell) *ncell = (int64_t)s->ncell;
    if (Q) *Q = s->L->Q;
    if (D) *D = s->L->D;
    if (bytes_per_step) *bytes_per_step = 2ll * s->L->Q * (int64_t)s->ncell * s->esize;
    return LBM_OK;
}

lbm_status lbm_set_shear_wave(lbm_sim *s, double u0, int32_t wave_axis, double rho_noise, uint64_t seed) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    lbm_status st = check_axis(s, wave_axis);
    if (st != LBM_OK) return st;
    if (!isfinite(u0) || !isfinite(rho_noise) || fabs(rho_noise) >= 1.0)
        return fail(LBM_EINVAL, "u0 and rho_noise must be finite, |rho_noise| < 1");
    WaveArgs a{};
    a.f = s->buf[0];
    a.nx = s->g.nx;
    a.ny = s->g.ny;
    a.nz = s->g.nz;
    a.lay = s->lay;
    a.wave_axis = wave_axis;
    a.u0 = u0;
    a.rho_noise = rho_noise;
    a.seed = seed;
    a.sin_tab = sin_table(s, wave_axis);
    HIP_TRY(s->ks->init_wave(a, s->stream));
    s->cur = 0;
    s->nstep = 0;
    s->stress_valid = false;
    return LBM_OK;
}

lbm_status lbm_init_equilibrium(lbm_sim *s, const double *rho, const double *u) {
    if (!s || !rho || !u) return fail(LBM_EINVAL, "NULL argument");
    const size_t n = s->ncell, D = (size_t)s->L->D;
    double *d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(double) * n * (1 + D)));
    hipError_t e = hipMemcpyAsync(d, rho, sizeof(double) * n, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d + n, u, sizeof(double) * n * D, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = s->ks->init_fields(s->buf[0], s->lay, (uint32_t)n, d, d + n, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d);
    HIP_TRY(e);
    s->cur = 0;
    s->nstep = 0;
    s->stress_valid = false;
    return LBM_OK;
}

lbm_status lbm_step(lbm_sim *s, int64_t n) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
    for (int64_t k = 0; k < n; ++k) {
        HIP_TRY(launch_step(s, s->buf[s->cur], s->buf[s->cur ^ 1], s->tile, true));
        s->cur ^= 1;
        s->nstep += 1;
        s->stress_valid = s->forced;
        if (s->o.check_every > 0 && s->nstep % s->o.check_every == 0) {
            HIP_TRY(fill_zero(s->d_flag, 1, s->stream));
            HIP_TRY(s->ks->finite(s->buf[s->cur], s->lay, (uint32_t)s->ncell, s->L->Q, s->d_flag, s->stream));
            int flag = 0;
            HIP_TRY(hipMemcpyAsync(&flag, s->d_flag, sizeof(int), hipMemcpyDeviceToHost, s->stream));
            HIP_TRY(hipStreamSynchronize(s->stream));
            if (flag) return fail(LBM_ENONFINITE, "non-finite population after step %lld", (long long)s->nstep);
        }
    }
    return LBM_OK;
}

lbm_status lbm_moments(lbm_sim *s, double *rho, double *u) {
    if (!s || !rho || !u) return fail(LBM_EINVAL, "NULL argument");
    const size_t n = s->ncell, D = (size_t)s->L->D;
    double *d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(double) * n * (1 + D)));
    DiagArgs a{};
    a.f = s->buf[s->cur];
    a.nx = s->g.nx;
    a.ny = s->g.ny;
    a.nz = s->g.nz;
    a.lay = s->lay;
    a.half_g = 0.5 * force_g_at(s, s->nstep);
    a.force_cos = s->d_ftab;
    a.force_axis = s->f_axis;
    hipError_t e = s->ks->moments(a, d, d + n, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(rho, d, sizeof(double) * n, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(u, d + n, sizeof(double) * n * D, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d);
    HIP_TRY(e);
    return LBM_OK;
}

lbm_status lbm_shear_amplitude(lbm_sim *s, int32_t wave_axis, double *a_sin, double *a_cos) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    lbm_status st = check_axis(s, wave_axis);
    if (st != LBM_OK) return st;
    double r[6];
    st = run_diag(s, wave_axis, r);
    if (st != LBM_OK) return st;
    const double scale = 2.0 / (double)s->ncell;
    if (a_sin) *a_sin = scale * r[0];
    if (a_cos) *a_cos = scale * r[1];
    return LBM_OK;
}

lbm_status lbm_shear_amplitude_noalloc(lbm_sim *s, int32_t wave_axis, double *dev_out) {
    if (!s || !dev_out) return fail(LBM_EINVAL, "NULL argument");
    lbm_status st = check_axis(s, wave_axis);
    if (st != LBM_OK) return st;
    if (6u * s->diag_blocks > kNoAllocFinal)
        return fail(LBM_EINVAL, "reduction of %u workgroups exceeds the scratch of %u workgroups", s->diag_blocks,
                    kNoAllocFinal / 6u);
    double *scr = nullptr;
    const hipError_t e = noalloc_scratch(s->device, &scr);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "device scratch unavailable on device %d: %s", s->device, hipGetErrorString(e));
    const DiagArgs a = diag_args(s, wave_axis, scr);
    HIP_TRY(s->ks->diag(a, s->diag_blocks, s->stream));
    HIP_TRY(diag_final(scr, s->diag_blocks, 6, scr + kNoAllocFinal, s->stream));
    HIP_TRY(noalloc_scale2(scr + kNoAllocFinal, 2.0 / (double)s->ncell, dev_out, s->stream));
    return LBM_OK;
}

lbm_status lbm_totals(lbm_sim *s, double *mass, double *mom) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    double r[6];
    lbm_status st = run_diag(s, 1, r);
    if (st != LBM_OK) return st;
    if (mass) *mass = (is_dev(s->o.storage) ? (double)s->ncell : 0.0) + r[2];
    if (mom)
        for (int d = 0; d < s->L->D; ++d) mom[d] = r[3 + d];
    return LBM_OK;
}

lbm_status lbm_get_populations(lbm_sim *s, double *f) {
    if (!s || !f) return fail(LBM_EINVAL, "NULL argument");
    const size_t n = s->ncell;
    double *d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(double) * n));
    hipError_t e = hipSuccess;
    for (int a = 0; a < s->L->Q && e == hipSuccess; ++a) {
        const double add = is_dev(s->o.storage) ? s->L->w[a] : 0.0;
        const double mul = is_scaled(s->o.storage) ? s->L->w[a] : 1.0;
        e = s->ks->decode(s->buf[s->cur], s->lay, (uint32_t)n, a, add, mul, d, s->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(f + (size_t)a * n, d, sizeof(double) * n, hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    }
    (void)hipFree(d);
    HIP_TRY(e);
    return LBM_OK;
}

lbm_status lbm_get_cells(lbm_sim *s, const int64_t *cells, int64_t count, double *f) {
    if (!s || (count > 0 && (!cells || !f))) return fail(LBM_EINVAL, "NULL argument");
    if (count < 0 || count > (int64_t)(0x7fffffff / kMaxQ)) return fail(LBM_EINVAL, "count out of range");
    if (count == 0) return LBM_OK;
    std::vector<uint32_t> idx((size_t)count);
    for (int64_t k = 0; k < count; ++k) {
        if (cells[k] < 0 || cells[k] >= (int64_t)s->ncell)
            return fail(LBM_EINVAL, "cell %lld out of range [0, %zu)", (long long)cells[k], s->ncell);
        idx[(size_t)k] = (uint32_t)cells[k];
    }
    GatherArgs g{};
    g.f = s->buf[s->cur];
    g.lay = s->lay;
    g.count = (uint32_t)count;
    g.Q = s->L->Q;
    for (int a = 0; a < s->L->Q; ++a) {
        g.add[a] = is_dev(s->o.storage) ? s->L->w[a] : 0.0;
        g.mul[a] = is_scaled(s->o.storage) ? s->L->w[a] : 1.0;
    }
    const size_t nout = (size_t)count * (size_t)s->L->Q;
    void *d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(uint32_t) * (size_t)count + sizeof(double) * nout + 8));
    g.cells = static_cast<const uint32_t *>(d);
    g.out = reinterpret_cast<double *>(static_cast<char *>(d) + ((sizeof(uint32_t) * (size_t)count + 7) & ~(size_t)7));
    hipError_t e = hipMemcpyAsync(d, idx.data(), sizeof(uint32_t) * (size_t)count, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = s->ks->gather(g, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f, g.out, sizeof(double) * nout, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d);
    HIP_TRY(e);
    return LBM_OK;
}

lbm_status lbm_set_populations(lbm_sim *s, const double *f) {
    if (!s || !f) return fail(LBM_EINVAL, "NULL argument");
    const size_t n = s->ncell;
    double *d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(double) * n));
    hipError_t e = hipSuccess;
    const uint32_t key = (uint32_t)splitmix64(s->o.sr_seed ^ 0xC0FFEEull);
    for (int a = 0; a < s->L->Q && e == hipSuccess; ++a) {
        const double add = is_dev(s->o.storage) ? s->L->w[a] : 0.0;
        const double scale = is_scaled(s->o.storage) ? 1.0 / s->L->w[a] : 1.0;
        e = hipMemcpyAsync(d, f + (size_t)a * n, sizeof(double) * n, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = s->ks->encode(s->buf[s->cur], s->lay, (uint32_t)n, a, add, scale, d, key, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    }
    (void)hipFree(d);
    s->stress_valid = false;
    HIP_TRY(e);
    return LBM_OK;
}

lbm_status lbm_set_step_count(lbm_sim *s, int64_t n) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (n < 0) return fail(LBM_EINVAL, "step count must be >= 0");
    s->nstep = n;
    return LBM_OK;
}

lbm_status lbm_state_bytes(const lbm_sim *s, int64_t *bytes) {
    if (!s || !bytes) return fail(LBM_EINVAL, "NULL argument");
    *bytes = (int64_t)s->L->Q * (int64_t)s->ncell * s->esize;
    return LBM_OK;
}

lbm_status lbm_save_state(lbm_sim *s, void *host, int64_t bytes) {
    int64_t need = 0;
    lbm_status st = lbm_state_bytes(s, &need);
    if (st != LBM_OK) return st;
    if (!host || bytes != need) return fail(LBM_EINVAL, "state needs exactly %lld bytes", (long long)need);
    HIP_TRY(hipMemcpyAsync(host, s->buf[s->cur], (size_t)need, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return LBM_OK;
}

lbm_status lbm_load_state(lbm_sim *s, const void *host, int64_t bytes) {
    int64_t need = 0;
    lbm_status st = lbm_state_bytes(s, &need);
    if (st != LBM_OK) return st;
    if (!host || bytes != need) return fail(LBM_EINVAL, "state needs exactly %lld bytes", (long long)need);
    s->stress_valid = false;
    HIP_TRY(hipMemcpyAsync(s->buf[s->cur], host, (size_t)need, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return LBM_OK;
}

lbm_status lbm_device_copy(void *dst, const void *src, int64_t bytes, int32_t blocks, void *hip_stream) {
    if (!dst || !src || bytes < 0) return fail(LBM_EINVAL, "NULL pointer or negative size");
    if ((((uintptr_t)dst | (uintptr_t)src | (uintptr_t)bytes) & 15u) != 0)
        return fail(LBM_EINVAL, "pointers and size must be multiples of 16 bytes");
    if (blocks < 1) return fail(LBM_EINVAL, "blocks must be >= 1");
    const uintptr_t d = (uintptr_t)dst, sp = (uintptr_t)src;
    if (bytes > 0 && (d < sp ? sp - d : d - sp) < (uint64_t)bytes) return fail(LBM_EINVAL, "buffers overlap");
    if (bytes == 0) return LBM_OK;
    HIP_TRY(copy16(src, dst, (uint64_t)bytes / 16u, (uint32_t)blocks, (hipStream_t)hip_stream));
    return LBM_OK;
}

lbm_status lbm_fit_decay(const double *amp, const int64_t *steps, int64_t count, int64_t n_first, int64_t n_last,
                         double *gamma) {
    if (!amp || !steps || !gamma || count < 0) return fail(LBM_EINVAL, "NULL argument or negative count");
    double st = 0, sy = 0;
    int64_t m = 0;
    for (int64_t k = 0; k < count; ++k)
        if (steps[k] >= n_first && steps[k] <= n_last) {
            if (!(amp[k] != 0.0) || !isfinite(amp[k])) return fail(LBM_EINVAL, "amplitude %lld is zero or non-finite", (long long)k);
            st += (double)steps[k];
            sy += -log(fabs(amp[k]));
            ++m;
        }
    if (m < 2) return fail(LBM_EINVAL, "fewer than two points in the fit window");
    const double tm = st / (double)m, ym = sy / (double)m;
    double sxy = 0, sxx = 0;
    for (int64_t k = 0; k < count; ++k)
        if (steps[k] >= n_first && steps[k] <= n_last) {
            const double dt = (double)steps[k] - tm;
            sxy += dt * (-log(fabs(amp[k])) - ym);
            sxx += dt * dt;
        }
    if (!(sxx > 0.0)) return fail(LBM_EINVAL, "fit window has a single distinct step");
    *gamma = sxy / sxx;
    return LBM_OK;
}

lbm_status lbm_fit_oscillation(const double *amp, const int64_t *steps, int64_t count, double dt, double frequency,
                               int64_t n_first, int64_t n_last, double *re, double *im) {
    if (!amp || !steps || !re || !im || count < 0) return fail(LBM_EINVAL, "NULL argument or negative count");
    if (!(dt > 0.0) || !isfinite(frequency)) return fail(LBM_EINVAL, "dt must be > 0 and frequency finite");
    // least squares for amp(n) = a cos(w t) + b sin(w t), t = n dt; z = a - i b
    double scc = 0, sss = 0, scs = 0, sac = 0, sas = 0, sa = 0;
    int64_t m = 0;
    for (int64_t k = 0; k < count; ++k)
        if (steps[k] >= n_first && steps[k] <= n_last) {
            if (!isfinite(amp[k])) return fail(LBM_EINVAL, "amplitude %lld is not finite", (long long)k);
            const double ph = frequency * (double)steps[k] * dt, c = cos(ph), sn = sin(ph);
            scc += c * c;
            sss += sn * sn;
            scs += c * sn;
            sac += amp[k] * c;
            sas += amp[k] * sn;
            sa += amp[k];
            ++m;
        }
    if (m < 1) return fail(LBM_EINVAL, "no point in the fit window");
    if (frequency == 0.0) {
        *re = sa / (double)m;
        *im = 0.0;
        return LBM_OK;
    }
    const double det = scc * sss - scs * scs;
    if (!(fabs(det) > 1e-12 * scc * sss)) return fail(LBM_EINVAL, "fit window does not resolve the oscillation");
    const double a = (sac * sss - sas * scs) / det, b = (sas * scc - sac * scs) / det;
    *re = a;
    *im = -b;
    return LBM_OK;
}

lbm_status lbm_set_force(lbm_sim *s, double amplitude, double frequency, int32_t wave_axis) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (wave_axis == 0) {                       // back to the unforced kernels
        s->forced = false;
        s->stress_valid = false;
        return LBM_OK;
    }
    lbm_status st = check_axis(s, wave_axis);
    if (st != LBM_OK) return st;
    if (s->move == LBM_MOVE_BW2 && wave_axis != 1) return fail(LBM_EINVAL, "upwind advection is two-dimensional");
    if (!isfinite(amplitude) || !isfinite(frequency)) return fail(LBM_EINVAL, "amplitude and frequency must be finite");
    const int nw = wave_axis == 1 ? s->g.ny : s->g.nz;
    const double dt = lbm_time_step((lbm_lattice)s->L->id, s->move, nw, s->o.cfl);
    if (!(dt > 0.0)) return fail(LBM_EINVAL, "no time step for this configuration");
    std::vector<double> h(2 * (size_t)nw);
    for (int j = 0; j < nw; ++j) {
        const double ph = 2.0 * M_PI * (double)j / (double)nw;
        h[j] = cos(ph);
        h[nw + j] = sin(ph);
    }
    // stress slots: the largest grid of the forced kernels (256 threads) over the tiles
    const bool was = s->forced;
    s->forced = true;
    uint32_t cap = 0;
    for (int t = 0; t < tile_count(s); ++t) cap = std::max(cap, stress_slots(s, t));
    s->forced = was;
    double *tab = nullptr, *stress = nullptr;
    hipError_t e = hipMalloc(&tab, sizeof(double) * h.size());
    if (e == hipSuccess) e = hipMalloc(&stress, sizeof(double) * 2 * (size_t)cap);
    if (e == hipSuccess) e = hipMemcpyAsync(tab, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        if (tab) (void)hipFree(tab);
        if (stress) (void)hipFree(stress);
        HIP_TRY(e);
    }
    if (s->d_ftab) (void)hipFree(s->d_ftab);
    if (s->d_stress) (void)hipFree(s->d_stress);
    s->d_ftab = tab;
    s->d_stress = stress;
    s->stress_cap = cap;
    s->forced = true;
    s->f_amp = amplitude;
    s->f_freq = frequency;
    s->f_dt = dt;
    s->f_axis = wave_axis;
    s->stress_valid = false;
    s->tile = std::min(s->tile, tile_count(s) - 1);
    return LBM_OK;
}

lbm_status lbm_shear_stress_amplitude(lbm_sim *s, double *s_sin, double *s_cos) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (!s->forced || !s->stress_valid)
        return fail(LBM_ESTATE, "no forced step since the force or the state was set");
    HIP_TRY(diag_final(s->d_stress, s->stress_slots, 2, s->d_result, s->stream));
    double r[2];
    HIP_TRY(hipMemcpyAsync(r, s->d_result, 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const double scale = 2.0 / (double)s->ncell;
    if (s_sin) *s_sin = scale * r[0];
    if (s_cos) *s_cos = scale * r[1];
    return LBM_OK;
}

int32_t lbm_tile_count(const lbm_sim *s) { return s ? tile_count(s) : 0; }

lbm_status lbm_set_tile(lbm_sim *s, int32_t tile) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (tile < 0 || tile >= tile_count(s)) return fail(LBM_EINVAL, "tile %d out of range [0, %d)", tile, tile_count(s));
    s->tile = tile;
    return LBM_OK;
}

lbm_status lbm_tile_info(const lbm_sim *s, int32_t tile, int32_t *block_threads, int32_t *cells_per_thread,
                         int32_t *vector_width, int64_t *blocks, int32_t *nontemporal) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (tile < 0 || tile >= tile_count(s)) return fail(LBM_EINVAL, "tile %d out of range [0, %d)", tile, tile_count(s));
    const host::StepShape h = step_shape(s);
    int blk = 0, cpt = 0, vw = 0;
    bool nt = false;
    host::tile_launch(h, tile, &blk, &cpt, &vw, &nt);
    if (block_threads) *block_threads = blk;
    if (cells_per_thread) *cells_per_thread = cpt;
    if (vector_width) *vector_width = vw;
    if (blocks) *blocks = (int64_t)host::step_geometry(h, tile).nblocks;
    if (nontemporal) *nontemporal = nt ? 1 : 0;
    return LBM_OK;
}

lbm_status lbm_autotune(lbm_sim *s, int32_t steps_per_trial, int32_t *best_tile, double *best_ms) {
    if (!s) return fail(LBM_EINVAL, "sim is NULL");
    if (steps_per_trial < 1) return fail(LBM_EINVAL, "steps_per_trial must be >= 1");
    const size_t bytes = (size_t)s->L->Q * s->ncell * (size_t)s->esize;
    void *scratch[2] = {nullptr, nullptr};
    HIP_TRY(hipMalloc(&scratch[0], bytes));
    hipError_t e = hipMalloc(&scratch[1], bytes);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMemcpyAsync(scratch[0], s->buf[s->cur], bytes, hipMemcpyDeviceToDevice, s->stream);
    int best = s->tile;
    float best_t = 1e30f;
    const int64_t saved_step = s->nstep;
    for (int t = 0; t < tile_count(s) && e == hipSuccess; ++t) {
        int c = 0;
        e = launch_step(s, scratch[c], scratch[c ^ 1], t, false);   // warm-up
        c ^= 1;
        if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
        for (int k = 0; k < steps_per_trial && e == hipSuccess; ++k) {
            e = launch_step(s, scratch[c], scratch[c ^ 1], t, false);
            c ^= 1;
        }
        if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms < best_t) {
            best_t = ms;
            best = t;
        }
    }
    s->nstep = saved_step;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(scratch[0]);
    if (scratch[1]) (void)hipFree(scratch[1]);
    HIP_TRY(e);
    s->tile = best;
    if (best_tile) *best_tile = best;
    if (best_ms) *best_ms = (double)best_t / steps_per_trial;
    return LBM_OK;
}

lbm_status lbm_autotune_cached(lbm_sim *s, const char *path, int32_t steps_per_trial, int32_t *best_tile,
                               double *best_ms, int32_t *hit) {
    if (!s || !path || !*path) return fail(LBM_EINVAL, "sim or path is NULL");
    if (steps_per_trial < 1) return fail(LBM_EINVAL, "steps_per_trial must be >= 1");
    hipDeviceProp_t prop{};
    HIP_TRY(hipGetDeviceProperties(&prop, s->device));
    const host::StepShape h = step_shape(s);
    const std::string key = host::tune_key(prop.gcnArchName, s->L->id, s->N, (int)s->o.storage, s->ks->sr, h);
    host::TuneEntry e;
    if (host::tune_lookup(path, key, &e) && e.tile >= 0 && e.tile < tile_count(s) && e.shape == host::tile_shape(h, e.tile)) {
        s->tile = e.tile;
        if (best_tile) *best_tile = e.tile;
        if (best_ms) *best_ms = e.ms;
        if (hit) *hit = 1;
        return LBM_OK;
    }
    int32_t t = 0;
    double ms = 0;
    const lbm_status st = lbm_autotune(s, steps_per_trial, &t, &ms);
    if (st != LBM_OK) return st;
    if (best_tile) *best_tile = t;
    if (best_ms) *best_ms = ms;
    if (hit) *hit = 0;
    e.key = key;
    e.tile = t;
    e.shape = host::tile_shape(h, t);
    e.ms = ms;
    std::string err;
    if (!host::tune_store(path, e, &err)) return fail(LBM_EINVAL, "autotuner cache: %s", err.c_str());
    return LBM_OK;
}

}  // extern "C"

// ======================================================================== batches
struct lbm_batch {
    int count = 0;
    lbm_storage storage = LBM_FP32_DEV;
    double cfl = 0.5;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<lbm_instance> inst;
    std::vector<BatchInst> desc;            // host copy of the descriptors
    std::vector<const KernelSet *> ks;
    std::vector<int32_t> cur;               // buffer holding each instance's state
    BatchInst *d_inst = nullptr;
    int32_t *d_order = nullptr;
    int32_t *d_cur = nullptr;
    void *pool = nullptr;
    size_t pool_bytes = 0;
    double *d_sin = nullptr;
    double *d_bw = nullptr;
    float *d_bwf = nullptr;
    double *d_amp = nullptr;
    size_t amp_cap = 0;                     // doubles allocated in d_amp
    int form = 0;                           // 0: workgroup per instance, 1: chunks + grid barrier,
                                            // 2: chunks + barrier per XCD
    int block = 512;
    int64_t cells = 0, bytes_per_step = 0;
    // grid-form plan (for plan_block, plan_form; host copy in plan)
    int plan_block = 0, plan_form = 0;
    host::BatchPlan plan;
    std::vector<int> kind;                  // per instance: index of its velocity set among those present
    int nkinds = 0;
    // chunk costs fitted by the autotuner per (form, block): per-cell cost of each kind, then the
    // per-chunk cost (absent: the default model)
    std::map<std::pair<int, int>, std::vector<double>> cal;
    uint32_t nchunks = 0, nwg = 0;
    int nxcd = 0;                           // XCDs seen by the probe (0: not probed, -1: form 2 unusable)
    int xcd_force = 0;                      // plan form 2 for this many XCDs instead (testing; 0 = probe)
    uint32_t wg_per_xcd = 0;
    uint32_t *d_sync = nullptr;
    BatchChunk *d_chunks = nullptr;
    uint32_t *d_inst_first = nullptr, *d_wg_first = nullptr, *d_wg_chunks = nullptr;
    uint64_t *d_barrier = nullptr;
    int32_t *d_abort = nullptr;
    uint32_t spin_limit = kSpinLimit;       // bound of a barrier wait (sleeps)
    bool poisoned = false;                  // a barrier wait expired: state undefined until reset
    double *d_partials = nullptr;
    size_t partials_cap = 0;
    // cached graph of one run configuration
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int64_t g_steps = -1;
    int g_record = -1, g_block = -1, g_first = -1, g_form = -1;
};

namespace {

void batch_drop_graph(lbm_batch *b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->g_steps = -1;
}

lbm_status batch_init_states(lbm_batch *b) {
    for (int i = 0; i < b->count; ++i) {
        const BatchInst &d = b->desc[i];
        WaveArgs a{};
        a.f = static_cast<char *>(b->pool) + d.off * (size_t)elem_size(b->storage);
        a.nx = d.nx;
        a.ny = d.ny;
        a.nz = 1;
        a.lay = Layout{(uint32_t)d.nx, d.pstride, (uint64_t)d.nx};   // one plane per population
        a.wave_axis = 1;
        a.u0 = b->inst[i].u0;
        a.rho_noise = 0.0;
        a.seed = 0;
        a.sin_tab = b->d_sin + d.sin_off;
        HIP_TRY(b->ks[i]->init_wave(a, b->stream));
    }
    std::fill(b->cur.begin(), b->cur.end(), 0);
    HIP_TRY(hipStreamSynchronize(b->stream));
    return LBM_OK;
}

template <class P>
lbm_status realloc_dev(P **p, size_t bytes) {
    if (*p) HIP_TRY(hipFree(*p));
    *p = nullptr;
    HIP_TRY(hipMalloc((void **)p, bytes));
    return LBM_OK;
}

// Number of XCDs, from the XCD ids of a probe launch of n workgroups (the grid size of the
// XCD-local form); -1 if the workgroups were not spread evenly over them.
lbm_status batch_probe_xcd(lbm_batch *b, uint32_t n) {
    uint32_t *d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(uint32_t) * n));
    std::vector<uint32_t> h(n);
    hipError_t e = probe_xcd(d, n, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(d);
    HIP_TRY(e);
    uint32_t nx = 0;
    for (uint32_t v : h) nx = std::max(nx, v + 1);
    std::vector<uint32_t> per(nx, 0);
    for (uint32_t v : h) ++per[v];
    bool even = nx >= 1 && nx <= kMaxXcd;
    for (uint32_t c : per) even = even && c == per[0];
    b->nxcd = even ? (int)nx : -1;
    return LBM_OK;
}

// Chunks of `block` cells per instance.  Form 1: chunks spread over the resident grid, each
// chunk (largest cost first) onto the least-loaded workgroup.  Form 2: instances (largest
// first) onto the least-loaded XCD, then each XCD's chunks over its share of the grid.
lbm_status batch_plan(lbm_batch *b, int block, int form) {
    if (b->plan_block == block && b->plan_form == form) return LBM_OK;
    int dev = 0, ncu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int per_cu = batch_grid_resident_per_cu((int)b->storage, form, block);
    if (per_cu < 1 || ncu < 1) return fail(LBM_EDEVICE, "grid form cannot be resident with %d threads", block);
    const uint32_t resident = (uint32_t)(per_cu * ncu);
    lbm_status st;
    if (form == 2) {
        if (b->nxcd == 0 && (st = batch_probe_xcd(b, resident)) != LBM_OK) return st;
        if (b->nxcd < 1) return fail(LBM_EDEVICE, "workgroups are not spread evenly over XCDs: XCD-local form unusable");
        const uint32_t nx = (uint32_t)(b->xcd_force > 0 ? b->xcd_force : b->nxcd);
        if (resident < nx) return fail(LBM_EDEVICE, "XCD-local form needs a resident workgroup per XCD");
    }
    std::vector<uint32_t> ncell(b->count);
    std::vector<double> per_cell(b->count);
    double per_chunk = 0.0;
    const auto c = b->cal.find({form, block});
    for (int i = 0; i < b->count; ++i) {
        const LatInfo *L = lat_info(b->desc[i].lattice);
        ncell[i] = b->desc[i].ncell;
        per_cell[i] = c != b->cal.end() ? c->second[b->kind[i]] : host::batch_cell_cost(L->on_lattice, L->Q);
    }
    if (c != b->cal.end()) per_chunk = c->second[b->nkinds];
    const uint32_t nx = form == 2 ? (uint32_t)(b->xcd_force > 0 ? b->xcd_force : b->nxcd) : 1u;
    b->plan = host::plan_batch(ncell, per_cell, per_chunk, (uint32_t)block, form, resident, nx);
    const host::BatchPlan &plan = b->plan;
    const uint32_t nchunks = (uint32_t)plan.chunks.size(), nwg = plan.nwg, per_xcd = plan.per_xcd;
    std::vector<BatchChunk> chunks(nchunks);
    for (uint32_t k = 0; k < nchunks; ++k)
        chunks[k] = BatchChunk{plan.chunks[k].inst, plan.chunks[k].start, plan.chunks[k].count};
    const std::vector<uint32_t> &inst_first = plan.inst_first, &wg_first = plan.wg_first, &wg_chunks = plan.wg_chunks;
    if ((st = realloc_dev(&b->d_chunks, sizeof(BatchChunk) * nchunks)) != LBM_OK) return st;
    if ((st = realloc_dev(&b->d_inst_first, sizeof(uint32_t) * inst_first.size())) != LBM_OK) return st;
    if ((st = realloc_dev(&b->d_wg_first, sizeof(uint32_t) * wg_first.size())) != LBM_OK) return st;
    if ((st = realloc_dev(&b->d_wg_chunks, sizeof(uint32_t) * wg_chunks.size())) != LBM_OK) return st;
    HIP_TRY(hipMemcpyAsync(b->d_chunks, chunks.data(), sizeof(BatchChunk) * nchunks, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_inst_first, inst_first.data(), sizeof(uint32_t) * inst_first.size(), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_wg_first, wg_first.data(), sizeof(uint32_t) * wg_first.size(), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_wg_chunks, wg_chunks.data(), sizeof(uint32_t) * wg_chunks.size(), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->nchunks = nchunks;
    b->nwg = nwg;
    b->wg_per_xcd = per_xcd;
    b->plan_block = block;
    b->plan_form = form;
    b->partials_cap = 0;
    batch_drop_graph(b);
    return LBM_OK;
}

lbm_status batch_ensure_logs(lbm_batch *b, size_t per) {
    const size_t n_amp = per * (size_t)b->count;
    if (n_amp > b->amp_cap) {
        lbm_status st = realloc_dev(&b->d_amp, sizeof(double) * n_amp);
        if (st != LBM_OK) return st;
        b->amp_cap = n_amp;
        batch_drop_graph(b);
    }
    if (b->form >= 1) {
        const size_t n_part = per * (size_t)b->nchunks;
        if (n_part > b->partials_cap) {
            lbm_status st = realloc_dev(&b->d_partials, sizeof(double) * n_part);
            if (st != LBM_OK) return st;
            b->partials_cap = n_part;
            batch_drop_graph(b);
        }
    }
    return LBM_OK;
}

BatchArgs batch_args(const lbm_batch *b, int64_t steps, int32_t record, int32_t first, uint32_t nrec) {
    BatchArgs a{};
    a.inst = b->d_inst;
    a.order = b->d_order;
    a.pool = b->pool;
    a.sin_tab = b->d_sin;
    a.bw = b->d_bw;
    a.bwf = b->d_bwf;
    a.amp = b->d_amp;
    a.cur = b->d_cur;
    a.steps = steps;
    a.record = record;
    a.record_first = first;
    a.chunks = b->d_chunks;
    a.inst_first = b->d_inst_first;
    a.wg_first = b->d_wg_first;
    a.wg_chunks = b->d_wg_chunks;
    a.nwg = b->nwg;
    a.nrec = nrec;
    a.barrier = b->d_barrier;
    a.abort = b->d_abort;
    a.spin_limit = b->spin_limit;
    a.partials = b->d_partials;
    a.sync = b->form == 2 ? b->d_sync : nullptr;
    a.nxcd = b->nxcd > 0 ? (uint32_t)(b->xcd_force > 0 ? b->xcd_force : b->nxcd) : 0u;
    a.wg_per_xcd = b->wg_per_xcd;
    return a;
}

// The abort flag of the last grid-form launch: 0 ok, 1 a barrier wait expired, 2 the XCD
// placement differed from the plan (nothing was stepped).
lbm_status batch_abort_flag(lbm_batch *b, int32_t *ab) {
    *ab = 0;
    if (b->form == 0) return LBM_OK;
    HIP_TRY(hipMemcpyAsync(ab, b->d_abort, sizeof(int32_t), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return LBM_OK;
}

// One step-profile launch of the current plan (form b->form, workgroup size b->block): steps
// steps from the state on the device, timestamps of steps first .. first + count - 1 into ts
// (host, nwg * count * 3).  *ab receives the launch's abort flag.  Does not flip b->cur.
lbm_status batch_profile_launch(lbm_batch *b, int64_t steps, int64_t first, int32_t count, uint64_t *ts, int32_t *ab) {
    lbm_status st;
    if ((st = batch_ensure_logs(b, 1)) != LBM_OK) return st;
    for (int i = 0; i < b->count; ++i) b->desc[i].amp_off = (uint64_t)i;
    batch_drop_graph(b);
    const size_t n_ts = (size_t)b->nwg * (size_t)count * 3;
    uint64_t *d_ts = nullptr;
    HIP_TRY(hipMalloc(&d_ts, sizeof(uint64_t) * n_ts));
    BatchArgs a = batch_args(b, steps, 0, 0, 1);
    a.ts = d_ts;
    a.ts_first = first;
    a.ts_count = count;
    hipError_t e = hipMemcpyAsync(b->d_inst, b->desc.data(), sizeof(BatchInst) * b->count, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_cur, b->cur.data(), sizeof(int32_t) * b->count, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = launch_batch((int)b->storage, b->form, b->block, a, (uint32_t)b->count, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ts, d_ts, sizeof(uint64_t) * n_ts, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(d_ts);
    HIP_TRY(e);
    return batch_abort_flag(b, ab);
}

// Fit the chunk costs of the current (form, block) to a step profile of `steps` steps (the state
// is stepped; the caller restores it).  On success the fitted costs are stored in b->cal and the
// batch is planned with them; *ok = false leaves the plan as it was.
lbm_status batch_calibrate(lbm_batch *b, int64_t steps, bool *ok) {
    *ok = false;
    const int32_t count = (int32_t)std::min<int64_t>(64, steps);
    const int64_t first = (steps - count) / 2;
    std::vector<uint64_t> ts((size_t)b->nwg * (size_t)count * 3);
    int32_t ab = 0;
    lbm_status st = batch_profile_launch(b, steps, first, count, ts.data(), &ab);
    if (st != LBM_OK || ab) return st;
    // per workgroup: median over the profiled steps of start-to-chunks-done
    std::vector<double> work(b->nwg), tmp(count);
    for (uint32_t w = 0; w < b->nwg; ++w) {
        for (int32_t k = 0; k < count; ++k) {
            const uint64_t *t = &ts[((size_t)w * count + k) * 3];
            tmp[k] = (double)(t[1] - t[0]);
        }
        std::nth_element(tmp.begin(), tmp.begin() + count / 2, tmp.end());
        work[w] = tmp[count / 2];
    }
    const std::vector<double> coef = host::fit_chunk_costs(b->plan, b->kind, b->nkinds, work);
    bool any = false;
    for (int k = 0; k <= b->nkinds; ++k) any = any || coef[k] > 0;
    if (!any) return LBM_OK;   // nothing fitted: keep the default model
    b->cal[{b->form, b->block}] = coef;
    b->plan_block = 0;
    if ((st = batch_plan(b, b->block, b->form)) != LBM_OK) return st;
    *ok = true;
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_create(lbm_batch **out, const lbm_instance *inst, int32_t count, const lbm_opts *opts) {
    if (!out || !inst) return fail(LBM_EINVAL, "NULL argument");
    if (count < 1) return fail(LBM_EINVAL, "count must be >= 1");
    lbm_opts o;
    lbm_opts_default(&o);
    o.storage = LBM_FP32_DEV;
    if (opts) o = *opts;
    int32_t storage = 0;   // read as the int a C caller passed (it may be outside the enumeration)
    memcpy(&storage, &o.storage, sizeof storage);
    if (storage != LBM_FP32_DEV && storage != LBM_FP64) return fail(LBM_EINVAL, "batches store LBM_FP32_DEV or LBM_FP64");
    if (o.dev_buf[0] || o.dev_buf[1]) return fail(LBM_EINVAL, "batches allocate their own pool: dev_buf must be NULL");
    if (!(o.cfl > 0.0 && o.cfl <= 1.0)) return fail(LBM_EINVAL, "cfl must be in (0, 1]");
    for (int i = 0; i < count; ++i) {
        const lbm_instance &q = inst[i];
        const LatInfo *L = lat_info((int)q.lat);
        if (!L || !batch_supports((int)q.lat, q.eq_order, (int)o.storage))
            return fail(LBM_EINVAL, "instance %d: lattice %d / order %d not supported in a batch", i, (int)q.lat, q.eq_order);
        if (!(q.tau > 0.5)) return fail(LBM_EINVAL, "instance %d: tau must be > 1/2", i);
        if (q.g.nx < 1 || q.g.ny < 1 || q.g.nz != 1) return fail(LBM_EINVAL, "instance %d: grid must be nx, ny >= 1, nz = 1", i);
        if ((long long)q.g.nx * q.g.ny > (1ll << 26)) return fail(LBM_EINVAL, "instance %d: more than 2^26 cells", i);
        if (q.wave_axis != 1) return fail(LBM_EINVAL, "instance %d: wave_axis must be 1", i);
        if (!isfinite(q.u0)) return fail(LBM_EINVAL, "instance %d: u0 must be finite", i);
    }
    lbm_batch *b = new lbm_batch();
    b->count = count;
    b->storage = o.storage;
    b->cfl = o.cfl;
    b->inst.assign(inst, inst + count);
    b->desc.resize(count);
    b->ks.resize(count);
    b->cur.assign(count, 0);
    const int es = elem_size(o.storage);
    size_t off = 0, sin_off = 0;
    std::vector<double> sin_h, bw_h((size_t)count * 4 * kMaxQ, 0.0);
    for (int i = 0; i < count; ++i) {
        const lbm_instance &q = inst[i];
        const LatInfo *L = lat_info((int)q.lat);
        BatchInst &d = b->desc[i];
        d.lattice = L->id;
        d.order = q.eq_order;
        d.nx = q.g.nx;
        d.ny = q.g.ny;
        d.ncell = (uint32_t)(q.g.nx * q.g.ny);
        d.pstride = (d.ncell + 63) / 64 * 64;
        d.off = off;
        off += 2ull * L->Q * d.pstride;
        off = (off + 63) / 64 * 64;
        d.sin_off = (uint32_t)sin_off;
        for (int j = 0; j < q.g.ny; ++j) sin_h.push_back(sin(2.0 * M_PI * (double)j / (double)q.g.ny));
        sin_off += (size_t)q.g.ny;
        d.bw_off = (uint32_t)((size_t)i * 4 * kMaxQ);
        if (!L->on_lattice) {
            const double lam = o.cfl / L->xi_max;
            for (int a = 0; a < L->Q; ++a)
                for (int ax = 0; ax < 2; ++ax) {
                    const double A = fabs(L->xi[a][ax] * lam), bb = 0.5 * A * (1.0 - A);
                    bw_h[d.bw_off + (2 * ax + 0) * kMaxQ + a] = A + bb;
                    bw_h[d.bw_off + (2 * ax + 1) * kMaxQ + a] = bb;
                }
        }
        d.omega = isinf(q.tau) ? 0.0 : 1.0 / q.tau;
        d.amp_off = 0;
        b->ks[i] = find_kernels(L->id, q.eq_order, (int)o.storage, 0);
        b->cells += d.ncell;
        b->bytes_per_step += 2ll * L->Q * d.ncell * es;
    }
    // kinds for the fitted cost model: the distinct velocity sets, in order of appearance
    std::vector<int> kind_lat;
    b->kind.resize(count);
    for (int i = 0; i < count; ++i) {
        const int id = b->desc[i].lattice;
        auto it = std::find(kind_lat.begin(), kind_lat.end(), id);
        if (it == kind_lat.end()) it = kind_lat.insert(kind_lat.end(), id);
        b->kind[i] = (int)(it - kind_lat.begin());
    }
    b->nkinds = (int)kind_lat.size();
    // per-instance form: workgroups take instances largest first (cost ~ Q * cells)
    std::vector<int32_t> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return (long long)lat_info(b->desc[x].lattice)->Q * b->desc[x].ncell >
               (long long)lat_info(b->desc[y].lattice)->Q * b->desc[y].ncell;
    });
    b->pool_bytes = off * (size_t)es;
    hipError_t e = hipSuccess;
    if (o.hip_stream) {
        b->stream = (hipStream_t)o.hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        b->own_stream = e == hipSuccess;
    }
    if (e == hipSuccess) e = hipMalloc(&b->pool, b->pool_bytes);
    if (e == hipSuccess) e = hipMalloc(&b->d_inst, sizeof(BatchInst) * count);
    if (e == hipSuccess) e = hipMalloc(&b->d_order, sizeof(int32_t) * count);
    if (e == hipSuccess) e = hipMalloc(&b->d_cur, sizeof(int32_t) * count);
    if (e == hipSuccess) e = hipMalloc(&b->d_sin, sizeof(double) * sin_h.size());
    if (e == hipSuccess) e = hipMalloc(&b->d_bw, sizeof(double) * bw_h.size());
    if (e == hipSuccess) e = hipMalloc(&b->d_bwf, sizeof(float) * bw_h.size());
    if (e == hipSuccess) e = hipMalloc(&b->d_barrier, sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc(&b->d_abort, sizeof(int32_t) * 2);
    if (e == hipSuccess) e = hipMalloc(&b->d_sync, sizeof(uint32_t) * kSyncWords);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_sin, sin_h.data(), sizeof(double) * sin_h.size(), hipMemcpyHostToDevice, b->stream);
    std::vector<float> bwf_h(bw_h.size(), 0.0f);   // per population alpha_x, beta_x, alpha_y, beta_y
    for (int i = 0; i < count; ++i)
        for (int a = 0; a < kMaxQ; ++a)
            for (int k = 0; k < 4; ++k)
                bwf_h[b->desc[i].bw_off + 4 * a + k] = (float)bw_h[b->desc[i].bw_off + k * kMaxQ + a];
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_bw, bw_h.data(), sizeof(double) * bw_h.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_bwf, bwf_h.data(), sizeof(float) * bwf_h.size(), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_order, order.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->pool, 0, b->pool_bytes, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        lbm_status st = fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "batch allocation: %s", hipGetErrorString(e));
        lbm_batch_free(b);
        (void)hipGetLastError();
        return st;
    }
    lbm_status st = batch_init_states(b);
    if (st != LBM_OK) {
        lbm_batch_free(b);
        return st;
    }
    *out = b;
    return LBM_OK;
}

void lbm_batch_free(lbm_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    batch_drop_graph(b);
    for (void *p : {b->pool, (void *)b->d_inst, (void *)b->d_order, (void *)b->d_cur, (void *)b->d_sin,
                    (void *)b->d_bw, (void *)b->d_bwf, (void *)b->d_amp, (void *)b->d_chunks, (void *)b->d_inst_first,
                    (void *)b->d_wg_first, (void *)b->d_wg_chunks, (void *)b->d_barrier, (void *)b->d_abort,
                    (void *)b->d_partials, (void *)b->d_sync})
        if (p) (void)hipFree(p);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

lbm_status lbm_batch_reset(lbm_batch *b) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    lbm_status st = batch_init_states(b);
    if (st == LBM_OK) b->poisoned = false;
    return st;
}

lbm_status lbm_batch_set_spin_limit(lbm_batch *b, uint32_t limit) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    b->spin_limit = limit == 0 ? kSpinLimit : std::min(limit, kSpinLimit);
    batch_drop_graph(b);
    return LBM_OK;
}

lbm_status lbm_batch_sizes(const lbm_batch *b, int64_t *cells, int64_t *bytes_per_step) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (cells) *cells = b->cells;
    if (bytes_per_step) *bytes_per_step = b->bytes_per_step;
    return LBM_OK;
}

lbm_status lbm_batch_run(lbm_batch *b, int64_t steps, int32_t record_every, double *amp) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (b->poisoned) return fail(LBM_ESTATE, "a barrier wait expired in an earlier run: call lbm_batch_reset");
    if (steps < 0 || record_every < 1) return fail(LBM_EINVAL, "steps >= 0 and record_every >= 1 required");
    const int64_t per = amp ? steps / record_every + 1 : 1;
    if (per * (int64_t)b->count > (1ll << 31)) return fail(LBM_EINVAL, "amplitude log too large");
    const int32_t rec = amp ? record_every : 0, first = amp ? 1 : 0;
    lbm_status st;
    if (b->form >= 1 && (st = batch_plan(b, b->block, b->form)) != LBM_OK) return st;
    if ((st = batch_ensure_logs(b, (size_t)per)) != LBM_OK) return st;
    bool changed = false;
    for (int i = 0; i < b->count; ++i) {
        const uint64_t ao = (uint64_t)i * (uint64_t)per;
        if (b->desc[i].amp_off != ao) changed = true;
        b->desc[i].amp_off = ao;
    }
    if (changed) batch_drop_graph(b);
    HIP_TRY(hipMemcpyAsync(b->d_inst, b->desc.data(), sizeof(BatchInst) * b->count, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_cur, b->cur.data(), sizeof(int32_t) * b->count, hipMemcpyHostToDevice, b->stream));
    if (!(b->gexec && b->g_steps == steps && b->g_record == rec && b->g_block == b->block && b->g_first == first &&
          b->g_form == b->form)) {
        batch_drop_graph(b);
        HIP_TRY(hipStreamSynchronize(b->stream));
        HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = launch_batch((int)b->storage, b->form, b->block, batch_args(b, steps, rec, first, (uint32_t)per),
                                    (uint32_t)b->count, b->stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->stream, &g);
        HIP_TRY(e);
        HIP_TRY(e2);
        b->graph = g;
        HIP_TRY(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
        b->g_steps = steps;
        b->g_record = rec;
        b->g_block = b->block;
        b->g_first = first;
        b->g_form = b->form;
    }
    HIP_TRY(hipGraphLaunch(b->gexec, b->stream));
    if (amp) HIP_TRY(hipMemcpyAsync(amp, b->d_amp, sizeof(double) * per * b->count, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    int32_t ab = 0;
    if ((st = batch_abort_flag(b, &ab)) != LBM_OK) return st;
    if (ab == 2) {
        // the workgroups did not land on the XCDs as planned and left before stepping:
        // run again in the device-wide form and keep it
        b->nxcd = -1;
        if ((st = lbm_batch_set_form(b, 1, b->block)) != LBM_OK) return st;
        return lbm_batch_run(b, steps, record_every, amp);
    }
    if (ab) {
        // the workgroups left the step loop at different steps: the instances are partly stepped
        b->poisoned = true;
        return fail(LBM_EDEVICE, "batch grid barrier timed out: workgroups were not resident together; "
                                 "the state is undefined until lbm_batch_reset");
    }
    if (steps & 1)
        for (auto &c : b->cur) c ^= 1;
    return LBM_OK;
}

lbm_status lbm_batch_profile(lbm_batch *b, int64_t steps, int64_t first, int32_t count, int32_t *nwg, uint64_t *ts) {
    if (!b || !nwg) return fail(LBM_EINVAL, "NULL argument");
    if (b->poisoned) return fail(LBM_ESTATE, "a barrier wait expired in an earlier run: call lbm_batch_reset");
    if (b->form == 0) return fail(LBM_EINVAL, "the step profile covers the grid forms (1 and 2) only");
    if (steps < 1 || first < 0 || count < 1 || first + (int64_t)count > steps)
        return fail(LBM_EINVAL, "need 0 <= first, 1 <= count, first + count <= steps");
    lbm_status st;
    if ((st = batch_plan(b, b->block, b->form)) != LBM_OK) return st;
    *nwg = (int32_t)b->nwg;
    if (!ts) return LBM_OK;
    if ((size_t)b->nwg * (size_t)count * 3 > ((size_t)1 << 28)) return fail(LBM_EINVAL, "profile too large");
    int32_t ab = 0;
    if ((st = batch_profile_launch(b, steps, first, count, ts, &ab)) != LBM_OK) return st;
    if (ab == 2) {
        // nothing was stepped; later runs use the device-wide form
        b->nxcd = -1;
        if ((st = lbm_batch_set_form(b, 1, b->block)) != LBM_OK) return st;
        return fail(LBM_EDEVICE, "workgroups did not land on the XCDs as planned: batch switched to form 1");
    }
    if (ab) {
        b->poisoned = true;
        return fail(LBM_EDEVICE, "batch grid barrier timed out: the state is undefined until lbm_batch_reset");
    }
    if (steps & 1)
        for (auto &c : b->cur) c ^= 1;
    return LBM_OK;
}

lbm_status lbm_batch_populations(lbm_batch *b, int32_t index, double *f) {
    if (!b || !f) return fail(LBM_EINVAL, "NULL argument");
    if (b->poisoned) return fail(LBM_ESTATE, "a barrier wait expired in an earlier run: call lbm_batch_reset");
    if (index < 0 || index >= b->count) return fail(LBM_EINVAL, "index out of range");
    const BatchInst &d = b->desc[index];
    const LatInfo *L = lat_info(d.lattice);
    const size_t es = (size_t)elem_size(b->storage);
    const void *base = static_cast<char *>(b->pool) + (d.off + (size_t)b->cur[index] * L->Q * d.pstride) * es;
    double *t = nullptr;
    HIP_TRY(hipMalloc(&t, sizeof(double) * d.ncell));
    hipError_t e = hipSuccess;
    for (int a = 0; a < L->Q && e == hipSuccess; ++a) {
        const double add = is_dev(b->storage) ? L->w[a] : 0.0;
        e = b->ks[index]->decode(base, Layout{(uint32_t)d.nx, d.pstride, (uint64_t)d.nx}, d.ncell, a, add, 1.0, t, b->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(f + (size_t)a * d.ncell, t, sizeof(double) * d.ncell, hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    }
    (void)hipFree(t);
    HIP_TRY(e);
    return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch *b, int32_t steps, int32_t *form, int32_t *block, double *ms_per_step) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (b->poisoned) return fail(LBM_ESTATE, "a barrier wait expired in an earlier run: call lbm_batch_reset");
    if (steps < 1) return fail(LBM_EINVAL, "steps must be >= 1");
    void *save = nullptr;
    HIP_TRY(hipMalloc(&save, b->pool_bytes));
    hipError_t e = hipMemcpyAsync(save, b->pool, b->pool_bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_inst, b->desc.data(), sizeof(BatchInst) * b->count, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_cur, b->cur.data(), sizeof(int32_t) * b->count, hipMemcpyHostToDevice, b->stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const int saved_form = b->form, saved_block = b->block;
    int best_form = b->form, best_block = b->block;
    float best_ms = 1e30f;
    lbm_status st = LBM_OK;
    // time `steps` steps of the current plan in (form, blk) after a one-step warm-up; *ms < 0 if
    // the launch did not complete as planned
    auto time_trial = [&](int form, int blk, float *ms) {
        *ms = -1.0f;
        const BatchArgs a1 = batch_args(b, 1, 0, 0, 1), an = batch_args(b, steps, 0, 0, 1);
        e = launch_batch((int)b->storage, form, blk, a1, (uint32_t)b->count, b->stream);
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        if (e == hipSuccess) e = launch_batch((int)b->storage, form, blk, an, (uint32_t)b->count, b->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        int32_t ab = 0;
        if (e == hipSuccess && form >= 1) {
            e = hipMemcpy(&ab, b->d_abort, sizeof(int32_t), hipMemcpyDeviceToHost);
            if (e == hipSuccess && ab == 2) b->nxcd = -1;
        }
        if (e == hipSuccess && !ab) *ms = t;
    };
    for (int form : {0, 1, 2}) {
        for (int blk : {1024, 512, 256}) {
            if (e != hipSuccess || st != LBM_OK) break;
            if (form >= 1) {
                if (batch_grid_resident_per_cu((int)b->storage, form, blk) < 1) continue;
                if (form == 2 && b->nxcd < 0) continue;
                b->cal.erase({form, blk});
                b->plan_block = 0;
                if ((st = batch_plan(b, blk, form)) != LBM_OK) {
                    if (form == 2 && b->nxcd < 0) {   // XCD-local form unusable here: skip it
                        st = LBM_OK;
                        continue;
                    }
                    break;
                }
            }
            b->form = form;
            b->block = blk;
            float ms = 0;
            time_trial(form, blk, &ms);
            if (e == hipSuccess && form >= 1 && ms >= 0) {
                // calibrate the plan's cost model to a step profile of this form, and keep the
                // calibrated plan if it runs faster
                bool ok = false;
                if ((st = batch_calibrate(b, steps, &ok)) != LBM_OK) break;
                if (ok) {
                    float ms_cal = 0;
                    time_trial(form, blk, &ms_cal);
                    if (e == hipSuccess && ms_cal >= 0 && ms_cal < ms) {
                        ms = ms_cal;
                    } else {
                        b->cal.erase({form, blk});
                        b->plan_block = 0;
                    }
                }
            }
            if (e == hipSuccess && ms >= 0 && ms < best_ms) {
                best_ms = ms;
                best_form = form;
                best_block = blk;
            }
        }
    }
    b->form = saved_form;
    b->block = saved_block;
    if (e == hipSuccess) e = hipMemcpyAsync(b->pool, save, b->pool_bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(save);
    HIP_TRY(e);
    if (st != LBM_OK) return st;
    batch_drop_graph(b);
    b->form = best_form;
    b->block = best_block;
    b->plan_block = 0;
    if (b->form >= 1 && (st = batch_plan(b, b->block, b->form)) != LBM_OK) return st;
    if (form) *form = best_form;
    if (block) *block = best_block;
    if (ms_per_step) *ms_per_step = (double)best_ms / steps;
    return LBM_OK;
}

lbm_status lbm_batch_calibrate(lbm_batch *b, int32_t steps, double *costs, int32_t *ncosts) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (b->poisoned) return fail(LBM_ESTATE, "a barrier wait expired in an earlier run: call lbm_batch_reset");
    if (b->form == 0) return fail(LBM_EINVAL, "the cost model plans the grid forms (1 and 2) only");
    if (steps < 0) return fail(LBM_EINVAL, "steps must be >= 0");
    if (ncosts) *ncosts = b->nkinds + 1;
    b->cal.erase({b->form, b->block});
    b->plan_block = 0;
    lbm_status st = batch_plan(b, b->block, b->form);
    if (st != LBM_OK || steps == 0) {
        if (st == LBM_OK && costs)
            for (int k = 0; k <= b->nkinds; ++k) costs[k] = 0.0;
        return st;
    }
    void *save = nullptr;
    HIP_TRY(hipMalloc(&save, b->pool_bytes));
    hipError_t e = hipMemcpyAsync(save, b->pool, b->pool_bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    bool ok = false;
    if (e == hipSuccess) st = batch_calibrate(b, steps, &ok);
    if (e == hipSuccess) e = hipMemcpyAsync(b->pool, save, b->pool_bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(save);
    HIP_TRY(e);
    if (st != LBM_OK) return st;
    if (!ok) return fail(LBM_EDEVICE, "step profile failed or fitted no cost: the default model stays");
    if (costs) {
        const std::vector<double> &c = b->cal[{b->form, b->block}];
        for (int k = 0; k <= b->nkinds; ++k) costs[k] = c[k];
    }
    return LBM_OK;
}

lbm_status lbm_batch_form(const lbm_batch *b, int32_t *form, int32_t *block) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (form) *form = b->form;
    if (block) *block = b->block;
    return LBM_OK;
}

lbm_status lbm_batch_plan_xcds(lbm_batch *b, int32_t nxcd) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (nxcd < 0 || nxcd > (int32_t)kMaxXcd) return fail(LBM_EINVAL, "nxcd must be in [0, %u]", kMaxXcd);
    b->xcd_force = nxcd;
    b->plan_block = 0;   // plan again before the next run
    batch_drop_graph(b);
    return LBM_OK;
}

lbm_status lbm_batch_set_form(lbm_batch *b, int32_t form, int32_t block) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (b->poisoned) return fail(LBM_ESTATE, "a barrier wait expired in an earlier run: call lbm_batch_reset");
    if ((form < 0 || form > 2) || (block != 256 && block != 512 && block != 1024))
        return fail(LBM_EINVAL, "form must be 0, 1 or 2 and block 256, 512 or 1024");
    if (form >= 1) {
        lbm_status st = batch_plan(b, block, form);
        if (st != LBM_OK) return st;
    }
    batch_drop_graph(b);
    b->form = form;
    b->block = block;
    return LBM_OK;
}

}  // extern "C"

// ======================================================================== reduced DVM
#include "gh_rules.inc"
#include "rdvm.h"

struct lbm_rdvm {
    int count = 0;
    double cfl = 0.5;
    hipStream_t stream = nullptr;
    std::vector<lbm_rdvm_instance> inst;
    std::vector<RdvmInst> desc;
    RdvmInst *d_inst = nullptr;
    int32_t *d_index = nullptr;             // instance indices grouped by kernel variant
    int group_first[kRdvmVariants + 1] = {};  // variant kRdvmK[g]: d_index[group_first[g] .. group_first[g+1])
    double *d_nodes = nullptr, *d_tabs = nullptr, *d_state = nullptr, *d_log = nullptr;
    size_t state_elems = 0, log_cap = 0, lds_bytes = 0;
    bool two = false;                      // two state buffers fit in LDS
    int64_t nstep = 0;
};

extern "C" {

lbm_status lbm_gauss_hermite(int32_t n, double *nodes, double *weights) {
    if (n < kGHMin || n > kGHMax) return fail(LBM_EINVAL, "Gauss-Hermite rules exist for %d..%d points", kGHMin, kGHMax);
    const int o = kGHOffset[n - kGHMin];
    for (int k = 0; k < n; ++k) {
        if (nodes) nodes[k] = kGHNodes[o + k];
        if (weights) weights[k] = kGHWeights[o + k];
    }
    return LBM_OK;
}

void lbm_rdvm_free(lbm_rdvm *r) {
    if (!r) return;
    (void)hipStreamSynchronize(r->stream);
    for (void *p : {(void *)r->d_inst, (void *)r->d_index, (void *)r->d_nodes, (void *)r->d_tabs, (void *)r->d_state,
                    (void *)r->d_log})
        if (p) (void)hipFree(p);
    delete r;
}

lbm_status lbm_rdvm_create(lbm_rdvm **out, const lbm_rdvm_instance *inst, int32_t count, double cfl, void *hip_stream) {
    if (!out || !inst) return fail(LBM_EINVAL, "NULL argument");
    if (count < 1) return fail(LBM_EINVAL, "count must be >= 1");
    if (!(cfl > 0.0 && cfl <= 1.0)) return fail(LBM_EINVAL, "cfl must be in (0, 1], got %g", cfl);
    std::vector<double> nodes, tabs;
    std::vector<RdvmInst> desc((size_t)count);
    size_t state = 0, maxv = 0;
    int maxm = 0;
    for (int i = 0; i < count; ++i) {
        const lbm_rdvm_instance &q = inst[i];
        if (q.nodes < kGHMin || q.nodes > kRdvmMaxNodes)
            return fail(LBM_EINVAL, "instance %d: nodes must be in [%d, %d]", i, kGHMin, kRdvmMaxNodes);
        if (q.cells < 1 || q.cells > kRdvmMaxCells)
            return fail(LBM_EINVAL, "instance %d: cells must be in [1, %d]", i, kRdvmMaxCells);
        if ((size_t)q.nodes * (size_t)q.cells > (size_t)kRdvmMaxValues)
            return fail(LBM_EINVAL, "instance %d: nodes * cells exceeds %d", i, kRdvmMaxValues);
        if (!(q.kn > 0.0) || !isfinite(q.amplitude) || !isfinite(q.frequency))
            return fail(LBM_EINVAL, "instance %d: kn must be > 0 (or +inf), amplitude and frequency finite", i);
        const int M = q.nodes, nw = q.cells, o = kGHOffset[M - kGHMin];
        const double ximax = fabs(kGHNodes[o + M - 1]);
        RdvmInst &d = desc[(size_t)i];
        d.M = M;
        d.nw = nw;
        d.P = rdvm_threads_per_cell(nw);
        d.dt = cfl * (2.0 * M_PI / (double)nw) / ximax;
        d.omega = isinf(q.kn) ? 0.0 : d.dt / (q.kn + 0.5 * d.dt);
        d.amp = q.amplitude;
        d.freq = q.frequency;
        d.node_off = (uint32_t)nodes.size();
        for (int k = 0; k < M; ++k) nodes.push_back(kGHNodes[o + k]);
        for (int k = 0; k < M; ++k) nodes.push_back(kGHWeights[o + k]);
        for (int k = 0; k < M; ++k) {
            const double A = fabs(kGHNodes[o + k]) * cfl / ximax;   // |Courant number|
            nodes.push_back(A + 0.5 * A * (1.0 - A));
        }
        for (int k = 0; k < M; ++k) {
            const double A = fabs(kGHNodes[o + k]) * cfl / ximax;
            nodes.push_back(0.5 * A * (1.0 - A));
        }
        d.tab_off = (uint32_t)tabs.size();
        for (int j = 0; j < nw; ++j) tabs.push_back(cos(2.0 * M_PI * (double)j / (double)nw));
        for (int j = 0; j < nw; ++j) tabs.push_back(sin(2.0 * M_PI * (double)j / (double)nw));
        d.state_off = state;
        state += (size_t)M * nw;
        maxv = std::max(maxv, (size_t)M * nw);
        maxm = std::max(maxm, M);
    }
    std::vector<int32_t> index;
    int group_first[kRdvmVariants + 1];
    for (int g = 0; g < kRdvmVariants; ++g) {
        group_first[g] = (int)index.size();
        for (int i = 0; i < count; ++i)
            if (rdvm_variant(inst[i].nodes, inst[i].cells) == kRdvmK[g]) index.push_back(i);
    }
    group_first[kRdvmVariants] = (int)index.size();
    lbm_rdvm *r = new lbm_rdvm();
    r->count = count;
    r->cfl = cfl;
    r->stream = (hipStream_t)hip_stream;
    r->inst.assign(inst, inst + count);
    r->desc = desc;
    r->state_elems = state;
    r->two = rdvm_two_buffers(maxv, maxm);
    r->lds_bytes = rdvm_lds_bytes(maxv, maxm, r->two);
    for (int g = 0; g <= kRdvmVariants; ++g) r->group_first[g] = group_first[g];
    hipError_t e = rdvm_allow_lds(r->lds_bytes);
    if (e == hipSuccess) e = hipMalloc(&r->d_inst, sizeof(RdvmInst) * desc.size());
    if (e == hipSuccess) e = hipMalloc(&r->d_index, sizeof(int32_t) * index.size());
    if (e == hipSuccess)
        e = hipMemcpyAsync(r->d_index, index.data(), sizeof(int32_t) * index.size(), hipMemcpyHostToDevice, r->stream);
    if (e == hipSuccess) e = hipMalloc(&r->d_nodes, sizeof(double) * nodes.size());
    if (e == hipSuccess) e = hipMalloc(&r->d_tabs, sizeof(double) * tabs.size());
    if (e == hipSuccess) e = hipMalloc(&r->d_state, sizeof(double) * state);
    if (e == hipSuccess) e = hipMemcpyAsync(r->d_inst, desc.data(), sizeof(RdvmInst) * desc.size(), hipMemcpyHostToDevice, r->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r->d_nodes, nodes.data(), sizeof(double) * nodes.size(), hipMemcpyHostToDevice, r->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r->d_tabs, tabs.data(), sizeof(double) * tabs.size(), hipMemcpyHostToDevice, r->stream);
    if (e == hipSuccess) e = hipMemsetAsync(r->d_state, 0, sizeof(double) * state, r->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) {
        lbm_status st = fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "reduced DVM set-up: %s", hipGetErrorString(e));
        lbm_rdvm_free(r);
        (void)hipGetLastError();
        return st;
    }
    *out = r;
    return LBM_OK;
}

lbm_status lbm_rdvm_reset(lbm_rdvm *r) {
    if (!r) return fail(LBM_EINVAL, "reduced DVM is NULL");
    HIP_TRY(hipMemsetAsync(r->d_state, 0, sizeof(double) * r->state_elems, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    r->nstep = 0;
    return LBM_OK;
}

lbm_status lbm_rdvm_run(lbm_rdvm *r, int64_t steps, int32_t record_every, double *velocity, double *stress) {
    if (!r) return fail(LBM_EINVAL, "reduced DVM is NULL");
    if (steps < 0 || record_every < 0) return fail(LBM_EINVAL, "steps and record_every must be >= 0");
    if (steps == 0) return LBM_OK;
    const int64_t nrec64 = record_every > 0 ? steps / record_every : 0;
    if (nrec64 > 0x7fffffff) return fail(LBM_EINVAL, "too many records");
    const int32_t nrec = (int32_t)nrec64;
    const size_t need = (size_t)r->count * 2 * (size_t)nrec;
    if (need > r->log_cap) {
        if (r->d_log) HIP_TRY(hipFree(r->d_log));
        r->d_log = nullptr;
        r->log_cap = 0;
        HIP_TRY(hipMalloc(&r->d_log, sizeof(double) * need));
        r->log_cap = need;
        // each instance's records sit at log_off .. + 2 nrec; refresh the descriptors
    }
    for (int i = 0; i < r->count; ++i) r->desc[(size_t)i].log_off = (uint64_t)i * 2 * (uint64_t)nrec;
    HIP_TRY(hipMemcpyAsync(r->d_inst, r->desc.data(), sizeof(RdvmInst) * r->desc.size(), hipMemcpyHostToDevice, r->stream));
    RdvmArgs a{};
    a.inst = r->d_inst;
    a.nodes = r->d_nodes;
    a.tabs = r->d_tabs;
    a.state = r->d_state;
    a.log = r->d_log;
    a.step0 = r->nstep;
    a.steps = steps;
    a.record = nrec > 0 ? record_every : 0;
    a.nrec = nrec;
    a.two = r->two ? 1 : 0;
    for (int g = 0; g < kRdvmVariants; ++g) {
        const int n = r->group_first[g + 1] - r->group_first[g];
        if (n > 0) HIP_TRY(launch_rdvm(kRdvmK[g], a, r->d_index + r->group_first[g], (uint32_t)n, r->lds_bytes, r->stream));
    }
    r->nstep += steps;
    if (nrec > 0 && (velocity || stress)) {
        std::vector<double> h(need);
        HIP_TRY(hipMemcpyAsync(h.data(), r->d_log, sizeof(double) * need, hipMemcpyDeviceToHost, r->stream));
        HIP_TRY(hipStreamSynchronize(r->stream));
        for (int i = 0; i < r->count; ++i)
            for (int32_t k = 0; k < nrec; ++k) {
                if (velocity) velocity[(size_t)i * nrec + k] = h[(size_t)i * 2 * nrec + k];
                if (stress) stress[(size_t)i * nrec + k] = h[(size_t)i * 2 * nrec + nrec + k];
            }
    } else {
        HIP_TRY(hipStreamSynchronize(r->stream));
    }
    return LBM_OK;
}

lbm_status lbm_rdvm_state(lbm_rdvm *r, int32_t index, double *g) {
    if (!r || !g) return fail(LBM_EINVAL, "NULL argument");
    if (index < 0 || index >= r->count) return fail(LBM_EINVAL, "instance %d out of range", index);
    const RdvmInst &d = r->desc[(size_t)index];
    HIP_TRY(hipMemcpyAsync(g, r->d_state + d.state_off, sizeof(double) * (size_t)d.M * d.nw, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return LBM_OK;
}

lbm_status lbm_rdvm_info(const lbm_rdvm *r, int32_t index, double *dt, double *omega, int64_t *step) {
    if (!r) return fail(LBM_EINVAL, "reduced DVM is NULL");
    if (index < 0 || index >= r->count) return fail(LBM_EINVAL, "instance %d out of range", index);
    if (dt) *dt = r->desc[(size_t)index].dt;
    if (omega) *omega = r->desc[(size_t)index].omega;
    if (step) *step = r->nstep;
    return LBM_OK;
}

}  // extern "C"
