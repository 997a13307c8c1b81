/*
 * lbm.h -- C ABI of the MI355X (gfx950) BGK step for high-order lattice Boltzmann (LB)
 * and discrete-velocity (DVM) models.
 *
 * Method (Meng & Zhang, "Accuracy analysis of high-order lattice Boltzmann models for
 * rarefied gas flows"): populations f_a of a Gauss-Hermite velocity set {xi_a, w_a}
 * (section 2.1, Eqs. approxf, an, lbgk; Table 1) evolve by the second-order BGK scheme
 * of section 2.2 (Eq. 2order).  One time step, fused in one kernel per step:
 *   move      f_a(r) = f*_a(r - c_a)  -- exact periodic shift for integer (on-lattice)
 *             velocity sets (Eq. slb, Eq. 2order), or second-order upwind (Beam-Warming)
 *             advection per axis for off-lattice Gauss-Hermite sets (section 3.2);
 *   moments   rho = sum_a f_a, rho u = sum_a xi_a f_a                 (Eq. an, n = 0, 1);
 *   f^eq_a    = w_a rho sum_{n<=N} He_n-terms of (xi_a.u, u.u)        (Eq. demoeq for N=2;
 *             general N from a_eq^(n) = rho u^n, section 2.1);
 *   relax     f*_a = f_a - omega (f_a - f^eq_a), omega = 1/tau, tau = Kn/dt + 1/2.
 * The state kept between steps is the post-collision population f*.
 *
 * Units.  Velocities are in Hermite units (scaled by sqrt(R T0), Eq. nondime).  Grid cells
 * are unit spaced; on-lattice sets move c_a = xi_a / scale cells per step; off-lattice sets
 * advect with Courant numbers nu_ad = xi_ad * cfl / max_ad|xi_ad|.
 *
 * Layout.  cell = x + nx*(y + ny*z); populations are structure-of-arrays: every host array
 * of populations is f[a * ncell + cell] in FP64, in the population order reported by
 * lbm_lattice_info.  Per-cell vectors are u[d * ncell + cell].
 *
 * Errors.  Every call returns lbm_status; nothing throws or aborts across the ABI.  On an
 * error lbm_last_error() returns a thread-local message.  Output arguments are written only
 * on LBM_OK.  Host pointers are borrowed for the duration of the call only.
 *
 * Streams.  Work is enqueued on the simulation's HIP stream (the null stream unless one is
 * given in lbm_opts).  lbm_step is asynchronous; calls that return host data synchronise
 * that stream first.  One simulation must not be used from two threads at once.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* an argument is out of range; nothing was changed */
    LBM_ENOMEM = -2,     /* device (or pinned host) allocation failed */
    LBM_EDEVICE = -3,    /* a HIP call failed; lbm_last_error() has the HIP message */
    LBM_ENONFINITE = -4, /* the finite check found a NaN/Inf in the state */
    LBM_ESTATE = -5      /* the call is not valid in the object's current state */
} lbm_status;

/* Velocity sets.  Degrees are those of polynomial exactness of the quadrature. */
typedef enum {
    LBM_D2Q9 = 1,     /* Table 1; degree 5; |c| <= 1 */
    LBM_D2Q37 = 2,    /* 9th-degree on-lattice set, shells (0,0)..(3,1); |c| <= 3 */
    LBM_D3Q39 = 3,    /* 7th-degree on-lattice set, r^2 = 3/2; |c| <= 3 */
    LBM_D2Q16_GH = 4, /* 4x4 Gauss-Hermite product, off-lattice; degree 7 */
    LBM_D2Q36_GH = 5, /* 6x6 Gauss-Hermite product, off-lattice; degree 11 */
    LBM_D2Q16_CK = 6, /* Table 1 D2Q16 (m=1, n=4); degree 5 with these integers; |c| <= 4 */
    LBM_D2Q17 = 7,    /* Table 1; degree 7; |c| <= 3 */
    LBM_D2Q21 = 8,    /* Table 1; degree 7; |c| <= 3 */
    LBM_D2Q25_CK = 9  /* Table 1 D2Q25 (m=3, n=7); degree 7 with these integers; |c| <= 7 */
} lbm_lattice;

/* How populations are stored in device memory between steps.  The collision runs in FP64
 * for LBM_FP64 and in FP32 for every other storage.  *_DEV stores the deviation
 * g_a = f_a - w_a rho0 (rho0 = 1); LBM_FP16_DEV stores g_a / w_a. */
typedef enum {
    LBM_FP64 = 0,
    LBM_FP32 = 1,
    LBM_FP32_DEV = 2,
    LBM_FP16_DEV = 3,
    LBM_BF16_DEV = 4
} lbm_storage;

/* How to move populations each step. */
typedef enum {
    LBM_MOVE_AUTO = 0,  /* SHIFT for on-lattice sets, BW2 for off-lattice sets */
    LBM_MOVE_SHIFT = 1, /* exact periodic shift by c_a (on-lattice sets only) */
    LBM_MOVE_BW2 = 2    /* Beam-Warming second-order upwind advection, x then y then z */
} lbm_move;

typedef struct { int32_t nx, ny, nz; } lbm_grid;   /* nz = 1 for 2-D velocity sets */

typedef struct {
    lbm_storage storage;      /* default LBM_FP64 */
    lbm_move move;            /* default LBM_MOVE_AUTO */
    double cfl;               /* largest Courant number for LBM_MOVE_BW2, in (0, 1]; default 0.5 */
    int32_t stochastic_round; /* 16-bit storages: 0 = round to nearest even, 1 = stochastic */
    uint64_t sr_seed;         /* seed of the stochastic rounding stream */
    void *hip_stream;         /* hipStream_t to enqueue on; NULL = null stream */
    int32_t check_every;      /* >0: lbm_step checks the state for NaN/Inf every this many steps */
    int32_t tile;             /* kernel tile choice (0 = autotuned / default); see lbm_tile_count */
    /* Caller-owned population buffers (both NULL by default: the simulation allocates and frees
     * its own).  If given, both must be distinct device allocations of the current HIP device,
     * 16-byte aligned, each of at least dev_buf_bytes >= Q * ncell * (bytes per stored value)
     * bytes (lbm_state_bytes); they must not overlap and must outlive the simulation, which uses
     * them as its two buffers of the stored state f* (section 2.2, Eq. 2order) and never frees
     * them.  Their contents are undefined between calls (the step alternates between them; the
     * current one is the one lbm_save_state copies).  Batches do not take them. */
    void *dev_buf[2];
    int64_t dev_buf_bytes;
} lbm_opts;

typedef struct lbm_sim lbm_sim;

/* Fill *o with the defaults listed above. */
void lbm_opts_default(lbm_opts *o);

/* Velocity-set description in the library's population order.  Q and D are written when
 * non-NULL; c (Q*3 ints, zero third component in 2-D, all zero for off-lattice sets),
 * xi (Q*3 doubles, Hermite units) and w (Q doubles) are written when non-NULL.
 * Returns LBM_EINVAL for an unknown lattice. */
lbm_status lbm_lattice_info(lbm_lattice lat, int32_t *Q, int32_t *D, int32_t *c, double *xi, double *w);

/* Relaxation time for a Knudsen number (Eq. 2order: omega = dt/(Kn + dt/2) = 1/tau).
 * The characteristic length of Eq. nondime is one wavelength over wavelength_cells cells,
 * theta = 2 pi / wavelength_cells, so dx = 2 pi / wavelength_cells; dt = dx / scale for
 * on-lattice sets (xi_a dt = c_a dx) and dt = cfl dx / max|xi| for advection.
 * Returns tau = Kn/dt + 1/2, or NaN for invalid arguments. */
double lbm_tau_from_kn(lbm_lattice lat, lbm_move move, double kn, int32_t wavelength_cells, double cfl);
/* The non-dimensional time step dt of one step in the same units (dt = dx / scale, or
 * cfl dx / max|xi| for advection); NaN for invalid arguments. */
double lbm_time_step(lbm_lattice lat, lbm_move move, int32_t wavelength_cells, double cfl);

/* Create a simulation with the default options.  eq_order N in 1..4; tau > 1/2 (INFINITY
 * means collisionless, omega = 0); every grid dimension >= 1; nz = 1 for 2-D sets.
 * Allocates two population buffers on the current HIP device, unless o->dev_buf gives them
 * (LBM_EINVAL if only one is given, if they are not device memory of the current device, are
 * misaligned, overlap or are smaller than needed).  The state is zero until one of the set
 * calls below.  A quadrature degree below 2N (section 2.1) is allowed; lbm_warnings() then
 * reports LBM_WARN_QUADRATURE. */
lbm_status lbm_init(lbm_sim **out, lbm_lattice lat, int32_t eq_order, double tau, lbm_grid g);
lbm_status lbm_init_ex(lbm_sim **out, lbm_lattice lat, int32_t eq_order, double tau, lbm_grid g,
                       const lbm_opts *o);
void lbm_free(lbm_sim *s);   /* NULL-safe; synchronises the stream first */

#define LBM_WARN_QUADRATURE 1u
uint32_t lbm_warnings(const lbm_sim *s);

/* Standing shear wave of section 4 without forcing, at equilibrium (f = f^eq, step 0):
 * u_x = u0 sin(2 pi j / N_w) with j the cell index along wave_axis (1 = y, 2 = z) and
 * N_w that axis' length; u_y = u_z = 0; rho = 1 + rho_noise (2U - 1) with
 * U = (h >> 11) 2^-53 and h = SplitMix64 output number cell+1 of the stream started at
 * seed.  Runs on the device; asynchronous. */
lbm_status lbm_set_shear_wave(lbm_sim *s, double u0, int32_t wave_axis, double rho_noise, uint64_t seed);

/* f = f^eq(rho, u) from host fields rho[ncell], u[D*ncell]; resets the step counter. */
lbm_status lbm_init_equilibrium(lbm_sim *s, const double *rho, const double *u);

/* Advance n >= 0 steps (asynchronous).  With check_every > 0 the state is checked for
 * non-finite values every check_every steps and LBM_ENONFINITE returned on the first hit. */
lbm_status lbm_step(lbm_sim *s, int64_t n);

/* Number of steps taken since the last set call. */
int64_t lbm_step_count(const lbm_sim *s);

/* Body force of the oscillating standing shear wave (section 4, Eq. force, real part):
 * F_x = amplitude cos(frequency t) cos(2 pi j / N_w), j the cell index along wave_axis
 * (1 = y, 2 = z for 3-D on-lattice sets; 1 for advection) and N_w that axis' length, with
 * amplitude and frequency in the units of Eq. nondime and t = n dt (lbm_time_step for N_w)
 * the time of step n's collision.  From the next step on, every step uses the forced kernels
 * of the second-order scheme (Eq. 2order with its force term; the Hermite force term of
 * section 2.1 at order eq_order, expanded with the equilibrium's coefficients rho u^n).  The
 * stored state is then the shifted variable of Eq. 2order: lbm_moments, lbm_shear_amplitude
 * and lbm_totals report the physical velocity rho u = sum_a xi_a f*_a - rho G/2 (G the force
 * times dt of the latest collision, none at step 0).  amplitude 0 keeps the forced kernels
 * (and the stress below); wave_axis 0 switches back to the unforced kernels.  The row-tiled
 * forced kernel has 7 tiles (the 256-thread plain-store and the 512-thread non-temporal ones).
 * Allocates two small device tables.  LBM_EINVAL for an invalid axis or non-finite values. */
lbm_status lbm_set_force(lbm_sim *s, double amplitude, double frequency, int32_t wave_axis);

/* Sine and cosine projections over the force's wave axis (as lbm_shear_amplitude) of the
 * physical shear stress sum_a xi_ax xi_aw (f_a - f^eq_a), w the wave axis, at the collision of
 * the latest step, where f = f^eq + (1 - omega/2)(f~ - f^eq + F/2) is the distribution behind
 * the stored variable f~ (the inverse of its definition in section 2.2).  Summed in FP64 in a
 * fixed order.  LBM_ESTATE if no forced step ran since lbm_set_force or a set call. */
lbm_status lbm_shear_stress_amplitude(lbm_sim *s, double *s_sin, double *s_cos);

/* Host copies (synchronising): rho[ncell] and u[D*ncell] in FP64 from the stored f*
 * (the collision conserves rho and rho u, so these are the moments at the current step;
 * with a body force, u is the physical velocity described at lbm_set_force). */
lbm_status lbm_moments(lbm_sim *s, double *rho, double *u);

/* Sine and cosine projections of the x-velocity along wave_axis, in FP64:
 * a_sin = (2/N_w) sum_j ubar_x(j) sin(2 pi j/N_w), ubar_x(j) the mean of u_x over the cells
 * with wave-axis index j (the velocity amplitude of section 4); a_cos likewise. */
lbm_status lbm_shear_amplitude(lbm_sim *s, int32_t wave_axis, double *a_sin, double *a_cos);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops): lbm_shear_amplitude without any allocation and without synchronising.  Enqueues the same
 * reduction kernels on the simulation's stream and writes a_sin to dev_out[0] and a_cos to
 * dev_out[1], where dev_out points to two doubles of device memory (bit for bit the values
 * lbm_shear_amplitude returns).  The reduction's partial sums go to a static scratch array of
 * the library (about 96 KiB per GPU, held until the process ends; at most 2048 reduction
 * workgroups, which every simulation satisfies, else LBM_EINVAL); calls that overlap on one GPU,
 * on any streams, share that array and race.  LBM_EINVAL for NULL pointers or an invalid axis,
 * LBM_EDEVICE if the scratch could not be located on the simulation's device. */
lbm_status lbm_shear_amplitude_noalloc(lbm_sim *s, int32_t wave_axis, double *dev_out);

/* Global FP64 sums: mass = sum rho, mom[d] = sum rho u_d (D entries). */
lbm_status lbm_totals(lbm_sim *s, double *mass, double *mom);

/* Decoded FP64 copy of the stored state f*[a * ncell + cell] (checkpoint), and its inverse
 * (encodes into the storage format, rounding as configured; resets nothing else). */
lbm_status lbm_get_populations(lbm_sim *s, double *f);
lbm_status lbm_set_populations(lbm_sim *s, const double *f);
/* Decoded FP64 populations of `count` listed cells (cell = x + nx (y + ny z), each in
 * [0, ncell)), as lbm_get_populations computes them: f[a * count + k] is population a of
 * cells[k].  For inspecting grids too large to copy whole.  LBM_EINVAL for a cell out of
 * range (nothing is copied). */
lbm_status lbm_get_cells(lbm_sim *s, const int64_t *cells, int64_t count, double *f);
/* Restore the step counter together with lbm_set_populations (checkpoint resume). */
lbm_status lbm_set_step_count(lbm_sim *s, int64_t n);

/* Raw checkpoint of the stored state in its storage format (bit-exact restore):
 * lbm_state_bytes gives the size (Q ncell values); save copies the current buffer to host
 * memory, load copies it back.  Together with lbm_step_count / lbm_set_step_count this resumes
 * a run exactly.  Device layout: the Q populations of each grid row follow one another,
 * population a of cell (x, y, z) at value ((z ny + y) Q + a) nx + x. */
lbm_status lbm_state_bytes(const lbm_sim *s, int64_t *bytes);
lbm_status lbm_save_state(lbm_sim *s, void *host, int64_t bytes);
lbm_status lbm_load_state(lbm_sim *s, const void *host, int64_t bytes);

/* Least-squares slope of -ln|amp[k]| against steps[k] over n_first <= steps[k] <= n_last,
 * in FP64 (the decay rate per step of the shear-wave amplitude).  Needs >= 2 points. */
lbm_status lbm_fit_decay(const double *amp, const int64_t *steps, int64_t count, int64_t n_first,
                         int64_t n_last, double *gamma);

/* Complex amplitude z = re + i im of a periodic response amp[k] = Re(z e^{i frequency t_k}),
 * t_k = steps[k] dt, by least squares over n_first <= steps[k] <= n_last (for frequency 0:
 * the mean, im = 0).  Against a force proportional to cos(frequency t) the amplitude is |z|
 * and the phase lag -arg z.  LBM_EINVAL for NULL pointers, dt <= 0, an empty window or one
 * that does not resolve the oscillation. */
lbm_status lbm_fit_oscillation(const double *amp, const int64_t *steps, int64_t count, double dt, double frequency,
                               int64_t n_first, int64_t n_last, double *re, double *im);

/* Tile choices of the step kernel for this simulation's configuration; lbm_set_tile picks one
 * (0 = default), lbm_autotune times every choice on a scratch copy of the state and keeps the
 * fastest (the state itself is left unchanged). */
int32_t lbm_tile_count(const lbm_sim *s);
lbm_status lbm_set_tile(lbm_sim *s, int32_t tile);
/* Launch shape of tile `tile` (0 <= tile < lbm_tile_count): threads per workgroup, cells each
 * thread updates (consecutive chunks of a row for the shift kernel, rows of a strip for the
 * Beam-Warming kernel), cells per vector access (4 for the shift tiles that load and store 4
 * consecutive cells at once, else 1), workgroups per step launch, and whether the step kernel
 * writes with non-temporal stores.  Host only; any output pointer may be NULL.  LBM_EINVAL for a
 * NULL sim or a tile out of range. */
lbm_status lbm_tile_info(const lbm_sim *s, int32_t tile, int32_t *block_threads, int32_t *cells_per_thread,
                         int32_t *vector_width, int64_t *blocks, int32_t *nontemporal);
lbm_status lbm_autotune(lbm_sim *s, int32_t steps_per_trial, int32_t *best_tile, double *best_ms);
/* lbm_autotune with a persistent cache in the text file `path` (JSON lines, one choice each:
 * {"key": k, "tile": t, "shape": d, "ms": m}).  The key names the device architecture (HIP's
 * gcnArchName), lattice, eq_order, storage, rounding, move, whether the body force is on, and the
 * grid class: ceil(log2 nx), ceil(log2 (ny nz)) and whether nx is a multiple of 256 (grids of one
 * class share their best tile).  If the file holds the key, and the tile it names is valid for
 * this simulation and the library still describes that tile's launch as d, the tile is set
 * without timing: *hit = 1, *best_ms = m (the time stored when it was tuned).  Otherwise the
 * choice is tuned as by lbm_autotune, *hit = 0, and the file is rewritten with the new line
 * (replacing an older one of the same key) into a temporary file beside it that is renamed over
 * it: a reader never sees a torn file, and of two processes storing at once the later rename
 * wins.  A missing file is an empty cache; lines that do not parse are dropped on rewrite.
 * LBM_EINVAL for a NULL sim or path or steps_per_trial < 1, and if the file cannot be read or
 * written (the tuned tile is set all the same).  Output pointers may be NULL. */
lbm_status lbm_autotune_cached(lbm_sim *s, const char *path, int32_t steps_per_trial, int32_t *best_tile,
                               double *best_ms, int32_t *hit);

/* Information: cells, populations and bytes moved per step (2 Q ncell * bytes per value). */
lbm_status lbm_sizes(const lbm_sim *s, int64_t *ncell, int32_t *Q, int32_t *D, int64_t *bytes_per_step);

/* ---- Batches: many independent shear-wave instances advanced together (a Kn sweep).
 * Every instance is a decaying standing shear wave (as lbm_set_shear_wave with no density
 * noise) on its own periodic nx x ny grid with its own velocity set, Hermite order and tau.
 * lbm_batch_run advances all of them by `steps` steps in one persistent kernel launch (the
 * step loop on the device; an instance owned by one workgroup or cut over several, by the
 * form below), replayed from a captured HIP graph, and records each instance's sine amplitude of u_x (as lbm_shear_amplitude,
 * wave along y) every record_every steps.  Supported: 2-D sets D2Q9, D2Q37 (exact shift),
 * D2Q16_GH, D2Q36_GH (Beam-Warming advection at o->cfl); eq_order 1..4; storage
 * LBM_FP32_DEV or LBM_FP64; wave_axis 1; nz = 1; at most 2^26 cells per instance. */
typedef struct {
    lbm_lattice lat;
    int32_t eq_order;
    double tau;            /* > 1/2, or INFINITY */
    lbm_grid g;            /* nz = 1 */
    double u0;             /* amplitude of u_x = u0 sin(2 pi y / ny) at step 0 */
    int32_t wave_axis;     /* must be 1 */
} lbm_instance;

typedef struct lbm_batch lbm_batch;

/* Allocates every instance's two population buffers in one device pool and initialises
 * each instance to its shear wave at step 0.  o may be NULL (storage LBM_FP32_DEV, cfl 0.5);
 * o->hip_stream NULL means the batch creates its own stream (graph capture needs one);
 * o->dev_buf must be NULL (LBM_EINVAL otherwise). */
lbm_status lbm_batch_create(lbm_batch **out, const lbm_instance *inst, int32_t count, const lbm_opts *o);
/* Every instance back to its shear wave at step 0.  Also the way out of the undefined state a
 * barrier timeout leaves (see lbm_batch_set_form). */
lbm_status lbm_batch_reset(lbm_batch *b);
/* Advance every instance by steps >= 0 steps.  If amp is non-NULL it receives, per instance
 * in input order, steps / record_every + 1 amplitudes (before the first step, then after
 * every record_every steps): amp[i * (steps / record_every + 1) + k].  record_every >= 1.
 * Synchronises before returning. */
lbm_status lbm_batch_run(lbm_batch *b, int64_t steps, int32_t record_every, double *amp);
/* Decoded FP64 populations f[a * ncell + cell] of instance `index` (ncell = nx * ny). */
lbm_status lbm_batch_populations(lbm_batch *b, int32_t index, double *f);
/* Three persistent forms: form 0 gives each instance one workgroup for the whole run (no
 * synchronisation across CUs; the largest instance bounds the run time); form 1 cuts every
 * instance into chunks of one cell per thread, spreads them over a grid that is resident at
 * once, and meets at a device-wide barrier after every step; form 2 is form 1 with all chunks of
 * an instance on workgroups of one XCD and a barrier per XCD (no data crosses an XCD's L2).
 * Barrier waits are bounded.  If one expires (the workgroups were not resident together), every
 * workgroup leaves its step loop, the run returns LBM_EDEVICE, and the instances are left partly
 * stepped: the state is undefined, and lbm_batch_run, lbm_batch_populations, lbm_batch_autotune
 * and lbm_batch_set_form return LBM_ESTATE until lbm_batch_reset succeeds (lbm_batch_form,
 * lbm_batch_sizes and lbm_batch_free still work).
 * Form 2 needs the grid's workgroups spread evenly over the XCDs: lbm_batch_set_form returns
 * LBM_EDEVICE if a probe launch finds otherwise, and if a run finds otherwise it changes
 * nothing, switches the batch to form 1 and runs in that form.  Workgroup size 256, 512 or
 * 1024.  lbm_batch_set_form picks one; lbm_batch_autotune times every (form, size) pair over
 * `steps` steps, keeps the fastest and restores the state as it was; lbm_batch_form reports
 * the form and size in use.  The grid forms deal chunks to workgroups by a cost model (a fixed
 * cost per chunk plus a cost per cell and velocity set); for each grid (form, size) the autotuner
 * also takes a step profile (as lbm_batch_profile), fits the model's costs to the workgroups'
 * measured times by non-negative least squares, plans again with them, times that plan, and keeps
 * the fitted costs for that (form, size) only if they run faster.  The plan never changes what
 * is computed: every cell is stepped by the same arithmetic in every form and plan. */
lbm_status lbm_batch_set_form(lbm_batch *b, int32_t form, int32_t block);
lbm_status lbm_batch_autotune(lbm_batch *b, int32_t steps, int32_t *form, int32_t *block, double *ms_per_step);
lbm_status lbm_batch_form(const lbm_batch *b, int32_t *form, int32_t *block);
/* The autotuner's calibration step for the form and size in use (grid forms only): a step
 * profile of `steps` >= 1 steps, the cost model fitted to it, and the batch planned with the
 * fitted costs (kept for this form and size until a later calibration or autotune replaces them).
 * The state is left as it was.  costs (may be NULL) receives *ncosts = K + 1 values: the fitted
 * cost per cell of each of the K velocity sets present (in order of their first instance), then
 * the cost per chunk (device clock ticks).  steps = 0 drops the fitted costs of this form and size
 * (back to the default model; costs receives zeros).  LBM_EINVAL in form 0 or for steps < 0;
 * LBM_EDEVICE if the profile did not complete as planned or nothing could be fitted (the default
 * model then stays). */
lbm_status lbm_batch_calibrate(lbm_batch *b, int32_t steps, double *costs, int32_t *ncosts);
/* Testing hook of form 2's fallback: plan it for nxcd XCDs (1..16) instead of the number a probe
 * launch finds (nxcd = 0 restores the probe).  A plan for fewer XCDs than the device has leaves
 * the workgroups of the other XCDs without a slot; the next lbm_batch_run sees that before any
 * step, switches to form 1 and runs there (no kernel waits on a missing workgroup).  LBM_EINVAL
 * for nxcd outside 0..16. */
lbm_status lbm_batch_plan_xcds(lbm_batch *b, int32_t nxcd);
/* Testing hook of the timeout path: bound every barrier wait of the grid forms by `limit` sleeps
 * of about 50 ns (0 restores the default of 2^26, seconds; larger values are capped there).  A
 * tiny bound makes waits expire and exercises the undefined-state rule above; every workgroup
 * still leaves normally. */
lbm_status lbm_batch_set_spin_limit(lbm_batch *b, uint32_t limit);
/* Step profile of the grid forms (1 and 2): advances every instance by `steps` >= 1 steps as
 * lbm_batch_run does (no amplitudes, no graph), and every workgroup of the persistent grid
 * stores three timestamps of the device's constant 100 MHz clock for each of the steps
 * first .. first + count - 1: when the step started, when the workgroup's chunks were done (all
 * its threads), and when the step's barrier released it.  ts (host, may be NULL) receives
 * nwg * count * 3 values, ts[(w * count + k) * 3 + j] for workgroup w of the plan, step first + k,
 * timestamp j; *nwg receives the number of workgroups (with ts NULL nothing runs: a size query).
 * The chunk work and barrier wait per step follow as differences, which is what the batch's
 * load balance is judged by.  LBM_EINVAL in form 0, for an empty or out-of-range step window,
 * or above 2^28 timestamps; barrier timeouts and the XCD fallback act as in lbm_batch_run, except
 * that after a fallback nothing was stepped and LBM_EDEVICE is returned (profile again). */
lbm_status lbm_batch_profile(lbm_batch *b, int64_t steps, int64_t first, int32_t count, int32_t *nwg, uint64_t *ts);
/* Total cells and algorithmic bytes per step (2 Q ncell x bytes per value, summed). */
lbm_status lbm_batch_sizes(const lbm_batch *b, int64_t *cells, int64_t *bytes_per_step);
void lbm_batch_free(lbm_batch *b);   /* NULL-safe */

/* ---- Reduced discrete-velocity model of the forced standing shear wave (section 4, Eqs. ga
 * and gb): the linearised BGK equation of Eq. LBGK with xi_x integrated out.  Started from
 * rest, G_a stays zero (Eq. ga has no source), so an instance carries G_b on the M-point
 * Gauss-Hermite rule in xi_y (lbm_gauss_hermite; u_x = sum_k w_k G_b(xi_k)) times N_w periodic
 * cells of y in [0, 2 pi) (one wavelength), driven by F_x = amplitude cos(frequency t)
 * cos(2 pi j / N_w).  One step: Beam-Warming advection of every velocity at Courant number
 * xi_k dt / dy, dt = cfl dy / max|xi_k|, then the second-order relaxation and source of
 * Eq. 2order on the shifted variable G~ = G + dt/(2 Kn)(G - u_x) - dt F_x / 2:
 *   u_x = sum_k w_k G~_k + dt F_x / 2,   G~_k <- G~_k - omega (G~_k - u_x) + (1 - omega/2) dt F_x,
 * omega = dt / (Kn + dt/2), F_x at the step's collision time t = n dt.  FP64 throughout. */
typedef struct {
    int32_t nodes;       /* Gauss-Hermite points M in xi_y, 2..64 */
    int32_t cells;       /* N_w, 1..256 */
    double kn;           /* Knudsen number > 0 (INFINITY = collisionless) */
    double amplitude;    /* force amplitude A (units of Eq. nondime) */
    double frequency;    /* force frequency phi (0 = steady force) */
} lbm_rdvm_instance;
typedef struct lbm_rdvm lbm_rdvm;

/* The n-point Gauss-Hermite rule (2 <= n <= 64) for the weight exp(-x^2/2)/sqrt(2 pi): nodes
 * ascending and weights summing to 1 (tables generated in 60-digit arithmetic).  Host only;
 * either pointer may be NULL.  LBM_EINVAL for n out of range. */
lbm_status lbm_gauss_hermite(int32_t n, double *nodes, double *weights);

/* count >= 1 instances at rest (G~ = 0, step 0), advanced together: one workgroup per instance
 * keeps its whole state in on-chip memory for a run.  cfl in (0, 1].  hip_stream may be NULL
 * (the default stream).  Copies inst. */
lbm_status lbm_rdvm_create(lbm_rdvm **out, const lbm_rdvm_instance *inst, int32_t count, double cfl,
                           void *hip_stream);
/* All instances back to rest, step 0. */
lbm_status lbm_rdvm_reset(lbm_rdvm *r);
/* Advance all instances by steps >= 0 steps in one launch.  With record_every >= 1 and
 * non-NULL arrays, after every record_every steps of this run it records per instance the
 * cosine projection of the velocity, (2/N_w) sum_j u_x(j) cos(2 pi j/N_w), into
 * velocity[i * nrec + k], and the sine projection of the shear stress sum_k w_k xi_k G_k
 * (G the distribution behind G~, G - u_x = (1 - omega/2)(G~ - u_x + dt F/2)) into
 * stress[i * nrec + k], nrec = steps / record_every, both at the collision of that step.
 * Synchronises before returning. */
lbm_status lbm_rdvm_run(lbm_rdvm *r, int64_t steps, int32_t record_every, double *velocity, double *stress);
/* FP64 copy of instance `index`'s state G~[k * N_w + j] (M * N_w values). */
lbm_status lbm_rdvm_state(lbm_rdvm *r, int32_t index, double *g);
/* Time step, omega and the step count (shared by all instances); any pointer may be NULL. */
lbm_status lbm_rdvm_info(const lbm_rdvm *r, int32_t index, double *dt, double *omega, int64_t *step);
void lbm_rdvm_free(lbm_rdvm *r);   /* NULL-safe */

/* Measurement aid: copy `bytes` of device memory from src to dst (asynchronous, on hip_stream;
 * NULL = null stream) with a grid-stride loop of `blocks` workgroups of 256 threads, 16-byte
 * vector loads and non-temporal 16-byte stores.  Its bandwidth, 2 * bytes / time, is the
 * practical ceiling for a kernel that reads and writes each byte once.  LBM_EINVAL for NULL
 * pointers, sizes or addresses that are not multiples of 16, blocks < 1, or overlap. */
lbm_status lbm_device_copy(void *dst, const void *src, int64_t bytes, int32_t blocks, void *hip_stream);

/* Thread-local text of the last error (empty string if none). */
const char *lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
