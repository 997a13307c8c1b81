// host_logic.h -- the runtime's host-only decisions, free of HIP so that they also build and run
// in a plain CPU program: step-kernel tile tables and launch geometry, argument validation, the
// batch's chunk-to-workgroup plan, and the autotuner's persistent cache.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "lbm.h"

namespace lbm {
namespace host {

constexpr uint32_t kCellBlock = 256;   // threads per workgroup of the one-thread-per-cell kernels

// Shift tiles: kernel variant (0: 256 threads, 1: 256 threads with non-temporal stores, 2: 512
// threads with non-temporal stores, 3: 256 threads x 4 cells per thread with vector accesses) and
// chunks per block (of block threads x cells per thread).
struct ShiftTile {
    int variant, block, chunks;
};
// Beam-Warming tiles: rows per strip and variant (0: plain stores, 1: non-temporal stores,
// 2: non-temporal stores and alternating walk directions of neighbouring strips, 3: variant 2
// with non-temporal loads of the stencil's own column, 4: variant 2 with the next row's loads
// issued before the current row is computed).
struct BWTile {
    int rows, variant;
};
extern const ShiftTile kShiftTiles[];
extern const BWTile kBWTiles[];
constexpr int kShiftTileCount = 11;
constexpr int kPlainShiftTiles = 9;    // without the vector tiles (variant 3)
constexpr int kForcedShiftTiles = 7;   // the forced row kernel exists as variants 0 and 2 only
constexpr int kBWTileCount = 22;
constexpr int kForcedBWTiles = 5;      // the forced Beam-Warming kernel exists as variant 0 only

// What the tile choice depends on.
struct StepShape {
    bool bw2;          // Beam-Warming advection (else the exact shift)
    bool rows_ok;      // the row-tiled shift kernel is valid for the grid
    bool forced;       // body-force kernels
    bool vector_ok;    // the 4-cells-per-thread shift kernel exists and nx % 256 == 0
    int nx, ny, nz;
};

// Launch geometry of one step: tile (rows per strip, or chunks per block), blocks per row (or
// strip row) and the 1-D grid size.
struct StepGeom {
    uint32_t tile, per_row, nblocks;
};

int tile_count(const StepShape &s);
// tile must be in [0, tile_count(s)).
StepGeom step_geometry(const StepShape &s, int tile);
// Threads per workgroup, cells per thread, vector width and whether stores are non-temporal.
void tile_launch(const StepShape &s, int tile, int *block, int *cells_per_thread, int *vector_width, bool *nontemporal);

// The row-tiled shift kernel needs whole 256-cell rows, rows at least as long and as many as
// the largest |c| in each direction, and one grid row of all populations below 2^31 bytes.
bool row_tiles_ok(bool shift, int Q, int D, int R, const lbm_grid &g, int esize);

// Velocity-set facts the validation needs (the library's tables hold the rest).
struct LatShape {
    int Q, D, R;
    bool on_lattice;
};

// Bytes per stored value of o.storage (0 for a value outside the enumeration).
int storage_bytes(const lbm_opts &o);
// lbm_init_ex's argument checks that need no device (everything but dev_buf's memory type).
// esize = storage_bytes(o) (any value if the storage is invalid, which is reported first).
// L = nullptr for an unknown lattice.  On success *move receives the resolved move.
lbm_status check_init(const LatShape *L, int eq_order, double tau, const lbm_grid &g, const lbm_opts &o,
                      int esize, lbm_move *move, std::string *msg);
// dev_buf checks that need no device: both or neither, size, alignment, overlap.
lbm_status check_dev_buf_shape(const lbm_opts &o, uint64_t need, std::string *msg);

// ---- batch plan
struct PlanChunk {
    int32_t inst;
    uint32_t start, count;
};
struct BatchPlan {
    std::vector<PlanChunk> chunks;        // in instance order, each instance cut into block-cell chunks
    std::vector<uint32_t> inst_first;     // chunks of instance i: inst_first[i] .. inst_first[i + 1] - 1
    std::vector<uint32_t> wg_first;       // chunks of workgroup w: wg_chunks[wg_first[w] .. wg_first[w + 1] - 1]
    std::vector<uint32_t> wg_chunks;
    uint32_t nwg = 0, per_xcd = 0;        // per_xcd: workgroups per XCD in form 2
};
// Default model of the time per cell of one step of an instance (relative units, used only to
// balance); the autotuner replaces it by costs fitted to a step profile (fit_chunk_costs).
double batch_cell_cost(bool on_lattice, int Q);
// Longest-processing-time-first: items (largest cost first) onto the least-loaded of n bins;
// each bin's list is returned sorted.
std::vector<std::vector<uint32_t>> lpt(const std::vector<uint32_t> &items, const std::vector<double> &cost, uint32_t n);
// Cut instances (ncell[i] cells) into chunks of `block` cells, a chunk of n cells of instance i
// costing per_chunk + per_cell[i] n, and deal them to workgroups: form 1 over min(chunks,
// resident) workgroups; form 2 gives each of nxcd XCDs whole instances (balanced by cost) and up
// to resident / nxcd workgroups (form 2 needs resident >= nxcd, so that the whole grid is
// resident).  Within these, longest-processing-time-first.
BatchPlan plan_batch(const std::vector<uint32_t> &ncell, const std::vector<double> &per_cell, double per_chunk,
                     uint32_t block, int form, uint32_t resident, uint32_t nxcd);

// Non-negative least squares with few unknowns (1 <= n <= 8): the x >= 0 minimising |A x - y|
// (A row-major m x n), found exactly by solving the normal equations on every support set and
// keeping the best feasible solution.  Columns that are all zero get x = 0.
std::vector<double> nnls_small(const std::vector<double> &A, int m, int n, const std::vector<double> &y);

// Costs of the chunk model fitted to measured per-workgroup step times: work[w] ~ per_chunk
// (chunks of w) + sum over kinds k of cost[k] (cells of kind k in w), kind[i] in [0, nkinds) the
// kind (velocity set) of instance i.  Returns nkinds + 1 values (per-cell costs, then the
// per-chunk cost), by non-negative least squares and then floored (per-cell costs at 1% of the
// largest, the per-chunk cost at 1% of the mean measured time per chunk) so that no chunk costs
// nothing; all zero if nothing could be fitted.
std::vector<double> fit_chunk_costs(const BatchPlan &p, const std::vector<int> &kind, int nkinds,
                                    const std::vector<double> &work);

// ---- autotuner cache: a text file of JSON lines, one tuned choice per line,
// {"key": "...", "tile": t, "shape": "...", "ms": m}
struct TuneEntry {
    std::string key;
    int tile = -1;
    std::string shape;
    double ms = 0;
};
// Key of a simulation's choice: device architecture, lattice, order, storage, rounding, move,
// force, and grid class (ceil log2 of nx and of ny nz, whether nx is a multiple of 256).
std::string tune_key(const char *arch, int lattice, int order, int storage, int sr, const StepShape &s);
// Description of a tile's launch, stored beside it: a hit counts only if the library still
// describes that tile the same way.
std::string tile_shape(const StepShape &s, int tile);
// Entries of a cache file in file order (lines that do not parse are skipped; a missing file is
// empty).  Returns false only if the file exists and cannot be read.
bool tune_read(const std::string &path, std::vector<TuneEntry> *out);
// The last entry with this key, if any.
bool tune_lookup(const std::string &path, const std::string &key, TuneEntry *out);
// Replace (or append) the entry with e.key: the file is rewritten into path + a unique suffix and
// renamed over path, so readers never see a torn file (concurrent writers: the last rename wins).
bool tune_store(const std::string &path, const TuneEntry &e, std::string *err);
// One JSON line (no newline) and its parser.
std::string tune_format(const TuneEntry &e);
bool tune_parse(const std::string &line, TuneEntry *out);

}  // namespace host
}  // namespace lbm
