// host_logic.cpp -- see host_logic.h.  Plain C++ (no HIP): the runtime links it, and a CPU
// harness builds it with the address and undefined-behaviour sanitizers.
#include "host_logic.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>

namespace lbm {
namespace host {

const ShiftTile kShiftTiles[kShiftTileCount] = {{0, 256, 1}, {0, 256, 2}, {0, 256, 4}, {0, 256, 8},
                                                {2, 512, 4}, {2, 512, 2}, {2, 512, 1}, {1, 256, 4},
                                                {1, 256, 8}, {3, 256, 1}, {3, 256, 2}};
const BWTile kBWTiles[kBWTileCount] = {{16, 0}, {32, 0}, {8, 0},  {4, 0},  {64, 0}, {16, 1}, {32, 1}, {8, 1},
                                       {16, 2}, {32, 2}, {8, 2},  {4, 2},  {64, 2}, {10, 2}, {12, 2}, {13, 2},
                                       {8, 3},  {16, 3}, {8, 4},  {16, 4}, {4, 4},  {32, 4}};

namespace {

std::string fmt(const char *f, ...) __attribute__((format(printf, 1, 2)));
std::string fmt(const char *f, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, f);
    vsnprintf(buf, sizeof buf, f, ap);
    va_end(ap);
    return buf;
}

lbm_status bad(std::string *msg, const std::string &m) {
    if (msg) *msg = m;
    return LBM_EINVAL;
}

// Enum fields arrive from C callers as plain 32-bit ints: read them as ints, since a value outside
// the enumeration is not a valid value of the C++ enum type.
template <class E>
int32_t raw(const E &e) {
    static_assert(sizeof(E) == sizeof(int32_t), "32-bit enum");
    int32_t v;
    memcpy(&v, &e, sizeof v);
    return v;
}

int ceil_log2(uint64_t v) {
    int k = 0;
    while (k < 63 && (1ull << k) < v) ++k;
    return k;
}

}  // namespace

int tile_count(const StepShape &s) {
    if (s.bw2) return s.forced ? kForcedBWTiles : kBWTileCount;
    if (s.rows_ok) {
        if (s.forced) return kForcedShiftTiles;
        return s.vector_ok ? kShiftTileCount : kPlainShiftTiles;
    }
    return 1;
}

StepGeom step_geometry(const StepShape &s, int tile) {
    StepGeom g{};
    const uint32_t nx = (uint32_t)s.nx;
    if (s.bw2) {
        const uint32_t H = (uint32_t)kBWTiles[tile].rows;
        g.tile = H;
        g.per_row = (nx + kCellBlock - 1) / kCellBlock;   // blocks of 4 waves x 64 columns
        g.nblocks = g.per_row * (((uint32_t)s.ny + H - 1) / H);
    } else if (s.rows_ok) {
        const ShiftTile &t = kShiftTiles[tile];
        const uint32_t cpt = (uint32_t)t.chunks, blk = (uint32_t)t.block * (t.variant == 3 ? 4u : 1u);
        g.tile = cpt;
        g.per_row = (nx + blk * cpt - 1) / (blk * cpt);
        g.nblocks = g.per_row * (uint32_t)s.ny * (uint32_t)s.nz;
    } else {
        const uint64_t ncell = (uint64_t)s.nx * (uint64_t)s.ny * (uint64_t)s.nz;
        g.tile = 1;
        g.per_row = 1;
        g.nblocks = (uint32_t)((ncell + kCellBlock - 1) / kCellBlock);
    }
    return g;
}

void tile_launch(const StepShape &s, int tile, int *block, int *cells_per_thread, int *vector_width, bool *nontemporal) {
    const StepGeom g = step_geometry(s, tile);
    const bool rows = !s.bw2 && s.rows_ok;
    const int vw = rows && kShiftTiles[tile].variant == 3 ? 4 : 1;
    if (block) *block = rows ? kShiftTiles[tile].block : (int)kCellBlock;
    if (cells_per_thread) *cells_per_thread = (int)g.tile * vw;
    if (vector_width) *vector_width = vw;
    if (nontemporal) *nontemporal = rows ? kShiftTiles[tile].variant != 0 : (s.bw2 && kBWTiles[tile].variant != 0);
}

bool row_tiles_ok(bool shift, int Q, int D, int R, const lbm_grid &g, int esize) {
    const bool row_fits = (uint64_t)Q * (uint64_t)g.nx * (uint64_t)esize < (1ull << 31);
    return shift && row_fits && g.nx >= 256 && g.nx >= R && g.ny >= R && (D == 2 || g.nz >= R);
}

int storage_bytes(const lbm_opts &o) {
    switch (raw(o.storage)) {
        case LBM_FP64: return 8;
        case LBM_FP32:
        case LBM_FP32_DEV: return 4;
        case LBM_FP16_DEV:
        case LBM_BF16_DEV: return 2;
        default: return 0;
    }
}

lbm_status check_init(const LatShape *L, int eq_order, double tau, const lbm_grid &g, const lbm_opts &o,
                      int esize, lbm_move *move, std::string *msg) {
    if (!L) return bad(msg, "unknown lattice");
    if (eq_order < 1 || eq_order > 4) return bad(msg, fmt("eq_order must be 1..4, got %d", eq_order));
    if (!(tau > 0.5)) return bad(msg, fmt("tau must be > 1/2 (or +inf), got %g", tau));
    if (g.nx < 1 || g.ny < 1 || g.nz < 1) return bad(msg, "grid dimensions must be >= 1");
    if (L->D == 2 && g.nz != 1) return bad(msg, fmt("2-D velocity set needs nz = 1, got %d", g.nz));
    const unsigned long long ncell = (unsigned long long)g.nx * g.ny * g.nz;
    if (ncell > 0x7fffffffull) return bad(msg, fmt("grid of %llu cells exceeds 2^31 - 1", ncell));
    const int32_t storage = raw(o.storage), mv = raw(o.move);
    if (storage < LBM_FP64 || storage > LBM_BF16_DEV) return bad(msg, fmt("unknown storage %d", storage));
    if (mv < LBM_MOVE_AUTO || mv > LBM_MOVE_BW2) return bad(msg, fmt("unknown move %d", mv));
    lbm_move m = (lbm_move)mv;
    if (m == LBM_MOVE_AUTO) m = L->on_lattice ? LBM_MOVE_SHIFT : LBM_MOVE_BW2;
    if (m == LBM_MOVE_SHIFT && !L->on_lattice) return bad(msg, "exact shift needs an on-lattice velocity set");
    if (m == LBM_MOVE_BW2) {
        if (L->on_lattice) return bad(msg, "upwind advection is provided for the off-lattice sets");
        if (!(o.cfl > 0.0 && o.cfl <= 1.0)) return bad(msg, fmt("cfl must be in (0, 1], got %g", o.cfl));
        if ((uint64_t)L->Q * (uint64_t)g.nx * (uint64_t)esize >= (1ull << 31))
            return bad(msg, "upwind advection needs a grid row of all populations below 2^31 bytes");
    }
    if (o.check_every < 0) return bad(msg, "check_every must be >= 0");
    if (move) *move = m;
    return LBM_OK;
}

lbm_status check_dev_buf_shape(const lbm_opts &o, uint64_t need, std::string *msg) {
    if (!o.dev_buf[0] || !o.dev_buf[1]) return bad(msg, "dev_buf: give both buffers or neither");
    if (o.dev_buf_bytes < 0 || (uint64_t)o.dev_buf_bytes < need)
        return bad(msg, fmt("dev_buf: %lld bytes per buffer given, the state needs %llu", (long long)o.dev_buf_bytes,
                            (unsigned long long)need));
    const uintptr_t p0 = (uintptr_t)o.dev_buf[0], p1 = (uintptr_t)o.dev_buf[1];
    if ((p0 | p1) & 15u) return bad(msg, "dev_buf: buffers must be 16-byte aligned");
    if ((p0 < p1 ? p1 - p0 : p0 - p1) < need) return bad(msg, "dev_buf: the two buffers overlap");
    return LBM_OK;
}

// ---------------------------------------------------------------- batch plan
double batch_cell_cost(bool on_lattice, int Q) {
    // time per cell of one step, fitted to per-instance runs of one 512-thread workgroup per CU
    // on MI355X (ns): D2Q9 4.0, D2Q37 8.8 (exact shift); D2Q16-GH 9.3, D2Q36-GH 20 (Beam-Warming
    // reads three rows per population and applies two difference stencils), where the fit gave
    // 11.5 and 25: on the 256-instance sweep the plan with the lower Beam-Warming costs runs 4%
    // faster (XCD-local form, 1024 threads), and 25% higher or lower on-lattice costs 4% slower
    return on_lattice ? 2.5 + 0.17 * Q : 0.56 + 0.544 * Q;
}

std::vector<std::vector<uint32_t>> lpt(const std::vector<uint32_t> &items, const std::vector<double> &cost, uint32_t n) {
    std::vector<uint32_t> idx(items);
    std::stable_sort(idx.begin(), idx.end(), [&](uint32_t x, uint32_t y) { return cost[x] > cost[y]; });
    std::vector<double> load(n, 0.0);
    std::vector<std::vector<uint32_t>> lists(n);
    for (uint32_t k : idx) {
        uint32_t best = 0;
        for (uint32_t w = 1; w < n; ++w)
            if (load[w] < load[best]) best = w;
        load[best] += cost[k];
        lists[best].push_back(k);
    }
    for (auto &l : lists) std::sort(l.begin(), l.end());
    return lists;
}

BatchPlan plan_batch(const std::vector<uint32_t> &ncell, const std::vector<double> &per_cell, double per_chunk,
                     uint32_t block, int form, uint32_t resident, uint32_t nxcd) {
    BatchPlan p;
    const uint32_t count = (uint32_t)ncell.size();
    p.inst_first.assign(count + 1, 0);
    std::vector<double> cost;
    for (uint32_t i = 0; i < count; ++i) {
        p.inst_first[i] = (uint32_t)p.chunks.size();
        for (uint32_t s0 = 0; s0 < ncell[i]; s0 += block) {
            const uint32_t n = std::min<uint32_t>(block, ncell[i] - s0);
            p.chunks.push_back(PlanChunk{(int32_t)i, s0, n});
            cost.push_back(per_chunk + per_cell[i] * n);
        }
    }
    p.inst_first[count] = (uint32_t)p.chunks.size();
    const uint32_t nchunks = (uint32_t)p.chunks.size();
    std::vector<std::vector<uint32_t>> lists;
    if (form == 2) {
        std::vector<uint32_t> insts(count);
        std::vector<double> icost(count, 0.0);
        for (uint32_t i = 0; i < count; ++i) {
            insts[i] = i;
            for (uint32_t c = p.inst_first[i]; c < p.inst_first[i + 1]; ++c) icost[i] += cost[c];
        }
        const auto bins = lpt(insts, icost, nxcd);
        size_t most = 1;
        std::vector<std::vector<uint32_t>> xchunks(nxcd);
        for (uint32_t x = 0; x < nxcd; ++x) {
            for (uint32_t i : bins[x])
                for (uint32_t c = p.inst_first[i]; c < p.inst_first[i + 1]; ++c) xchunks[x].push_back(c);
            most = std::max(most, xchunks[x].size());
        }
        p.per_xcd = (uint32_t)std::min<size_t>(most, std::max<uint32_t>(1u, resident / nxcd));
        p.nwg = p.per_xcd * nxcd;
        for (uint32_t x = 0; x < nxcd; ++x) {
            auto part = lpt(xchunks[x], cost, p.per_xcd);
            for (auto &l : part) lists.push_back(std::move(l));
        }
    } else {
        p.nwg = std::min<uint32_t>(nchunks, resident);
        std::vector<uint32_t> all(nchunks);
        for (uint32_t k = 0; k < nchunks; ++k) all[k] = k;
        lists = lpt(all, cost, p.nwg);
    }
    p.wg_first.assign(p.nwg + 1, 0);
    for (uint32_t w = 0; w < p.nwg; ++w) {
        p.wg_first[w] = (uint32_t)p.wg_chunks.size();
        p.wg_chunks.insert(p.wg_chunks.end(), lists[w].begin(), lists[w].end());
    }
    p.wg_first[p.nwg] = (uint32_t)p.wg_chunks.size();
    return p;
}

namespace {

// Solve the k x k system M z = r in place (Gaussian elimination, partial pivoting); false if a
// pivot is below tol times the largest diagonal entry (the support set is rank-deficient).
bool solve_small(std::vector<double> &M, std::vector<double> &r, int k, double tol) {
    double scale = 0;
    for (int i = 0; i < k; ++i) scale = std::max(scale, fabs(M[i * k + i]));
    if (!(scale > 0)) return false;
    for (int c = 0; c < k; ++c) {
        int piv = c;
        for (int i = c + 1; i < k; ++i)
            if (fabs(M[i * k + c]) > fabs(M[piv * k + c])) piv = i;
        if (!(fabs(M[piv * k + c]) > tol * scale)) return false;
        if (piv != c) {
            for (int j = 0; j < k; ++j) std::swap(M[c * k + j], M[piv * k + j]);
            std::swap(r[c], r[piv]);
        }
        for (int i = c + 1; i < k; ++i) {
            const double f = M[i * k + c] / M[c * k + c];
            for (int j = c; j < k; ++j) M[i * k + j] -= f * M[c * k + j];
            r[i] -= f * r[c];
        }
    }
    for (int c = k - 1; c >= 0; --c) {
        double v = r[c];
        for (int j = c + 1; j < k; ++j) v -= M[c * k + j] * r[j];
        r[c] = v / M[c * k + c];
    }
    return true;
}

}  // namespace

std::vector<double> nnls_small(const std::vector<double> &A, int m, int n, const std::vector<double> &y) {
    std::vector<double> best(n, 0.0);
    if (n < 1 || n > 8 || m < 1 || (int)A.size() != m * n || (int)y.size() != m) return best;
    // normal equations once: G = A^T A, h = A^T y
    std::vector<double> G(n * n, 0.0), h(n, 0.0);
    for (int r = 0; r < m; ++r)
        for (int i = 0; i < n; ++i) {
            h[i] += A[r * n + i] * y[r];
            for (int j = 0; j < n; ++j) G[i * n + j] += A[r * n + i] * A[r * n + j];
        }
    // equilibrate: columns of unit norm (cells per workgroup and chunk counts differ by ~10^3);
    // an all-zero column is left out of every support
    std::vector<double> sc(n, 0.0);
    for (int i = 0; i < n; ++i) sc[i] = G[i * n + i] > 0 ? sqrt(G[i * n + i]) : 0.0;
    for (int i = 0; i < n; ++i) {
        h[i] = sc[i] > 0 ? h[i] / sc[i] : 0.0;
        for (int j = 0; j < n; ++j) G[i * n + j] = (sc[i] > 0 && sc[j] > 0) ? G[i * n + j] / (sc[i] * sc[j]) : 0.0;
    }
    auto residual = [&](const std::vector<double> &x) {
        double s = 0;
        for (int r = 0; r < m; ++r) {
            double v = -y[r];
            for (int i = 0; i < n; ++i) v += A[r * n + i] * x[i];
            s += v * v;
        }
        return s;
    };
    double best_res = residual(best);   // the empty support: x = 0
    for (unsigned mask = 1; mask < (1u << n); ++mask) {
        std::vector<int> idx;
        bool zero_col = false;
        for (int i = 0; i < n; ++i)
            if (mask & (1u << i)) {
                idx.push_back(i);
                zero_col = zero_col || sc[i] == 0.0;
            }
        if (zero_col) continue;
        const int k = (int)idx.size();
        std::vector<double> M(k * k), r(k);
        for (int a = 0; a < k; ++a) {
            r[a] = h[idx[a]];
            for (int c = 0; c < k; ++c) M[a * k + c] = G[idx[a] * n + idx[c]];
        }
        if (!solve_small(M, r, k, 1e-9)) continue;
        if (std::any_of(r.begin(), r.end(), [](double v) { return !(v >= 0); })) continue;
        std::vector<double> x(n, 0.0);
        for (int a = 0; a < k; ++a) x[idx[a]] = r[a] / sc[idx[a]];
        const double res = residual(x);
        if (res < best_res) {
            best_res = res;
            best = x;
        }
    }
    return best;
}

std::vector<double> fit_chunk_costs(const BatchPlan &p, const std::vector<int> &kind, int nkinds,
                                    const std::vector<double> &work) {
    const int n = nkinds + 1, m = (int)p.nwg;
    if (nkinds < 1 || n > 8 || (int)work.size() != m || m < 1) return std::vector<double>(std::max(n, 1), 0.0);
    std::vector<double> A((size_t)m * n, 0.0);
    for (int w = 0; w < m; ++w)
        for (uint32_t j = p.wg_first[w]; j < p.wg_first[w + 1]; ++j) {
            const PlanChunk &c = p.chunks[p.wg_chunks[j]];
            A[(size_t)w * n + kind[c.inst]] += c.count;
            A[(size_t)w * n + nkinds] += 1.0;
        }
    std::vector<double> x = nnls_small(A, m, n, work);
    // No chunk may cost nothing: longest-processing-time-first would pile every free chunk onto
    // one workgroup.  Floor the per-cell costs at 1% of the largest and the per-chunk cost at 1%
    // of the mean measured time per chunk.
    double top = 0, chunks = 0, total = 0;
    for (int k = 0; k < nkinds; ++k) top = std::max(top, x[k]);
    for (int w = 0; w < m; ++w) {
        chunks += A[(size_t)w * n + nkinds];
        total += work[w];
    }
    if (top <= 0 && x[nkinds] <= 0) return std::vector<double>(n, 0.0);
    for (int k = 0; k < nkinds; ++k) x[k] = std::max(x[k], 0.01 * top);
    if (chunks > 0) x[nkinds] = std::max(x[nkinds], 0.01 * total / chunks);
    return x;
}

// ---------------------------------------------------------------- autotuner cache
std::string tune_key(const char *arch, int lattice, int order, int storage, int sr, const StepShape &s) {
    std::string a;
    for (const char *c = arch ? arch : "unknown"; *c; ++c) {
        const char ch = *c;
        const bool ok = (ch >= 'a' && ch <= 'z') || (ch >= 'A' && ch <= 'Z') || (ch >= '0' && ch <= '9') ||
                        ch == ':' || ch == '+' || ch == '-' || ch == '_' || ch == '.';
        a.push_back(ok ? ch : '_');
    }
    const uint64_t rows = (uint64_t)s.ny * (uint64_t)s.nz;
    return a + fmt("|lat%d|N%d|st%d|sr%d|%s|%s|nx2^%d|rows2^%d|%s", lattice, order, storage, sr, s.bw2 ? "bw2" : "shift",
                   s.forced ? "forced" : "free", ceil_log2((uint64_t)s.nx), ceil_log2(rows),
                   s.nx % 256 == 0 ? "nx256" : "nxany");
}

std::string tile_shape(const StepShape &s, int tile) {
    int block = 0, cpt = 0, vw = 0;
    bool nt = false;
    tile_launch(s, tile, &block, &cpt, &vw, &nt);
    if (s.bw2) return fmt("bw2:%dx%d:v%d%s", block, kBWTiles[tile].rows, kBWTiles[tile].variant, nt ? ":nt" : "");
    if (s.rows_ok) return fmt("rows:%dx%d:w%d%s", block, cpt, vw, nt ? ":nt" : "");
    return "cells:256";
}

std::string tune_format(const TuneEntry &e) {
    // key and shape may be longer than fmt's buffer: concatenate them
    return "{\"key\": \"" + e.key + "\", \"tile\": " + std::to_string(e.tile) + ", \"shape\": \"" + e.shape +
           "\", \"ms\": " + fmt("%.6g", e.ms) + "}";
}

namespace {

bool field_str(const std::string &line, const char *name, std::string *out) {
    const std::string pat = std::string("\"") + name + "\": \"";
    const size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    const size_t b = p + pat.size(), q = line.find('"', b);
    if (q == std::string::npos) return false;
    *out = line.substr(b, q - b);
    return true;
}

bool field_num(const std::string &line, const char *name, double *out) {
    const std::string pat = std::string("\"") + name + "\": ";
    const size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    const char *s = line.c_str() + p + pat.size();
    char *end = nullptr;
    const double v = strtod(s, &end);
    if (end == s || !isfinite(v)) return false;
    *out = v;
    return true;
}

}  // namespace

bool tune_parse(const std::string &line, TuneEntry *out) {
    TuneEntry e;
    double t = 0, ms = 0;
    if (!field_str(line, "key", &e.key) || e.key.empty()) return false;
    if (!field_num(line, "tile", &t) || t < 0 || t > 1e6 || t != floor(t)) return false;
    if (!field_str(line, "shape", &e.shape)) return false;
    if (!field_num(line, "ms", &ms) || ms < 0) return false;
    e.tile = (int)t;
    e.ms = ms;
    *out = e;
    return true;
}

bool tune_read(const std::string &path, std::vector<TuneEntry> *out) {
    out->clear();
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return access(path.c_str(), F_OK) != 0;   // missing: an empty cache
    std::string line;
    char buf[1024];
    bool ok = true;
    while (fgets(buf, sizeof buf, f)) {
        line += buf;
        if (line.empty() || line.back() != '\n') {
            if (!feof(f)) continue;   // a line longer than the buffer: keep reading it
        }
        TuneEntry e;
        if (tune_parse(line, &e)) out->push_back(e);
        line.clear();
    }
    if (!line.empty()) {
        TuneEntry e;
        if (tune_parse(line, &e)) out->push_back(e);
    }
    if (ferror(f)) ok = false;
    fclose(f);
    return ok;
}

bool tune_lookup(const std::string &path, const std::string &key, TuneEntry *out) {
    std::vector<TuneEntry> all;
    if (!tune_read(path, &all)) return false;
    for (auto it = all.rbegin(); it != all.rend(); ++it)
        if (it->key == key) {
            *out = *it;
            return true;
        }
    return false;
}

bool tune_store(const std::string &path, const TuneEntry &e, std::string *err) {
    std::vector<TuneEntry> all;
    if (!tune_read(path, &all)) {
        if (err) *err = "cannot read " + path;
        return false;
    }
    std::vector<TuneEntry> keep;
    for (const auto &x : all)
        if (x.key != e.key) keep.push_back(x);
    keep.push_back(e);
    static std::atomic<unsigned> serial{0};
    const std::string tmp = fmt("%s.tmp.%ld.%u", path.c_str(), (long)getpid(), serial.fetch_add(1));
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) {
        if (err) *err = "cannot write " + tmp;
        return false;
    }
    bool ok = true;
    for (const auto &x : keep) ok = ok && fprintf(f, "%s\n", tune_format(x).c_str()) > 0;
    ok = (fclose(f) == 0) && ok;
    if (ok && rename(tmp.c_str(), path.c_str()) != 0) ok = false;
    if (!ok) {
        (void)remove(tmp.c_str());
        if (err) *err = "cannot replace " + path;
    }
    return ok;
}

}  // namespace host
}  // namespace lbm
