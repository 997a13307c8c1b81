// Checks of the runtime's host-only logic (paper_0908_4520_amd/csrc/host_logic.cpp), built with
// the address and undefined-behaviour sanitizers by tests/test_sanitizers_cpu.py:
//  - the step launch geometry of every tile covers the grid exactly once and fits the kernels'
//    32-bit indices, at the benchmark shapes (4096^2 shift, 2048^2 Beam-Warming, 512^3 D3Q39) and
//    at the largest grids the library accepts;
//  - argument validation accepts the valid configurations and names every invalid one;
//  - the batch plan deals every chunk to exactly one workgroup, keeps an instance's chunks on one
//    XCD in the XCD-local form, stays within the resident workgroups and balances the modelled
//    cost to within one chunk;
//  - the autotuner cache round-trips entries, replaces by key, skips damaged lines and leaves no
//    temporary files behind.
// argv[1]: a scratch directory for the cache files.  Exit status 0 only if every check passes.
#include <dirent.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "host_logic.h"
#include "lattices.inc"

using namespace lbm;
using namespace lbm::host;

static int failures = 0;

static void check(bool ok, const std::string &what) {
    if (!ok) {
        printf("FAIL %s\n", what.c_str());
        ++failures;
    }
}

template <class L>
static LatShape shape_of() {
    return LatShape{L::Q, L::D, L::R, L::on_lattice};
}

// ---------------------------------------------------------------- launch geometry
static void geometry_case(const char *name, const LatShape &L, lbm_grid g, int esize, bool forced, bool vec_kernel) {
    const bool bw2 = !L.on_lattice;
    StepShape s{};
    s.bw2 = bw2;
    s.rows_ok = row_tiles_ok(!bw2, L.Q, L.D, L.R, g, esize);
    s.forced = forced;
    s.vector_ok = vec_kernel && g.nx % 256 == 0;
    s.nx = g.nx;
    s.ny = g.ny;
    s.nz = g.nz;
    const int n = tile_count(s);
    check(n >= 1, std::string(name) + ": no tiles");
    const uint64_t ncell = (uint64_t)g.nx * g.ny * g.nz;
    for (int t = 0; t < n; ++t) {
        const StepGeom geo = step_geometry(s, t);
        int block = 0, cpt = 0, vw = 0;
        bool nt = false;
        tile_launch(s, t, &block, &cpt, &vw, &nt);
        char what[256];
        snprintf(what, sizeof what, "%s tile %d (block %d, cells/thread %d, blocks %u)", name, t, block, cpt, geo.nblocks);
        check(geo.nblocks >= 1, std::string(what) + ": empty grid");
        if (bw2) {
            // strips of H rows by 256 columns: every (column, row) in exactly one block
            const uint64_t cols = (uint64_t)geo.per_row * 256, strips = (uint64_t)geo.nblocks / geo.per_row;
            check(geo.nblocks % geo.per_row == 0, std::string(what) + ": partial strip row");
            check(cols >= (uint64_t)g.nx && cols < (uint64_t)g.nx + 256, std::string(what) + ": columns");
            check(strips * geo.tile >= (uint64_t)g.ny && (strips - 1) * geo.tile < (uint64_t)g.ny,
                  std::string(what) + ": strips");
        } else if (s.rows_ok) {
            const uint64_t per_block = (uint64_t)block * (uint64_t)cpt;
            check(geo.per_row * per_block >= (uint64_t)g.nx && (geo.per_row - 1) * per_block < (uint64_t)g.nx,
                  std::string(what) + ": row coverage");
            check((uint64_t)geo.nblocks == (uint64_t)geo.per_row * g.ny * g.nz, std::string(what) + ": rows");
            // the kernels index a row's populations with 32-bit byte offsets
            check((uint64_t)L.Q * g.nx * esize < (1ull << 31), std::string(what) + ": row bytes");
        } else {
            check((uint64_t)geo.nblocks * kCellBlock >= ncell && ((uint64_t)geo.nblocks - 1) * kCellBlock < ncell,
                  std::string(what) + ": cell coverage");
        }
        // grid size in threads fits the 32-bit global index the kernels compute
        check((uint64_t)geo.nblocks * (uint64_t)block < (1ull << 32), std::string(what) + ": 32-bit thread index");
        const std::string sh = tile_shape(s, t);
        check(!sh.empty() && sh.find('"') == std::string::npos, std::string(what) + ": shape string");
    }
}

static void geometry_checks() {
    geometry_case("D2Q37 4096^2 fp32", shape_of<D2Q37>(), {4096, 4096, 1}, 4, false, true);
    geometry_case("D2Q37 4096^2 fp32 forced", shape_of<D2Q37>(), {4096, 4096, 1}, 4, true, true);
    geometry_case("D2Q37 4096^2 fp64", shape_of<D2Q37>(), {4096, 4096, 1}, 8, false, false);
    geometry_case("D2Q16-GH 2048^2 fp32", shape_of<D2Q16_GH>(), {2048, 2048, 1}, 4, false, false);
    geometry_case("D2Q36-GH 2048^2 fp32 forced", shape_of<D2Q36_GH>(), {2048, 2048, 1}, 4, true, false);
    geometry_case("D3Q39 512^3 fp32", shape_of<D3Q39>(), {512, 512, 512}, 4, false, true);
    geometry_case("D3Q39 512^3 bf16", shape_of<D3Q39>(), {512, 512, 512}, 2, false, false);
    geometry_case("D2Q9 4x64 fp64", shape_of<D2Q9>(), {4, 64, 1}, 8, false, false);
    geometry_case("D2Q9 300x7 ragged", shape_of<D2Q9>(), {300, 7, 1}, 8, false, false);
    geometry_case("D2Q25-CK 1000x3 (ny < R)", shape_of<D2Q25_CK>(), {1000, 3, 1}, 4, false, true);
    geometry_case("D2Q16-GH 1x1", shape_of<D2Q16_GH>(), {1, 1, 1}, 4, false, false);
    geometry_case("D2Q16-GH 257x3 ragged", shape_of<D2Q16_GH>(), {257, 3, 1}, 4, false, false);
    // the largest grids the library accepts: 2^31 - 1 cells
    geometry_case("D2Q9 65536x32767 fp32", shape_of<D2Q9>(), {65536, 32767, 1}, 4, false, true);
    geometry_case("D2Q9 2147483647x1 fp64", shape_of<D2Q9>(), {2147483647, 1, 1}, 8, false, false);
    geometry_case("D3Q39 1290x1290x1290", shape_of<D3Q39>(), {1290, 1290, 1290}, 2, false, false);
    geometry_case("D2Q16-GH 1048576x2047 fp32", shape_of<D2Q16_GH>(), {1048576, 2047, 1}, 4, false, false);
}

// ---------------------------------------------------------------- validation
static void validation_checks() {
    lbm_opts o{};
    o.storage = LBM_FP32_DEV;
    o.move = LBM_MOVE_AUTO;
    o.cfl = 0.5;
    const LatShape q37 = shape_of<D2Q37>(), q39 = shape_of<D3Q39>(), gh16 = shape_of<D2Q16_GH>();
    std::string msg;
    lbm_move mv = LBM_MOVE_AUTO;
    check(check_init(&q37, 4, 0.8, {4096, 4096, 1}, o, 4, &mv, &msg) == LBM_OK && mv == LBM_MOVE_SHIFT, "valid D2Q37");
    check(check_init(&gh16, 3, INFINITY, {2048, 2048, 1}, o, 4, &mv, &msg) == LBM_OK && mv == LBM_MOVE_BW2,
          "valid D2Q16-GH collisionless");
    check(check_init(&q39, 4, 0.6, {512, 512, 512}, o, 2, &mv, &msg) == LBM_OK, "valid D3Q39");
    struct Bad {
        const LatShape *L;
        int N;
        double tau;
        lbm_grid g;
        int storage, move;
        double cfl;
        int check_every, esize;
        const char *expect;
    };
    const Bad bad[] = {
        {nullptr, 2, 0.8, {4, 4, 1}, 2, 0, 0.5, 0, 4, "unknown lattice"},
        {&q37, 0, 0.8, {4, 4, 1}, 2, 0, 0.5, 0, 4, "eq_order"},
        {&q37, 5, 0.8, {4, 4, 1}, 2, 0, 0.5, 0, 4, "eq_order"},
        {&q37, 2, 0.5, {4, 4, 1}, 2, 0, 0.5, 0, 4, "tau"},
        {&q37, 2, NAN, {4, 4, 1}, 2, 0, 0.5, 0, 4, "tau"},
        {&q37, 2, 0.8, {0, 4, 1}, 2, 0, 0.5, 0, 4, "grid dimensions"},
        {&q37, 2, 0.8, {4, -1, 1}, 2, 0, 0.5, 0, 4, "grid dimensions"},
        {&q37, 2, 0.8, {4, 4, 2}, 2, 0, 0.5, 0, 4, "nz = 1"},
        {&q39, 2, 0.8, {2048, 2048, 512}, 2, 0, 0.5, 0, 4, "exceeds 2^31"},
        {&q37, 2, 0.8, {4, 4, 1}, 9, 0, 0.5, 0, 4, "unknown storage"},
        {&q37, 2, 0.8, {4, 4, 1}, -1, 0, 0.5, 0, 4, "unknown storage"},
        {&gh16, 2, 0.8, {4, 4, 1}, 2, 1, 0.5, 0, 4, "on-lattice"},
        {&q37, 2, 0.8, {4, 4, 1}, 2, 2, 0.5, 0, 4, "off-lattice"},
        {&gh16, 2, 0.8, {4, 4, 1}, 2, 0, 0.0, 0, 4, "cfl"},
        {&gh16, 2, 0.8, {4, 4, 1}, 2, 0, 1.5, 0, 4, "cfl"},
        {&gh16, 2, 0.8, {4, 4, 1}, 2, 0, NAN, 0, 4, "cfl"},
        {&gh16, 2, 0.8, {33554432, 1, 1}, 2, 0, 0.5, 0, 4, "2^31 bytes"},
        {&q37, 2, 0.8, {4, 4, 1}, 2, 7, 0.5, 0, 4, "unknown move"},
        {&q37, 2, 0.8, {4, 4, 1}, 2, 0, 0.5, -1, 4, "check_every"},
    };
    for (const Bad &b : bad) {
        lbm_opts x = o;
        // as a C caller passes them: plain ints, possibly outside the enumerations
        const int32_t st_raw = b.storage, mv_raw = b.move;
        memcpy(&x.storage, &st_raw, sizeof st_raw);
        memcpy(&x.move, &mv_raw, sizeof mv_raw);
        x.cfl = b.cfl;
        x.check_every = b.check_every;
        msg.clear();
        const lbm_status st = check_init(b.L, b.N, b.tau, b.g, x, storage_bytes(x), &mv, &msg);
        check(st == LBM_EINVAL && msg.find(b.expect) != std::string::npos,
              std::string("invalid case not named '") + b.expect + "': got '" + msg + "'");
    }
    // dev_buf shape checks (the device memory type is checked by the runtime)
    alignas(16) static char pool[4096];
    lbm_opts d = o;
    d.dev_buf[0] = pool;
    d.dev_buf[1] = pool + 2048;
    d.dev_buf_bytes = 2048;
    check(check_dev_buf_shape(d, 2048, &msg) == LBM_OK, "dev_buf valid");
    check(check_dev_buf_shape(d, 2049, &msg) == LBM_EINVAL && msg.find("needs") != std::string::npos, "dev_buf small");
    d.dev_buf_bytes = 4096;
    check(check_dev_buf_shape(d, 4096, &msg) == LBM_EINVAL && msg.find("overlap") != std::string::npos, "dev_buf overlap");
    d.dev_buf[1] = pool + 8;
    d.dev_buf_bytes = 8;
    check(check_dev_buf_shape(d, 8, &msg) == LBM_EINVAL && msg.find("aligned") != std::string::npos, "dev_buf alignment");
    d.dev_buf[1] = nullptr;
    check(check_dev_buf_shape(d, 8, &msg) == LBM_EINVAL && msg.find("both") != std::string::npos, "dev_buf one given");
    d.dev_buf[1] = pool + 16;
    d.dev_buf_bytes = -1;
    check(check_dev_buf_shape(d, 8, &msg) == LBM_EINVAL, "dev_buf negative size");
}

// ---------------------------------------------------------------- batch plan
static void plan_case(const char *name, const std::vector<uint32_t> &ncell, const std::vector<double> &per_cell,
                      uint32_t block, int form, uint32_t resident, uint32_t nxcd, double per_chunk = 0.0) {
    const BatchPlan p = plan_batch(ncell, per_cell, per_chunk, block, form, resident, form == 2 ? nxcd : 1);
    char what[256];
    snprintf(what, sizeof what, "%s block %u form %d resident %u xcds %u", name, block, form, resident, nxcd);
    const std::string w = what;
    const uint32_t nch = (uint32_t)p.chunks.size();
    check(p.inst_first.size() == ncell.size() + 1 && p.inst_first.back() == nch, w + ": inst_first");
    for (size_t i = 0; i < ncell.size(); ++i) {
        uint32_t next = 0;
        for (uint32_t k = p.inst_first[i]; k < p.inst_first[i + 1]; ++k) {
            const PlanChunk &c = p.chunks[k];
            check(c.inst == (int32_t)i && c.start == next && c.count >= 1 && c.count <= block, w + ": chunk layout");
            next += c.count;
        }
        check(next == ncell[i], w + ": instance cells covered");
    }
    check(p.nwg >= 1 && p.wg_first.size() == (size_t)p.nwg + 1 && p.wg_first[0] == 0 &&
              p.wg_first.back() == p.wg_chunks.size(),
          w + ": wg_first");
    for (uint32_t g = 0; g < p.nwg; ++g) check(p.wg_first[g] <= p.wg_first[g + 1], w + ": wg_first monotone");
    std::vector<int> seen(nch, 0);
    for (uint32_t k : p.wg_chunks) {
        check(k < nch, w + ": chunk index");
        if (k < nch) ++seen[k];
    }
    check(std::all_of(seen.begin(), seen.end(), [](int v) { return v == 1; }), w + ": every chunk exactly once");
    if (form == 2) {
        check(p.nwg == p.per_xcd * nxcd && p.per_xcd >= 1 && p.per_xcd <= std::max(1u, resident / nxcd),
              w + ": XCD slots");
        std::vector<int> xcd_of(ncell.size(), -1);
        for (uint32_t g = 0; g < p.nwg; ++g)
            for (uint32_t j = p.wg_first[g]; j < p.wg_first[g + 1]; ++j) {
                const int i = p.chunks[p.wg_chunks[j]].inst, x = (int)(g / p.per_xcd);
                check(xcd_of[i] < 0 || xcd_of[i] == x, w + ": instance split over XCDs");
                xcd_of[i] = x;
            }
    } else {
        check(p.nwg <= resident && p.nwg <= nch, w + ": workgroups");
        // LPT: the busiest workgroup carries at most the mean plus one chunk
        std::vector<double> load(p.nwg, 0.0);
        double total = 0, largest = 0;
        for (uint32_t g = 0; g < p.nwg; ++g)
            for (uint32_t j = p.wg_first[g]; j < p.wg_first[g + 1]; ++j) {
                const PlanChunk &c = p.chunks[p.wg_chunks[j]];
                const double cost = per_chunk + per_cell[c.inst] * c.count;
                load[g] += cost;
                total += cost;
                largest = std::max(largest, cost);
            }
        const double busiest = *std::max_element(load.begin(), load.end());
        check(busiest <= total / p.nwg + largest * (1 + 1e-12), w + ": balance");
    }
}

static void plan_checks() {
    // a sweep like the benchmark's: 256 instances, nx 4, ny in [32, 1024], four velocity sets
    unsigned long long st = 12345;
    auto next = [&]() {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        return (uint32_t)(st >> 33);
    };
    const double cost[4] = {batch_cell_cost(true, 9), batch_cell_cost(true, 37), batch_cell_cost(false, 16),
                            batch_cell_cost(false, 36)};
    std::vector<uint32_t> ncell;
    std::vector<double> pc;
    for (int i = 0; i < 256; ++i) {
        ncell.push_back(4 * (32 + next() % 993));
        pc.push_back(cost[next() % 4]);
    }
    for (uint32_t block : {256u, 512u, 1024u})
        for (uint32_t resident : {256u, 512u, 768u}) {
            plan_case("sweep", ncell, pc, block, 1, resident, 8);
            plan_case("sweep", ncell, pc, block, 2, resident, 8);
        }
    plan_case("sweep on 3 XCDs", ncell, pc, 512, 2, 256, 3);
    plan_case("sweep, chunk cost", ncell, pc, 512, 1, 256, 8, 2000.0);
    plan_case("sweep, chunk cost", ncell, pc, 256, 2, 768, 8, 2000.0);
    plan_case("sweep on 1 XCD", ncell, pc, 512, 2, 256, 1);
    // degenerate batches
    plan_case("one cell", {1}, {1.0}, 256, 1, 256, 8);
    plan_case("one cell", {1}, {1.0}, 256, 2, 256, 8);
    plan_case("exact multiples", {512, 1024, 256}, {1.0, 2.0, 3.0}, 256, 1, 4, 8);
    plan_case("one resident workgroup per XCD", {300, 300, 300}, {1.0, 1.0, 1.0}, 256, 2, 8, 8);
    plan_case("largest instance", {1u << 26, 100}, {1.0, 5.0}, 1024, 1, 2048, 8);
    plan_case("largest instance", {1u << 26, 100}, {1.0, 5.0}, 1024, 2, 2048, 8);
}

// ---------------------------------------------------------------- cost fit
static void fit_checks() {
    // exact non-negative solution is recovered
    {
        const int m = 40, n = 4;
        std::vector<double> A(m * n), y(m);
        const double x0[4] = {3.0, 0.5, 0.0, 7.0};
        unsigned long long st = 7;
        for (int r = 0; r < m; ++r) {
            y[r] = 0;
            for (int i = 0; i < n; ++i) {
                st = st * 6364136223846793005ull + 1442695040888963407ull;
                A[r * n + i] = (double)(st >> 40) * (i == 3 ? 1e-3 : 1.0);   // very different column scales
                y[r] += A[r * n + i] * x0[i];
            }
        }
        const std::vector<double> x = nnls_small(A, m, n, y);
        double err = 0;
        for (int i = 0; i < n; ++i) err = std::max(err, fabs(x[i] - x0[i]));
        check(err < 1e-6, "nnls recovers an exact non-negative solution");
    }
    // the unconstrained least-squares solution has a negative entry: KKT conditions hold
    {
        const std::vector<double> A = {1, 0, 0, 1, 1, 1};   // 3 x 2
        const std::vector<double> y = {1, -1, 0.2};
        const std::vector<double> x = nnls_small(A, 3, 2, y);
        // optimum: x1 = 0, x0 minimises (x0-1)^2 + 1 + (x0-0.2)^2 -> x0 = 0.6
        check(fabs(x[0] - 0.6) < 1e-12 && x[1] == 0.0, "nnls clamps a negative coefficient");
        // gradient A^T (A x - y) is zero on the support and >= 0 off it
        const double g1 = (x[0] * 0 + x[1] - y[1]) + (x[0] + x[1] - y[2]);
        check(g1 >= 0, "nnls KKT");
    }
    // a zero column gets 0; a collinear pair is handled
    {
        const std::vector<double> A = {1, 0, 2, 2, 0, 4, 3, 0, 6};   // columns: c, 0, 2c
        const std::vector<double> y = {2, 4, 6};
        const std::vector<double> x = nnls_small(A, 3, 3, y);
        check(x[1] == 0.0 && fabs(x[0] + 2 * x[2] - 2.0) < 1e-9 && x[0] >= 0 && x[2] >= 0, "nnls zero and collinear columns");
    }
    check(nnls_small({}, 0, 3, {}).size() == 3, "nnls empty input");
    // fit_chunk_costs recovers the costs that generated the workgroup times
    {
        std::vector<uint32_t> ncell;
        std::vector<double> pc;
        std::vector<int> kind;
        unsigned long long st = 99;
        for (int i = 0; i < 64; ++i) {
            st = st * 6364136223846793005ull + 1442695040888963407ull;
            ncell.push_back(100 + (uint32_t)((st >> 33) % 3000));
            kind.push_back((int)((st >> 20) % 3));
            pc.push_back(1.0);
        }
        const BatchPlan p = plan_batch(ncell, pc, 0.0, 256, 1, 48, 1);
        const double truth[4] = {0.004, 0.010, 0.025, 2.0};
        std::vector<double> work(p.nwg, 0.0);
        for (uint32_t w = 0; w < p.nwg; ++w)
            for (uint32_t j = p.wg_first[w]; j < p.wg_first[w + 1]; ++j) {
                const PlanChunk &c = p.chunks[p.wg_chunks[j]];
                work[w] += truth[3] + truth[kind[c.inst]] * c.count;
            }
        const std::vector<double> x = fit_chunk_costs(p, kind, 3, work);
        double err = 0;
        for (int i = 0; i < 4; ++i) err = std::max(err, fabs(x[i] - truth[i]) / truth[i]);
        check(x.size() == 4 && err < 1e-6, "fit_chunk_costs recovers the generating costs");
        // times that only the cells of kind 2 explain: the other costs are floored, not zero,
        // and a plan with them spreads the chunks (no workgroup takes all the cheap ones)
        std::vector<double> w2(p.nwg, 0.0);
        for (uint32_t w = 0; w < p.nwg; ++w)
            for (uint32_t j = p.wg_first[w]; j < p.wg_first[w + 1]; ++j) {
                const PlanChunk &c = p.chunks[p.wg_chunks[j]];
                if (kind[c.inst] == 2) w2[w] += 0.02 * c.count;
            }
        const std::vector<double> y = fit_chunk_costs(p, kind, 3, w2);
        check(y[0] > 0 && y[1] > 0 && y[3] > 0 && y[2] >= 50 * std::max(y[0], y[1]), "fitted costs are floored");
        check(fit_chunk_costs(p, kind, 3, std::vector<double>(p.nwg, 0.0))[3] == 0.0, "nothing to fit: all zero");
    }
}

// ---------------------------------------------------------------- autotuner cache
static size_t count_files(const std::string &dir, const std::string &prefix) {
    size_t n = 0;
    if (DIR *d = opendir(dir.c_str())) {
        while (dirent *e = readdir(d))
            if (std::string(e->d_name).rfind(prefix, 0) == 0) ++n;
        closedir(d);
    }
    return n;
}

static void cache_checks(const std::string &dir) {
    const std::string path = dir + "/tune.jsonl";
    remove(path.c_str());
    TuneEntry e;
    check(!tune_lookup(path, "any", &e), "missing cache file is empty");
    StepShape s{};
    s.rows_ok = true;
    s.vector_ok = true;
    s.nx = s.ny = 4096;
    s.nz = 1;
    const std::string k1 = tune_key("gfx950:sramecc+:xnack-", 2, 4, 2, 0, s);
    StepShape s3 = s;
    s3.nx = s3.ny = s3.nz = 512;
    const std::string k2 = tune_key("gfx950:sramecc+:xnack-", 3, 4, 4, 1, s3);
    const std::string k3 = tune_key("weird\"arch\\name", 1, 2, 0, 0, s);
    const std::string long_arch(2000, 'g');
    check(tune_key(long_arch.c_str(), 1, 2, 0, 0, s).size() > 2000, "long architecture names are kept whole");
    check(k1 != k2 && k3.find('"') == std::string::npos && k3.find('\\') == std::string::npos, "keys");
    StepShape s_same = s;
    s_same.nx = 3000;   // same class as 4096 (ceil log2 12) but not a multiple of 256
    check(tune_key("gfx950", 2, 4, 2, 0, s_same) != tune_key("gfx950", 2, 4, 2, 0, s), "nx % 256 in the key");
    s_same.nx = 4000 / 256 * 256;
    check(tune_key("gfx950", 2, 4, 2, 0, s_same) == tune_key("gfx950", 2, 4, 2, 0, s), "grid class shares a key");
    std::string err;
    check(tune_store(path, TuneEntry{k1, 6, tile_shape(s, 6), 0.8318}, &err), "store 1: " + err);
    check(tune_store(path, TuneEntry{k2, 8, tile_shape(s3, 8), 3.5}, &err), "store 2: " + err);
    check(tune_store(path, TuneEntry{k3, 0, "cells:256", 0.0024}, &err), "store 3: " + err);
    check(tune_lookup(path, k1, &e) && e.tile == 6 && e.shape == tile_shape(s, 6) && fabs(e.ms - 0.8318) < 1e-9, "lookup 1");
    check(tune_lookup(path, k2, &e) && e.tile == 8, "lookup 2");
    check(tune_store(path, TuneEntry{k1, 5, tile_shape(s, 5), 0.84}, &err), "replace 1: " + err);
    check(tune_lookup(path, k1, &e) && e.tile == 5, "replaced entry wins");
    std::vector<TuneEntry> all;
    check(tune_read(path, &all) && all.size() == 3, "one line per key after a replace");
    // damaged lines are skipped, long lines are read whole
    if (FILE *f = fopen(path.c_str(), "a")) {
        fputs("garbage\n{\"key\": \"x\", \"tile\": -3, \"shape\": \"s\", \"ms\": 1}\n{\"key\": \"trunc", f);
        fputs("\n{\"key\": \"", f);
        for (int i = 0; i < 3000; ++i) fputc('k', f);
        fputs("\", \"tile\": 2, \"shape\": \"s\", \"ms\": 1.5}\n{\"key\": \"nan\", \"tile\": 1, \"shape\": \"s\", \"ms\": nan}", f);
        fclose(f);
    }
    check(tune_read(path, &all) && all.size() == 4, "damaged lines skipped, long line kept");
    check(tune_lookup(path, std::string(3000, 'k'), &e) && e.tile == 2, "long key");
    check(tune_store(path, TuneEntry{k2, 9, tile_shape(s3, 9), 3.4}, &err), "store after damage: " + err);
    check(tune_read(path, &all) && all.size() == 4, "rewrite drops damaged lines");
    check(count_files(dir, "tune.jsonl.tmp") == 0, "no temporary files left");
    check(!tune_store(dir + "/no/such/dir/tune.jsonl", TuneEntry{k1, 1, "x", 1}, &err) && !err.empty(),
          "unwritable path reports an error");
    check(!tune_read(dir, &all), "a directory is not a readable cache");
    TuneEntry p;
    check(tune_parse(tune_format(TuneEntry{"a|b", 3, "rows:256x4:w1:nt", 1.25}), &p) && p.key == "a|b" && p.tile == 3 &&
              p.shape == "rows:256x4:w1:nt" && p.ms == 1.25,
          "format/parse round trip");
    check(!tune_parse("{\"key\": \"a\", \"tile\": 2.5, \"shape\": \"s\", \"ms\": 1}", &p), "fractional tile rejected");
    check(!tune_parse("{\"key\": \"\", \"tile\": 2, \"shape\": \"s\", \"ms\": 1}", &p), "empty key rejected");
}

int main(int argc, char **argv) {
    if (argc < 2) {
        fprintf(stderr, "usage: host_logic_check SCRATCH_DIR\n");
        return 2;
    }
    geometry_checks();
    validation_checks();
    plan_checks();
    fit_checks();
    cache_checks(argv[1]);
    printf("%d failures\n", failures);
    return failures ? 1 : 0;
}
