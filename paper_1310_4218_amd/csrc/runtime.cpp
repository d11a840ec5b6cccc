// Host runtime of liblbgrid: the C ABI declared in include/lbgrid.h.
//
// A context owns the chunk table, the tiles (work items), the cost-field
// table, the chunk->slot map and the per-slot work queues, and replays the
// time step on the caller's stream.  The paper's migration loop (Fig. 2:
// steps, then measure, then MPI_Migrate) maps onto
//   lb_step (n steps)  ->  lb_measure (read the window's per-chunk loads)
//   ->  lb_rebalance (new chunk->slot map; the queues are rebuilt in place, so
//   captured graphs stay valid because only buffer contents change).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbgrid.h"
#include "lbgrid_internal.h"

using namespace lbgrid;

namespace {

thread_local std::string g_err;

int fail(std::string* where, int code, const std::string& msg) {
    if (where) *where = msg;
    g_err = msg;
    return code;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

}  // namespace

// The thread's last error, for entry points defined with the kernels.
int lbgrid::report_error(int code, const char* msg) { return fail(nullptr, code, msg); }

namespace {

// Everything lb_query / lb_grid_init derive from a configuration.
struct Plan {
    int32_t nx = 0, ny = 0, nz = 0, nfields = 1, px = 0, py = 0, C = 0, S = 0, Q = 0, G = 0, nwg = 0;
    int32_t nwg_cap = 0;    // workgroup counters sized for this many
    int32_t RD = 2;         // register pipeline depth (rows in flight)
    int32_t prec = 0, vec = 1, elem = 4, TX = 16, TY = 16, block = 0, ntiles = 0;
    int32_t nrows = 0;      // tile rows over all tiles: the most items a plan can have
    int32_t M = 0;          // rows in flight of the column march; 0 = another pipeline
    bool IG = false;        // balanced steps launch one workgroup per item
    int32_t F = 1;          // steps per launch of one workgroup per item (1, or 2 or 3 fused)
    int32_t block2 = 0;     // threads per workgroup of the two-step item launch
    size_t lds2 = 0;        // its LDS bytes
    int32_t block3 = 0;     // ... of the three-step item launch
    size_t lds3 = 0;
    int32_t CPW = 0;        // march: whole columns per wave (vertical physics, NQ not dividing 64)
    int32_t vec2 = 4;       // levels per thread of the two-step launch (4 or 5)
    int32_t CPW2 = 0;       // its whole columns per wave
    int32_t B = 0;          // rows per direct global->LDS batch; 0 = register pipeline
    int32_t ring = 4;       // LDS ring rows
    int32_t r2cut = 0;
    size_t lds = 0;
    int64_t ncells = 0;
    std::vector<int32_t> xs, ys;
    // workspace layout (byte offsets)
    size_t off_ctrl = 0, off_ktab = 0, off_items = 0, off_itemoff = 0, off_queue = 0, off_seg = 0,
           off_heads = 0, off_lw = 0, off_lt = 0, off_tw = 0, off_part = 0, off_hist = 0, off_busy = 0, off_tl = 0,
           off_visits = 0, off_sum = 0, off_first = 0, off_wstate = 0, off_pstate = 0, ws_bytes = 0;
    size_t st_loads = 0, st_tiles = 0, st_items = 0, st_queue = 0, st_first = 0, st_off = 0, st_seg = 0, st_n = 0,
           st_bytes = 0;  // pinned staging layout
    size_t field_bytes = 0;
};

bool strictly_increasing(const std::vector<int32_t>& s, int32_t n) {
    if (s.front() != 0 || s.back() != n) return false;
    for (size_t i = 1; i < s.size(); ++i)
        if (s[i] <= s[i - 1]) return false;
    return true;
}

// Ascending sort of keys (hi 32 bits: ~float bits of a non-negative cost,
// lo 32 bits: index) given in ascending index order: a stable least-
// significant-digit radix sort on the high half (8-bit digits), which leaves
// equal costs in index order, i.e. the order of the full 64-bit keys.  One
// read fills the four histograms; a digit that is the same in every key needs
// no pass.
void sort_keys(uint64_t* k, int32_t n) {
    if (n < 2) return;
    if (n < 64) {
        std::sort(k, k + n);
        return;
    }
    int32_t count[4][256];
    std::memset(count, 0, sizeof(count));
    for (int32_t i = 0; i < n; ++i) {
        const uint32_t hi = static_cast<uint32_t>(k[i] >> 32);
        ++count[0][hi & 0xff];
        ++count[1][(hi >> 8) & 0xff];
        ++count[2][(hi >> 16) & 0xff];
        ++count[3][hi >> 24];
    }
    std::vector<uint64_t> tmp(static_cast<size_t>(n));
    uint64_t* a = k;
    uint64_t* b = tmp.data();
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 32 + 8 * pass;
        int32_t* c = count[pass];
        if (c[(a[0] >> shift) & 0xff] == n) continue;
        int32_t run = 0;
        for (int d = 0; d < 256; ++d) {
            const int32_t x = c[d];
            c[d] = run;
            run += x;
        }
        for (int32_t i = 0; i < n; ++i) b[c[(a[i] >> shift) & 0xff]++] = a[i];
        std::swap(a, b);
    }
    if (a != k) std::memcpy(k, a, sizeof(uint64_t) * static_cast<size_t>(n));
}

// a mod n in [0, n)
int32_t wrap(int64_t a, int32_t n) {
    const int64_t r = a % n;
    return static_cast<int32_t>(r < 0 ? r + n : r);
}

// (x0 + v*t) mod n without overflow: every factor is reduced first, so the
// product stays below n^2 <= 2^62.
int32_t moved(int32_t x0, int32_t v, int64_t t, int32_t n) {
    return wrap(static_cast<int64_t>(wrap(x0, n)) + static_cast<int64_t>(wrap(v, n)) * wrap(t, n), n);
}

// Largest r^2 whose table entry can exceed kmin, plus one: beyond it
// (kmax-kmin)*exp(-r^2/(2 sigma^2)) < exp(-1/(2 sigma^2)) < 1.
int64_t cost_table_cut(double sigma, int32_t kmin, int32_t kmax) {
    const int32_t span = kmax - kmin;
    if (span <= 0) return 0;
    return static_cast<int64_t>(std::ceil(2.0 * sigma * sigma * std::log(static_cast<double>(span)))) + 1;
}

// Busy-time counters a launch fills: one per workgroup of the persistent
// launch, or one per compute unit with one workgroup per item.
int32_t busy_slots(const Plan& p) { return p.IG ? kCuSlots : p.nwg; }

int make_plan(const lb_config* c, Plan& p, std::string* err) {
    if (!c) return fail(err, LB_E_INVAL, "config is NULL");
    auto bad = [&](const char* what) { return fail(err, LB_E_INVAL, std::string("invalid config: ") + what); };
    if (c->nx < 1 || c->ny < 1 || c->nx > 32768 || c->ny > 32768) return bad("nx, ny must be in [1, 32768]");
    if (c->nz < 1 || c->nz > 4096) return bad("nz must be in [1, 4096]");
    if (c->nfields < 1 || c->nfields > 1024) return bad("nfields must be in [1, 1024]");
    if (c->px < 1 || c->px > c->nx || c->py < 1 || c->py > c->ny) return bad("px, py must be in [1, nx], [1, ny]");
    if (c->precision < LB_FP32 || c->precision > LB_FP64) return bad("precision");
    if (!std::isfinite(c->c_center) || !std::isfinite(c->c_nbr) || !std::isfinite(c->eps)) return bad("coefficients must be finite");
    if (c->nhot < 0 || c->nhot > LB_MAX_HOT) return bad("nhot must be in [0, 4]");
    if (c->kmin < 0 || c->kmax < c->kmin || c->kmax > 1000000) return bad("need 0 <= kmin <= kmax <= 1e6");
    if (c->nhot > 0 && c->kmax > c->kmin && !(c->sigma > 0.0 && c->sigma <= 1e5)) return bad("sigma must be in (0, 1e5]");
    if (c->alpha_work < 0) return bad("alpha_work must be >= 0");
    if (c->nslots < 1 || c->nslots > 65536) return bad("nslots must be in [1, 65536]");
    if (c->nqueues < 0 || c->nqueues > c->nslots) return bad("nqueues must be in [0, nslots]");
    if (c->wg_per_queue < 0) return bad("wg_per_queue must be >= 0");
    if (c->tile_x < 0 || c->tile_y < 0) return bad("tile sizes must be >= 0");
    if (c->graph_steps < 1 || c->graph_steps > 1000) return bad("graph_steps must be in [1, 1000]");
    if (c->steal != 0 && c->steal != 1) return bad("steal must be 0 or 1");
    if (c->item_split < 0 || c->item_split > 64) return bad("item_split must be in [0, 64]");
    if (c->tail_split < 0 || c->tail_split > 64) return bad("tail_split must be in [0, 64]");
    if (c->item_alpha < -1 || c->item_alpha > 1000000) return bad("item_alpha must be in [-1, 1e6]");
    if (c->stage_rows < -8 || c->stage_rows > 32 ||
        (c->stage_rows < -2 && c->stage_rows != -4 && c->stage_rows != -8))
        return bad("stage_rows must be -8, -4, -2, -1 (register pipeline) or in [0, 32]");
    if (c->physics != LB_PHYS_POINTWISE && c->physics != LB_PHYS_VERTICAL) return bad("physics");
    if (c->march != 0 && c->march != 2 && c->march != 4 && c->march != 8)
        return bad("march must be 0 (off), 2, 4 or 8 rows in flight");
    if (c->queue_order != 0 && c->queue_order != 1) return bad("queue_order must be 0 or 1");
    if (c->hot_cut < 0) return bad("hot_cut must be >= 0");
    if (c->item_grid != 0 && c->item_grid != 1) return bad("item_grid must be 0 or 1");
    if (c->item_grid == 1 && c->march == 0) return bad("item_grid needs the column-march pipeline (march > 0)");
    if (c->fuse_steps < 0 || c->fuse_steps > 3) return bad("fuse_steps must be 0, 1, 2 or 3");
    if (c->fuse_steps >= 2 && c->item_grid != 1) return bad("fuse_steps 2 or 3 needs item_grid 1");
    if (c->xcd_group < 0 || c->xcd_group > 64) return bad("xcd_group must be 0 .. 64");
    if (c->xcd_group > 1 && c->item_grid != 1) return bad("xcd_group needs item_grid 1");
    if (c->lane_levels != 0 && c->lane_levels != 4 && c->lane_levels != 5)
        return bad("lane_levels must be 0, 4 or 5");
    if (c->lane_levels == 5 && c->fuse_steps != 2) return bad("lane_levels 5 needs fuse_steps 2");
    if (c->lane_levels == 5 && c->nz % 20 != 0)
        return bad("lane_levels 5 needs nz divisible by 20 (5 levels per thread in the two-step launch, "
                   "4 in the one-step launches)");
    if (c->lane_levels == 5 && c->march != 2 && c->march != 4) return bad("lane_levels 5 needs march 2 or 4");

    p.nx = c->nx; p.ny = c->ny; p.nz = c->nz; p.nfields = c->nfields;
    p.px = c->px; p.py = c->py; p.C = c->px * c->py; p.S = c->nslots;
    p.prec = c->precision;
    p.elem = (p.prec == LB_FP64) ? 8 : 4;
    p.vec = (p.nz % 4 == 0) ? 4 : (p.nz % 2 == 0) ? 2 : 1;
    p.ncells = static_cast<int64_t>(p.nx) * p.ny * p.nz;

    p.xs.resize(p.px + 1);
    p.ys.resize(p.py + 1);
    for (int i = 0; i <= p.px; ++i)
        p.xs[i] = c->xsplit ? c->xsplit[i] : static_cast<int32_t>((static_cast<int64_t>(i) * p.nx) / p.px);
    for (int j = 0; j <= p.py; ++j)
        p.ys[j] = c->ysplit ? c->ysplit[j] : static_cast<int32_t>((static_cast<int64_t>(j) * p.ny) / p.py);
    if (!strictly_increasing(p.xs, p.nx)) return bad("xsplit must rise strictly from 0 to nx");
    if (!strictly_increasing(p.ys, p.ny)) return bad("ysplit must rise strictly from 0 to ny");

    const int NQ = p.nz / p.vec;
    // The vertical physics passes levels up a column's lanes inside one wave:
    // with NQ dividing 64 every layout keeps columns whole in a wave; otherwise
    // only the march lays out whole columns per wave (64 / NQ per wave).
    if (c->physics == LB_PHYS_VERTICAL && (NQ > 64 || (64 % NQ != 0 && c->march == 0)))
        return fail(err, LB_E_UNSUPPORTED,
                    "vertical physics needs nz / V <= 64 lanes per column, and the column-march "
                    "pipeline (march > 0) unless nz / V divides 64 (V = 4, 2 or 1 by divisibility of nz)");
    p.CPW = (c->physics == LB_PHYS_VERTICAL && c->march > 0 && 64 % NQ != 0) ? 64 / NQ : 0;
    p.vec2 = c->lane_levels == 5 ? 5 : 4;
    const int NQ2 = p.nz / p.vec2;
    p.CPW2 = c->lane_levels == 5 ? ((c->physics == LB_PHYS_VERTICAL && 64 % NQ2 != 0) ? 64 / NQ2 : 0) : p.CPW;
    // pipeline: the column march (M rows in flight), direct global->LDS batches of B
    // rows (V = 4 only) or the register path
    p.M = c->march;
    p.IG = c->item_grid == 1;
    p.F = c->fuse_steps >= 2 ? c->fuse_steps : 1;
    if (p.M > 0) {
        if (p.vec != 4) return bad("march needs nz divisible by 4");
        if (static_cast<uint64_t>(p.ncells) * p.elem > 0xFFFFFE00ull)
            return bad("march needs every field below 4 GiB (32-bit buffer offsets)");
    }
    if (p.M == 0 && c->stage_rows > 0 && p.vec != 4) return bad("stage_rows > 0 needs nz divisible by 4");
    if (p.M == 0 && c->stage_rows < -2 && p.vec != 4) return bad("register pipeline depth 4 or 8 needs nz divisible by 4");
    if (p.M == 0 && c->stage_rows == -8 && p.prec == LB_FP64) return bad("register pipeline depth 8 is FP32 only");
    p.B = p.M > 0 ? 0 : c->stage_rows > 0 ? c->stage_rows : (c->stage_rows == 0 && p.vec == 4 ? 4 : 0);
    p.RD = c->stage_rows < -2 ? -c->stage_rows : 2;
    p.ring = p.M > 0 ? 2 : p.B > 0 ? 2 * p.B + 2 : kRingRows;
    p.TY = c->tile_y > 0 ? c->tile_y : 16;
    const size_t col_bytes = static_cast<size_t>(p.nz) * p.elem;
    auto lds_for = [&](int tx) {  // LDS: the row ring, then trip counts of one tile (two for
                                  // the direct-load pipeline, which looks one item ahead)
        return static_cast<size_t>(p.ring) * (tx + 2) * col_bytes +
               sizeof(int32_t) * static_cast<size_t>(tx) * p.TY * (p.B > 0 ? 2 : 1);
    };
    // threads per workgroup: TX columns (the march adds the two halo columns) of NQ threads
    auto threads_for = [&](int tx) {
        if (p.CPW > 0) return (tx + 2 + p.CPW - 1) / p.CPW * 64;   // whole columns per wave
        return (p.M > 0 ? tx + 2 : tx) * NQ;
    };
    // the two-step item launch: two halo columns on either side, four LDS rows
    // (two of each step) and the trip counts of both steps
    auto threads2_for = [&](int tx) {
        if (p.CPW2 > 0) return (tx + 4 + p.CPW2 - 1) / p.CPW2 * 64;
        return (tx + 4) * NQ2;
    };
    auto lds2_for = [&](int tx) {
        return size_t{4} * (tx + 4) * col_bytes +
               sizeof(int32_t) * (static_cast<size_t>(tx + 2) * (p.TY + 2) + static_cast<size_t>(tx) * p.TY);
    };
    // three steps: three halo columns on either side, six LDS rows, three trip-count tables
    auto threads3_for = [&](int tx) {
        if (p.CPW > 0) return (tx + 6 + p.CPW - 1) / p.CPW * 64;
        return (tx + 6) * NQ;
    };
    auto lds3_for = [&](int tx) {
        return size_t{6} * (tx + 6) * col_bytes +
               sizeof(int32_t) * (static_cast<size_t>(tx + 4) * (p.TY + 4) + static_cast<size_t>(tx + 2) * (p.TY + 2) +
                                  static_cast<size_t>(tx) * p.TY);
    };
    const int most = p.M > 0 ? (p.prec == LB_FP64 ? kMaxBlockDeep : kMaxBlock)
                             : (p.B == 0 && (p.RD >= 4 || p.prec == LB_FP64)) ? kMaxBlockDeep : kMaxBlock;
    if (c->tile_x > 0) {
        p.TX = c->tile_x;
    } else {
        p.TX = p.M > 0 ? 32 : 16;
        while (p.TX > 1 && (threads_for(p.TX) > most || lds_for(p.TX) > 64 * 1024 ||
                            (p.F >= 2 && (threads2_for(p.TX) > most || lds2_for(p.TX) > 64 * 1024)) ||
                            (p.F == 3 && (threads3_for(p.TX) > most || lds3_for(p.TX) > 64 * 1024))))
            --p.TX;
    }
    if (p.TX > 1024 || p.TY > 256) return bad("tile sizes must be at most 1024 x 256");
    p.block = threads_for(p.TX);
    if (p.block > kMaxBlock) return bad("tile_x * nz / vector width exceeds 1024 threads");
    if (p.M > 0 && p.block > most)
        return bad("the FP64 march needs (tile_x + 2) * nz / 4 <= 512 threads");
    if (p.M == 0 && p.B == 0 && p.RD >= 4 && p.block > kMaxBlockDeep)
        return bad("register pipeline depth 4 or 8 needs tile_x * nz / 4 <= 512 threads");
    if (p.M == 0 && p.B == 0 && p.prec == LB_FP64 && p.block > kMaxBlockDeep)
        return bad("FP64 with the register pipeline needs tile_x * nz / V <= 512 threads");
    p.lds = lds_for(p.TX);
    if (p.lds > kMaxLds) return bad("tile too large: the LDS row ring and trip counts exceed 160 KiB");
    if (p.F >= 2) {   // (three-step launches end an odd remainder with a two-step one)
        p.block2 = threads2_for(p.TX);
        p.lds2 = lds2_for(p.TX);
        if (p.block2 > most)
            return bad(p.prec == LB_FP64 ? "fuse_steps 2 in FP64 needs (tile_x + 4) * nz / V <= 512 threads "
                                           "(V = lane_levels, else 4)"
                                         : "fuse_steps 2 needs (tile_x + 4) * nz / V <= 1024 threads "
                                           "(V = lane_levels, else 4)");
        if (p.lds2 > kMaxLds) return bad("tile too large for fuse_steps 2: its LDS rows and trip counts exceed 160 KiB");
    }
    if (p.F == 3) {
        p.block3 = threads3_for(p.TX);
        p.lds3 = lds3_for(p.TX);
        if (p.block3 > most)
            return bad(p.prec == LB_FP64 ? "fuse_steps 3 in FP64 needs (tile_x + 6) * nz / 4 <= 512 threads"
                                         : "fuse_steps 3 needs (tile_x + 6) * nz / 4 <= 1024 threads");
        if (p.lds3 > kMaxLds) return bad("tile too large for fuse_steps 3: its LDS rows and trip counts exceed 160 KiB");
    }

    // tiles of every chunk, chunks in id order, tiles in raster order; every tile
    // row can become an item of its own
    int64_t nt = 0, nr = 0;
    for (int j = 0; j < p.py; ++j)
        for (int i = 0; i < p.px; ++i) {
            const int64_t w = p.xs[i + 1] - p.xs[i], h = p.ys[j + 1] - p.ys[j];
            const int64_t tx = (w + p.TX - 1) / p.TX;
            nt += tx * ((h + p.TY - 1) / p.TY);
            nr += tx * h;
        }
    if (nr > (int64_t{1} << 28)) return bad("too many tiles");
    p.ntiles = static_cast<int32_t>(nt);
    p.nrows = static_cast<int32_t>(nr);

    p.Q = c->nqueues > 0 ? c->nqueues : (p.S % 8 == 0 ? 8 : p.S);
    // G = 0: chosen at init from the kernel's occupancy (resident workgroups per CU x CUs)
    p.G = c->wg_per_queue;
    const int64_t nwg = static_cast<int64_t>(p.Q) * std::max(p.G, 1);
    if (nwg > 65536) return bad("nqueues * wg_per_queue must be <= 65536");
    p.nwg = static_cast<int32_t>(nwg);
    p.nwg_cap = p.G > 0 ? p.nwg : 65536;

    const int64_t cut = (c->nhot > 0) ? cost_table_cut(c->sigma, c->kmin, c->kmax) : 0;
    if (cut > (int64_t{1} << 26)) return bad("cost table too large (sigma too wide for kmax - kmin)");
    p.r2cut = static_cast<int32_t>(cut);

    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + std::max<size_t>(bytes, 1)); return at; };
    p.off_ctrl = take(sizeof(Ctrl));
    p.off_ktab = take(sizeof(int32_t) * (static_cast<size_t>(p.r2cut) + 1));
    p.off_items = take(sizeof(ItemDesc) * static_cast<size_t>(p.nrows));
    p.off_itemoff = take(sizeof(int32_t) * (static_cast<size_t>(p.C) + 1));
    p.off_queue = take(sizeof(ItemDesc) * static_cast<size_t>(p.nrows));
    p.off_seg = take(sizeof(int32_t) * (static_cast<size_t>(p.Q) + 1));
    p.off_heads = take(sizeof(int32_t) * 2 * static_cast<size_t>(p.Q));
    // loads (work, time), tile work and busy time are adjacent: a measurement clears
    // them in one launch (busy last, so that only its nwg used entries are cleared)
    p.off_lw = take(sizeof(double) * static_cast<size_t>(p.C));
    p.off_lt = take(sizeof(double) * static_cast<size_t>(p.C));
    p.off_tw = take(sizeof(double) * static_cast<size_t>(p.ntiles));
    p.off_busy = take(sizeof(double) * static_cast<size_t>(std::max(p.nwg_cap, kCuSlots)));
    p.off_part = take(sizeof(double) * kStepSlots * static_cast<size_t>(p.nrows));
    p.off_hist = take(sizeof(double) * kHistLen);
    p.off_tl = take(sizeof(uint64_t) * 4 * static_cast<size_t>(p.nwg_cap));
    p.off_visits = take(sizeof(int32_t) * static_cast<size_t>(p.nrows));
    p.off_sum = take(sizeof(double) * (kSumBlocks + 1));
    p.off_first = take(sizeof(ItemDesc) * 2 * static_cast<size_t>(p.nwg_cap));
    p.off_wstate = take(sizeof(WgState) * static_cast<size_t>(p.nwg_cap));
    p.off_pstate = take(sizeof(WgState) * kStepSlots);
    p.ws_bytes = o;
    // pinned staging: measured loads, then the plan tables of an upload
    size_t h = 0;
    auto htake = [&](size_t bytes) { size_t at = h; h = (h + bytes + 31) & ~size_t{31}; return at; };
    p.st_loads = htake(sizeof(double) * static_cast<size_t>(p.C));
    p.st_tiles = htake(sizeof(double) * static_cast<size_t>(p.ntiles));
    p.st_items = htake(sizeof(ItemDesc) * static_cast<size_t>(p.nrows));
    p.st_queue = htake(sizeof(ItemDesc) * static_cast<size_t>(p.nrows));
    p.st_first = htake(sizeof(ItemDesc) * 2 * static_cast<size_t>(p.nwg_cap));
    p.st_off = htake(sizeof(int32_t) * (static_cast<size_t>(p.C) + 1));
    p.st_seg = htake(sizeof(int32_t) * (static_cast<size_t>(p.Q) + 1));
    p.st_n = htake(sizeof(int32_t));
    p.st_bytes = h;
    p.field_bytes = static_cast<size_t>(p.ncells) * p.nfields * p.elem;
    return LB_OK;
}

}  // namespace

struct lb_ctx {
    lb_config cfg{};
    Plan plan;
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    void* field[2] = {nullptr, nullptr};
    char* ws = nullptr;
    DevArgs args{};
    std::vector<int32_t> tiles;       // 4 per tile
    std::vector<int32_t> tile_off;    // C + 1: tiles of chunk c
    std::vector<int32_t> row_base;    // per tile: its first row in the visit counters
    std::vector<int32_t> pos_rank;    // per tile: its rank by (first row, first column)
    std::vector<int32_t> pos_order;   // tiles by that rank
    std::vector<ItemDesc> items;      // the installed plan, chunk order
    std::vector<ItemDesc> dealt;      // scratch of the XCD dealing of the item queue
    std::vector<int32_t> item_off;    // C + 1
    int64_t plan_version = 0;
    int64_t plain_graph_version = -1;
    std::vector<int32_t> map;         // C
    std::vector<double> measured;     // loads kept by the last lb_measure
    std::vector<double> tile_measured;  // work of every tile in the same window
    int64_t tile_steps = 0;           // steps in that window
    int64_t rebalances = 0;           // lb_rebalance calls that installed a map
    bool have_measured = false;
    bool broken = false;              // a step failed part-way: device state no longer matches `steps`
    int64_t steps = 0;
    int64_t window_steps = 0;
    double clock_hz = 100e6;
    char* staging = nullptr;          // pinned: measured loads and the plan tables (Plan::st_*)
    const char* staging_dev = nullptr;  // the same memory as the device addresses it
    hipEvent_t upload_done = nullptr;
    hipEvent_t measured_ev = nullptr;   // end of the last measurement's copy
    bool upload_pending = false;
    bool measure_pending = false;     // lb_measure_begin enqueued a snapshot not yet collected
    int64_t pending_steps = 0;        // steps in that snapshot's window
    double host_balance_us = 0.0;     // all rebalances: the balancer
    double host_plan_us = 0.0;        // all plans: items, queue order, staging, upload launch
    hipGraphExec_t g_pers = nullptr;  // graph_steps persistent steps
    hipGraphExec_t g_pers1 = nullptr; // one persistent step
    // one workgroup per item: graph_steps steps and one step, per slot (number mod kStepSlots)
    // of the first step (the slot is a launch argument), for the plan they were taken on
    hipGraphExec_t g_items[kStepSlots] = {};
    hipGraphExec_t g_items1[kStepSlots] = {};
    int64_t items_graph_version[kStepSlots] = {-1, -1, -1, -1, -1, -1, -1, -1};
    int cur = 0;                      // field copy holding the current step's values
    bool wstate_stale = false;        // only the shared per-parity step state is current
    bool items_stale = false;         // the chunk-order item tables on the device are not the plan's
    hipGraphExec_t g_plain = nullptr; // one plain step
    std::string err;
};

namespace {

#define HIP_TRY(ctx, expr)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail((ctx) ? &(ctx)->err : nullptr, LB_E_HIP,                                \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                     \
    } while (0)

#define LAUNCH_TRY(ctx, expr)                                                                   \
    do {                                                                                        \
        int e_ = (expr);                                                                        \
        if (e_ != 0)                                                                            \
            return fail(&(ctx)->err, LB_E_HIP,                                                  \
                        std::string(#expr) + ": " +                                            \
                            hipGetErrorString(static_cast<hipError_t>(e_)));                   \
    } while (0)

const char* fail_site() { return std::getenv("LBGRID_FAIL_AT"); }
bool forced_failure(const char* site) {
    const char* f = fail_site();
    return f && std::strcmp(f, site) == 0;
}
// LBGRID_FAIL_AT=launch:N: the N-th kernel or graph launch of each lb_step call
// fails (N >= 1) as if the runtime had refused it; 0 when not set.
int forced_launch_failure() {
    const char* f = fail_site();
    if (!f || std::strncmp(f, "launch:", 7) != 0) return 0;
    return std::atoi(f + 7);
}

void build_tiles(lb_ctx* x) {
    const Plan& p = x->plan;
    x->tiles.clear();
    x->tiles.reserve(static_cast<size_t>(p.ntiles) * 4);
    x->tile_off.assign(static_cast<size_t>(p.C) + 1, 0);
    int32_t t = 0;
    for (int j = 0; j < p.py; ++j)
        for (int i = 0; i < p.px; ++i) {
            const int c = j * p.px + i;
            x->tile_off[c] = t;
            for (int y = p.ys[j]; y < p.ys[j + 1]; y += p.TY)
                for (int xx = p.xs[i]; xx < p.xs[i + 1]; xx += p.TX) {
                    const int w = std::min(p.TX, p.xs[i + 1] - xx);
                    const int h = std::min(p.TY, p.ys[j + 1] - y);
                    x->tiles.insert(x->tiles.end(), {xx, y, w | (h << 16), c});
                    ++t;
                }
        }
    x->tile_off[p.C] = t;
    {
        std::vector<uint64_t> k(static_cast<size_t>(p.ntiles));
        for (int32_t i = 0; i < p.ntiles; ++i)   // y0, x0 < 2^16 (validated grid sizes)
            k[i] = (static_cast<uint64_t>(x->tiles[4 * i + 1]) << 48) |
                   (static_cast<uint64_t>(x->tiles[4 * i + 0]) << 32) | static_cast<uint32_t>(i);
        std::sort(k.begin(), k.end());
        x->pos_rank.resize(static_cast<size_t>(p.ntiles));
        x->pos_order.resize(static_cast<size_t>(p.ntiles));
        for (int32_t r = 0; r < p.ntiles; ++r) {
            x->pos_rank[k[r] & 0xffffffffu] = r;
            x->pos_order[r] = static_cast<int32_t>(k[r] & 0xffffffffu);
        }
    }
    x->row_base.resize(static_cast<size_t>(p.ntiles));
    int32_t r = 0;
    for (int32_t i = 0; i < p.ntiles; ++i) {
        x->row_base[i] = r;
        r += x->tiles[4 * i + 2] >> 16;
    }
}

std::vector<int32_t> build_cost_table(const lb_config& c, int32_t r2cut) {
    std::vector<int32_t> tab(static_cast<size_t>(r2cut) + 1);
    const double span = static_cast<double>(c.kmax - c.kmin);
    for (int32_t r2 = 0; r2 <= r2cut; ++r2) {
        const double g = std::exp(-static_cast<double>(r2) / (2.0 * c.sigma * c.sigma));
        tab[r2] = c.kmin + static_cast<int32_t>(std::floor(span * g));
    }
    if (c.nhot == 0 || c.kmax == c.kmin) tab.assign(tab.size(), c.kmin);
    return tab;
}

// Work plan for a map and per-chunk costs (NULL: equal costs, no splitting).
//  - Items: a tile whose cost exceeds W / (nwg * item_split) is cut into that
//    many row ranges (at most one per row), so that no single item outlasts the
//    rest of the step; cheap tiles stay whole, which keeps their halo overhead
//    low.  After a measurement the tile cost is the tile's own measured work
//    (the load measurement of Section V taken per tile as well as per chunk);
//    with caller-given chunk costs it is chunk cost * tile area / chunk area.
//  - Queues: queue q gets the items of the chunks of the slots s with s mod Q = q,
//    tile by tile in descending cost per item (ties by tile index), the items of
//    a tile one after another (first row first).
int upload_plan(lb_ctx* x, const double* cost, const double* tile_cost) {
    const Plan& p = x->plan;
    const auto t_plan = std::chrono::steady_clock::now();

    // Cost of every tile: its measured work when the plan follows a measurement;
    // else its chunk's cost times its share of the chunk's area; without costs,
    // the tile's area (and no splitting).
    std::vector<double> tcost(static_cast<size_t>(p.ntiles));
    std::vector<int> pieces(static_cast<size_t>(p.ntiles), 1);
    double W = 0.0;
    for (int32_t c = 0; c < p.C; ++c) {
        const int i = c % p.px, j = c / p.px;
        const double area_c = static_cast<double>(p.xs[i + 1] - p.xs[i]) * (p.ys[j + 1] - p.ys[j]);
        for (int32_t t = x->tile_off[c]; t < x->tile_off[c + 1]; ++t) {
            const int w = x->tiles[4 * t + 2] & 0xffff, h = x->tiles[4 * t + 2] >> 16;
            const double area_t = static_cast<double>(w) * h;
            tcost[t] = tile_cost ? tile_cost[t] : cost ? cost[c] * (area_t / area_c) : area_t;
            if (tile_cost && x->cfg.item_alpha >= 0)  // count the stencil at item_alpha per cell
                tcost[t] = std::max(0.0, tcost[t] - static_cast<double>(x->cfg.alpha_work - x->cfg.item_alpha) *
                                                        p.nz * p.nfields * area_t * static_cast<double>(x->tile_steps));
            W += tcost[t];
        }
    }
    const int split = x->cfg.item_split;
    const bool costed = (cost || tile_cost) && split > 0 && W > 0.0;
    const double target = costed ? W / (static_cast<double>(p.nwg) * split) : 0.0;
    if (target > 0.0)
        for (int32_t t = 0; t < p.ntiles; ++t) {
            const int h = x->tiles[4 * t + 2] >> 16;
            if (tcost[t] > target) pieces[t] = static_cast<int>(std::min<double>(h, std::ceil(tcost[t] / target)));
        }
    // Tiles of every queue in longest-first order: cost per piece descending
    // (compared in single precision), tile index ascending on ties.  One sort serves the tail split and the
    // queue order (the items of a tile follow one another, first row first).
    std::vector<int32_t> qoff(static_cast<size_t>(p.Q) + 1, 0);
    for (int32_t c = 0; c < p.C; ++c) qoff[x->map[c] % p.Q + 1] += x->tile_off[c + 1] - x->tile_off[c];
    for (int32_t q = 0; q < p.Q; ++q) qoff[q + 1] += qoff[q];
    // The sort key is one integer: the complemented bits of the cost per piece
    // as a float (non-negative floats order like their bit patterns), then the
    // tile index; plain integer sorting keeps a plan of ~10^4 tiles cheap.
    // With queue_order 1 only the hot tiles (cost per piece above hot_cut
    // percent of the mean over all pieces) are keyed by cost; every other tile sorts after
    // them by its position rank (first row, then first column).  Keys: cost
    // keys have the top bit clear, position keys set.
    double hot_cut = 0.0;
    if (x->cfg.queue_order >= 1) {
        int64_t npieces = 0;
        for (int32_t t = 0; t < p.ntiles; ++t) npieces += pieces[t];
        hot_cut = npieces > 0 ? (x->cfg.hot_cut / 100.0) * W / static_cast<double>(npieces) : 0.0;
    }
    auto key_of = [&](int32_t t) -> uint64_t {
        const double pp = tcost[t] / pieces[t];
        if (x->cfg.queue_order >= 1 && !(pp > hot_cut))
            return (static_cast<uint64_t>(0x80000000u | static_cast<uint32_t>(x->pos_rank[t])) << 32) |
                   static_cast<uint32_t>(t);
        const float per_piece = static_cast<float>(pp);
        uint32_t bits;   // a non-negative float: top bit clear, so ~bits has it set
        std::memcpy(&bits, &per_piece, sizeof(bits));
        return (static_cast<uint64_t>(~bits & 0x7fffffffu) << 32) | static_cast<uint32_t>(t);
    };
    std::vector<uint64_t> order(static_cast<size_t>(p.ntiles));
    if (x->cfg.queue_order >= 1) {
        // the keys in sorted order without sorting the position keys: per queue,
        // its hot tiles (sorted), then its other tiles as they come in position order
        auto queue_of = [&](int32_t t) { return x->map[x->tiles[4 * t + 3]] % p.Q; };
        std::vector<int32_t> hot_end(qoff.begin(), qoff.end() - 1), tail(static_cast<size_t>(p.Q));
        for (int32_t t = 0; t < p.ntiles; ++t) {
            const uint64_t key = key_of(t);
            if (!(key >> 63)) order[hot_end[queue_of(t)]++] = key;
        }
        for (int32_t q = 0; q < p.Q; ++q) tail[q] = hot_end[q];
        for (int32_t r = 0; r < p.ntiles; ++r) {
            const int32_t t = x->pos_order[r];
            const uint64_t key = key_of(t);
            if (key >> 63) order[tail[queue_of(t)]++] = key;
        }
        for (int32_t q = 0; q < p.Q; ++q) sort_keys(order.data() + qoff[q], hot_end[q] - qoff[q]);
    } else {
        std::vector<int32_t> fill(qoff.begin(), qoff.end() - 1);
        for (int32_t c = 0; c < p.C; ++c) {
            int32_t& at = fill[x->map[c] % p.Q];
            for (int32_t t = x->tile_off[c]; t < x->tile_off[c + 1]; ++t) order[at++] = key_of(t);
        }
        for (int32_t q = 0; q < p.Q; ++q) sort_keys(order.data() + qoff[q], qoff[q + 1] - qoff[q]);
    }
    auto tile_at = [&](int32_t i) { return static_cast<int32_t>(order[i] & 0xffffffffu); };
    // Tail: in every queue, the cheapest tiles whose pieces make up the final
    // round of its G workgroups (the last G items in this order) are cut
    // tail_split times finer, so the step ends on small items and the
    // workgroups finish together instead of one item apart.  Their cost per
    // piece only drops, so the order stands.
    const int tail = x->cfg.tail_split;
    if (tail > 1)
        for (int32_t q = 0; q < p.Q; ++q) {
            int64_t covered = 0;
            for (int32_t i = qoff[q + 1] - 1; i >= qoff[q] && covered < p.G; --i) {
                const int32_t t = tile_at(i);
                covered += pieces[t];
                pieces[t] = std::min(x->tiles[4 * t + 2] >> 16, pieces[t] * tail);
            }
        }

    // Items in chunk order (tile raster, first row first); item_first[t] is the
    // first item of tile t.
    x->items.clear();
    x->item_off.assign(static_cast<size_t>(p.C) + 1, 0);
    std::vector<int32_t> item_first(static_cast<size_t>(p.ntiles));
    for (int32_t c = 0; c < p.C; ++c) {
        x->item_off[c] = static_cast<int32_t>(x->items.size());
        for (int32_t t = x->tile_off[c]; t < x->tile_off[c + 1]; ++t) {
            const int w = x->tiles[4 * t + 2] & 0xffff, h = x->tiles[4 * t + 2] >> 16;
            item_first[t] = static_cast<int32_t>(x->items.size());
            // piece k covers rows [floor(k h / parts), floor((k + 1) h / parts)),
            // stepped exactly with one division per tile: the next bound is the
            // last one plus h / parts, plus one when the kept remainder
            // k h mod parts wraps
            const int parts = pieces[t], step = h / parts, extra = h - step * parts;
            int r1 = 0, rem = 0;
            for (int k = 0; k < parts; ++k) {
                const int r0 = r1;
                rem += extra;
                r1 = r0 + step + (rem >= parts ? 1 : 0);
                if (rem >= parts) rem -= parts;
                ItemDesc d{};
                d.x0 = x->tiles[4 * t + 0];
                d.y0 = x->tiles[4 * t + 1] + r0;
                d.wh = w | ((r1 - r0) << 16);
                d.chunk = c;
                d.id = static_cast<int32_t>(x->items.size());
                d.vbase = x->row_base[t] + r0;
                d.tile = t;
                x->items.push_back(d);
            }
        }
    }
    const int32_t n = static_cast<int32_t>(x->items.size());
    x->item_off[p.C] = n;

    if (x->upload_pending) {
        HIP_TRY(x, hipEventSynchronize(x->upload_done));
        x->upload_pending = false;
    }
    ItemDesc* st_items = reinterpret_cast<ItemDesc*>(x->staging + p.st_items);
    ItemDesc* st_queue = reinterpret_cast<ItemDesc*>(x->staging + p.st_queue);
    ItemDesc* st_first = reinterpret_cast<ItemDesc*>(x->staging + p.st_first);
    int32_t* st_off = reinterpret_cast<int32_t*>(x->staging + p.st_off);
    int32_t* st_seg = reinterpret_cast<int32_t*>(x->staging + p.st_seg);
    int32_t* st_n = reinterpret_cast<int32_t*>(x->staging + p.st_n);
    // A context whose balanced steps launch one workgroup per item reads the
    // chunk-order tables only in plain steps: they go up on the first plain step
    // after a change (upload_items), not with every plan.
    const bool chunk_tables = !p.IG;
    x->items_stale = p.IG;
    if (chunk_tables) {
        std::memcpy(st_items, x->items.data(), sizeof(ItemDesc) * n);
        std::memcpy(st_off, x->item_off.data(), sizeof(int32_t) * x->item_off.size());
    }
    int32_t k = 0;
    for (int32_t q = 0; q < p.Q; ++q) {
        st_seg[q] = k;
        for (int32_t i = qoff[q]; i < qoff[q + 1]; ++i) {
            const int32_t t = tile_at(i);
            for (int32_t j = 0; j < pieces[t]; ++j) st_queue[k++] = x->items[item_first[t] + j];
        }
    }
    st_seg[p.Q] = k;
    // One workgroup per item: the hardware hands workgroup b to XCD b mod 8.  With
    // xcd_group G, runs of G consecutive items of the order (neighbours along x,
    // whose halo columns overlap) go to workgroups 8 apart, so that one XCD runs
    // them side by side and reads their shared halos from its own L2: item i =
    // (8 s + r) G + j runs as workgroup (s G + j) 8 + r.  The order stands at a
    // granularity of 8 G items; a last partial block of 8 G items keeps its place.
    const int G = x->cfg.xcd_group;
    if (p.IG && G > 1) {
        std::vector<ItemDesc>& tmp = x->dealt;
        tmp.assign(st_queue, st_queue + k);
        const int32_t full = (k / (8 * G)) * 8 * G;
        for (int32_t i = 0; i < full; ++i) {
            const int32_t g = i / G, j = i - g * G, sg = g >> 3, r = g & 7;
            st_queue[(sg * G + j) * 8 + r] = tmp[i];
        }
    }
    *st_n = n;
    // First two items of every workgroup: items `rank` and 2G - 1 - rank of its
    // home queue, with the same workgroup -> (queue, rank) assignment as the
    // device (home_queue in kernels.hip).
    const DevArgs& a = x->args;
    ItemDesc none{};
    none.id = -1;
    // (home, rank) of workgroup w, stepped with counters rather than two
    // divisions per workgroup: qh, qr are (w >> 3) mod and div Q / 8 with XCD
    // queues, else w mod and div Q
    const int per_xcd = a.xcd_queues ? p.Q / 8 : 1;
    int qh = 0, qr = 0;
    for (int32_t w = 0; w < (p.IG ? 0 : p.nwg); ++w) {   // (not read by a launch per item)
        int home, rank;
        if (a.xcd_queues) {
            home = (w & 7) + 8 * qh;
            rank = qr;
            if ((w & 7) == 7 && ++qh == per_xcd) {
                qh = 0;
                ++qr;
            }
        } else {
            home = qh;
            rank = qr;
            if (++qh == p.Q) {
                qh = 0;
                ++qr;
            }
        }
        const int nq = st_seg[home + 1] - st_seg[home];
        const int second = 2 * p.G - 1 - rank;
        st_first[2 * w] = rank < nq ? st_queue[st_seg[home] + rank] : none;
        st_first[2 * w + 1] = second < nq ? st_queue[st_seg[home] + second] : none;
    }
    // One kernel moves all tables from the pinned staging (read over the bus) into
    // the workspace: a single launch instead of one copy per table.
    auto seg = [&](size_t st, size_t off, size_t bytes) {
        return GatherSeg{reinterpret_cast<const uint32_t*>(x->staging_dev + st),
                         reinterpret_cast<uint32_t*>(x->ws + off), static_cast<uint32_t>(bytes / 4)};
    };
    const GatherSeg segs[] = {
        seg(p.st_queue, p.off_queue, sizeof(ItemDesc) * n),
        seg(p.st_seg, p.off_seg, sizeof(int32_t) * (p.Q + 1)),
        seg(p.st_n, p.off_ctrl + offsetof(Ctrl, nitems), sizeof(int32_t)),
        seg(p.st_items, p.off_items, sizeof(ItemDesc) * n),
        seg(p.st_off, p.off_itemoff, sizeof(int32_t) * (p.C + 1)),
        seg(p.st_first, p.off_first, sizeof(ItemDesc) * 2 * p.nwg),
    };
    const int nsegs = chunk_tables ? static_cast<int>(sizeof(segs) / sizeof(segs[0])) : 3;
    LAUNCH_TRY(x, launch_gather(segs, nsegs, x->stream));
    HIP_TRY(x, hipEventRecord(x->upload_done, x->stream));
    x->upload_pending = true;
    ++x->plan_version;
    x->host_plan_us += std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t_plan).count();
    return LB_OK;
}

// The chunk-order item tables of the installed plan, which plain steps read;
// deferred by upload_plan for contexts that launch one workgroup per item.
int upload_items(lb_ctx* x) {
    const Plan& p = x->plan;
    if (x->upload_pending) {
        HIP_TRY(x, hipEventSynchronize(x->upload_done));
        x->upload_pending = false;
    }
    const int32_t n = static_cast<int32_t>(x->items.size());
    std::memcpy(x->staging + p.st_items, x->items.data(), sizeof(ItemDesc) * n);
    std::memcpy(x->staging + p.st_off, x->item_off.data(), sizeof(int32_t) * x->item_off.size());
    const GatherSeg segs[] = {
        GatherSeg{reinterpret_cast<const uint32_t*>(x->staging_dev + p.st_items),
                  reinterpret_cast<uint32_t*>(x->ws + p.off_items),
                  static_cast<uint32_t>(sizeof(ItemDesc) * n / 4)},
        GatherSeg{reinterpret_cast<const uint32_t*>(x->staging_dev + p.st_off),
                  reinterpret_cast<uint32_t*>(x->ws + p.off_itemoff), static_cast<uint32_t>(p.C + 1)},
    };
    LAUNCH_TRY(x, launch_gather(segs, 2, x->stream));
    HIP_TRY(x, hipEventRecord(x->upload_done, x->stream));
    x->upload_pending = true;
    x->items_stale = false;
    return LB_OK;
}

// Steps a balanced launch takes when `left` steps remain: the plan's steps per
// launch (F) while at least that many remain, then the rest in one launch (a
// remainder of 1 or 2 steps: F is at most 3).
int launch_span(const Plan& p, int left) { return left < p.F ? left : p.F; }

// Field copies written by n balanced steps launched in spans of launch_span.
int launches_for(const Plan& p, int n) { return n / p.F + (n % p.F ? 1 : 0); }

// One balanced launch of n (= launch_span) steps, in the plan's form; slot is the
// number mod kStepSlots of its first step.
int launch_balanced(lb_ctx* x, int slot, int n, hipStream_t s) {
    const Plan& p = x->plan;
    const int nitems = static_cast<int>(x->items.size());
    if (p.IG && n == 3) return launch_items3(x->args, p.prec, p.vec, nitems, p.block3, p.lds3, slot, s);
    if (p.IG && n == 2) return launch_items2(x->args, p.prec, p.vec2, nitems, p.block2, p.lds2, slot, s);
    if (n != 1) return static_cast<int>(hipErrorInvalidValue);
    if (p.IG) return launch_items(x->args, p.prec, p.vec, nitems, p.block, p.lds, slot, s);
    return launch_persistent(x->args, p.prec, p.vec, p.nwg, p.block, p.lds, s);
}

int capture(lb_ctx* x, int mode, int nsteps, hipGraphExec_t* out, int slot0 = 0) {
    const Plan& p = x->plan;
    hipGraph_t g = nullptr;
    HIP_TRY(x, hipStreamBeginCapture(x->cap, hipStreamCaptureModeThreadLocal));
    int rc = 0;
    for (int i = 0; i < nsteps && rc == 0;) {
        if (mode == LB_PERSISTENT) {
            const int n = launch_span(p, nsteps - i);
            rc = launch_balanced(x, (slot0 + i) & kSlotMask, n, x->cap);
            i += n;
        } else {
            ++i;
            for (int32_t c = 0; c < p.C && rc == 0; ++c)
                rc = launch_plain_chunk(x->args, p.prec, p.vec, c, x->item_off[c + 1] - x->item_off[c],
                                        p.block, p.lds, x->cap);
            if (rc == 0) rc = launch_finish(x->args, x->cap);
        }
    }
    hipError_t e = hipStreamEndCapture(x->cap, &g);
    if (rc != 0 || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        const hipError_t shown = rc != 0 ? static_cast<hipError_t>(rc) : e;
        return fail(&x->err, LB_E_HIP, std::string("graph capture: ") + hipGetErrorString(shown));
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(&x->err, LB_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return LB_OK;
}

int sync(lb_ctx* x) {
    HIP_TRY(x, hipSetDevice(x->device));
    if (forced_failure("sync")) return fail(&x->err, LB_E_HIP, "forced failure at sync (LBGRID_FAIL_AT)");
    HIP_TRY(x, hipStreamSynchronize(x->stream));
    return LB_OK;
}

}  // namespace

extern "C" {

int lb_abi_version(void) { return LB_ABI_VERSION; }
size_t lb_config_bytes(void) { return sizeof(lb_config); }
size_t lb_stats_bytes(void) { return sizeof(lb_stats_t); }

void lb_config_default(lb_config* c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->nx = c->ny = 64;
    c->nz = 32;
    c->nfields = 1;
    c->px = c->py = 4;
    c->precision = LB_FP32;
    c->c_center = 0.4;
    c->c_nbr = 0.1;
    c->eps = 0.01;
    c->nhot = 0;
    c->sigma = 8.0;
    c->kmin = 1;
    c->kmax = 1;
    c->alpha_work = 32;
    c->nslots = 256;
    c->nqueues = 0;
    c->wg_per_queue = 0;
    c->tile_x = 0;
    c->tile_y = 0;
    c->steal = 1;
    c->graph_steps = 10;
    c->item_split = 2;
    c->stage_rows = 0;
    c->physics = LB_PHYS_POINTWISE;
    c->tail_split = 4;
    c->item_alpha = -1;
    c->march = 0;
    c->queue_order = 0;
    c->hot_cut = 200;
    c->item_grid = 0;
    c->fuse_steps = 0;
    c->lane_levels = 0;
    c->xcd_group = 0;
}

int lb_query(const lb_config* cfg, lb_buffers* out) {
    if (!out) return fail(nullptr, LB_E_INVAL, "sizes_out is NULL");
    Plan p;
    int rc = make_plan(cfg, p, nullptr);
    if (rc != LB_OK) return rc;
    std::memset(out, 0, sizeof(*out));
    out->bytes[0] = p.field_bytes;
    out->bytes[1] = p.field_bytes;
    out->bytes[2] = p.ws_bytes;
    return LB_OK;
}

int lb_grid_init(const lb_config* cfg, const lb_buffers* bufs, void* hip_stream,
                 const void* init_field, lb_ctx** out) {
    if (!out) return fail(nullptr, LB_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!bufs) return fail(nullptr, LB_E_INVAL, "buffers are NULL");
    Plan p;
    int rc = make_plan(cfg, p, nullptr);
    if (rc != LB_OK) return rc;
    const size_t need[3] = {p.field_bytes, p.field_bytes, p.ws_bytes};
    for (int i = 0; i < LB_NBUF; ++i) {
        if (!bufs->ptr[i]) return fail(nullptr, LB_E_INVAL, "buffer " + std::to_string(i) + " is NULL");
        if (bufs->bytes[i] < need[i])
            return fail(nullptr, LB_E_NOMEM, "buffer " + std::to_string(i) + " too small: " +
                                                 std::to_string(bufs->bytes[i]) + " < " + std::to_string(need[i]));
        if (reinterpret_cast<uintptr_t>(bufs->ptr[i]) % kAlign != 0)
            return fail(nullptr, LB_E_INVAL, "buffer " + std::to_string(i) + " is not 256-byte aligned");
    }
    if (forced_failure("init")) return fail(nullptr, LB_E_HIP, "forced failure at init (LBGRID_FAIL_AT)");

    lb_ctx* x = new (std::nothrow) lb_ctx();
    if (!x) return fail(nullptr, LB_E_NOMEM, "out of host memory");
    x->cfg = *cfg;
    x->cfg.xsplit = nullptr;  // copied into the plan
    x->cfg.ysplit = nullptr;
    x->plan = std::move(p);
    const Plan& P = x->plan;
    x->stream = static_cast<hipStream_t>(hip_stream);
    x->field[0] = bufs->ptr[0];
    x->field[1] = bufs->ptr[1];
    x->ws = static_cast<char*>(bufs->ptr[2]);

    auto bail = [&](int code) {
        lb_destroy(x);
        return code;
    };
    auto hip_bail = [&](hipError_t e, const char* what) {
        fail(nullptr, LB_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
        return bail(LB_E_HIP);
    };
    hipError_t e;
    if ((e = hipGetDevice(&x->device)) != hipSuccess) return hip_bail(e, "hipGetDevice");
    int wall_khz = 0;
    if ((e = hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, x->device)) != hipSuccess)
        return hip_bail(e, "hipDeviceGetAttribute(WallClockRate)");
    if (wall_khz > 0) x->clock_hz = 1e3 * wall_khz;
    if ((e = hipStreamCreateWithFlags(&x->cap, hipStreamNonBlocking)) != hipSuccess)
        return hip_bail(e, "hipStreamCreateWithFlags");
    if ((e = hipEventCreateWithFlags(&x->upload_done, hipEventDisableTiming)) != hipSuccess)
        return hip_bail(e, "hipEventCreateWithFlags");
    if ((e = hipEventCreateWithFlags(&x->measured_ev, hipEventDisableTiming)) != hipSuccess)
        return hip_bail(e, "hipEventCreateWithFlags");
    {
        void* st = nullptr;
        if ((e = hipHostMalloc(&st, P.st_bytes, hipHostMallocMapped | hipHostMallocPortable)) != hipSuccess)
            return hip_bail(e, "hipHostMalloc");
        x->staging = static_cast<char*>(st);
        void* dev = nullptr;
        if ((e = hipHostGetDevicePointer(&dev, st, 0)) != hipSuccess) return hip_bail(e, "hipHostGetDevicePointer");
        x->staging_dev = static_cast<const char*>(dev);
    }

    int lds_limit = 0;
    if ((e = hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, x->device)) != hipSuccess)
        return hip_bail(e, "hipDeviceGetAttribute(MaxSharedMemoryPerBlock)");
    if (P.lds > static_cast<size_t>(lds_limit)) {
        fail(nullptr, LB_E_INVAL, "tile needs " + std::to_string(P.lds) + " bytes of LDS, the device allows " +
                                      std::to_string(lds_limit));
        return bail(LB_E_INVAL);
    }
    build_tiles(x);
    const std::vector<int32_t> ktab = build_cost_table(*cfg, P.r2cut);
    // resolve this device's copy of the allocation-free entry point's scratch now,
    // at set-up, rather than on that entry point's first call
    if ((e = static_cast<hipError_t>(prepare_static_scratch(x->device))) != hipSuccess)
        return hip_bail(e, "hipGetSymbolAddress(scratch)");

    DevArgs& a = x->args;
    a.field0 = x->field[0];
    a.field1 = x->field[1];
    a.ktab = reinterpret_cast<const int32_t*>(x->ws + P.off_ktab);
    a.items = reinterpret_cast<const ItemDesc*>(x->ws + P.off_items);
    a.item_off = reinterpret_cast<const int32_t*>(x->ws + P.off_itemoff);
    a.queue = reinterpret_cast<const ItemDesc*>(x->ws + P.off_queue);
    a.seg = reinterpret_cast<const int32_t*>(x->ws + P.off_seg);
    a.firstd = reinterpret_cast<const ItemDesc*>(x->ws + P.off_first);
    a.heads = reinterpret_cast<int32_t*>(x->ws + P.off_heads);
    a.wstate = reinterpret_cast<WgState*>(x->ws + P.off_wstate);
    a.pstate = reinterpret_cast<WgState*>(x->ws + P.off_pstate);
    a.ctrl = reinterpret_cast<Ctrl*>(x->ws + P.off_ctrl);
    a.loads_work = reinterpret_cast<double*>(x->ws + P.off_lw);
    a.loads_time = reinterpret_cast<double*>(x->ws + P.off_lt);
    a.tile_work = reinterpret_cast<double*>(x->ws + P.off_tw);
    a.partials = reinterpret_cast<double*>(x->ws + P.off_part);
    a.hist = reinterpret_cast<double*>(x->ws + P.off_hist);
    a.wg_busy = reinterpret_cast<double*>(x->ws + P.off_busy);
    a.wg_timeline = reinterpret_cast<uint64_t*>(x->ws + P.off_tl);
    a.visits = reinterpret_cast<int32_t*>(x->ws + P.off_visits);
    a.ncells = P.ncells;
    a.part_stride = P.nrows;
    a.nx = P.nx; a.ny = P.ny; a.nz = P.nz; a.nfields = P.nfields;
    a.tile_x = P.TX;
    a.tile_y = P.TY;
    a.block = P.block;
    a.block2 = P.block2;
    a.block3 = P.block3;
    a.stage_rows = P.B;
    a.reg_depth = P.RD;
    a.march = P.M;
    a.item_grid = P.IG ? 1 : 0;
    // the next read of an output cell comes a whole field later: past the
    // last-level cache (256 MB on this GPU) when the two copies exceed it
    a.stream_store = 2 * P.field_bytes > (size_t{256} << 20) ? 1 : 0;
    a.field_bytes = static_cast<uint32_t>(std::min<uint64_t>(static_cast<uint64_t>(P.ncells) * P.elem, 0xFFFFFFFFull));
    a.vertical = cfg->physics == LB_PHYS_VERTICAL ? 1 : 0;
    a.col_per_wave = P.CPW;
    a.col_per_wave2 = P.CPW2;
    if (P.G == 0) {  // as many workgroups as can be resident, split evenly over the queues
        int ncu = 0;
        if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, x->device)) != hipSuccess)
            return hip_bail(e, "hipDeviceGetAttribute(MultiprocessorCount)");
        const int occ = persistent_occupancy(a, P.prec, P.vec, P.block, P.lds);
        if (occ < 1) {
            fail(nullptr, LB_E_HIP, "persistent kernel occupancy query failed");
            return bail(LB_E_HIP);
        }
        Plan& W = x->plan;
        W.G = std::max(1, (occ * ncu) / W.Q);
        W.nwg = W.Q * W.G;
        if (W.nwg > W.nwg_cap) {
            W.G = std::max(1, W.nwg_cap / W.Q);
            W.nwg = W.Q * W.G;
        }
    }
    a.nqueues = P.Q; a.nwg = P.nwg; a.steal = cfg->steal; a.head0 = 2 * P.G;
    a.r2cut = P.r2cut;
    a.kmin = cfg->kmin;
    a.alpha = cfg->alpha_work;
    a.nhot = cfg->nhot;
    a.xcd_queues = (P.Q % 8 == 0 && P.nwg % 8 == 0) ? 1 : 0;
    for (int h = 0; h < kMaxHot; ++h) {
        // centres at step 0 (t = t0) and velocities, reduced into the grid on the host
        const bool on = h < cfg->nhot;
        a.hx_first[h] = on ? moved(cfg->hx0[h], cfg->hvx[h], cfg->t0, P.nx) : 0;
        a.hy_first[h] = on ? moved(cfg->hy0[h], cfg->hvy[h], cfg->t0, P.ny) : 0;
        a.hvx[h] = on ? wrap(cfg->hvx[h], P.nx) : 0;
        a.hvy[h] = on ? wrap(cfg->hvy[h], P.ny) : 0;
    }
    a.cc = cfg->c_center; a.cn = cfg->c_nbr; a.eps = cfg->eps;

    x->err.clear();
    int r;
    // zero the whole workspace, then fill tables
    if ((r = launch_zero(x->ws, P.ws_bytes, x->stream)) != 0) return hip_bail(static_cast<hipError_t>(r), "zero workspace");
    if ((e = hipMemcpyAsync(x->ws + P.off_ktab, ktab.data(), sizeof(int32_t) * ktab.size(),
                            hipMemcpyHostToDevice, x->stream)) != hipSuccess) return hip_bail(e, "upload cost table");
    if ((r = launch_reset_control(a, x->stream)) != 0) return hip_bail(static_cast<hipError_t>(r), "reset control");
    if (init_field) {
        if ((e = hipMemcpyAsync(x->field[0], init_field, P.field_bytes, hipMemcpyDefault, x->stream)) != hipSuccess)
            return hip_bail(e, "copy initial field");
    } else {
        if ((r = launch_init_field(x->field[0], P.prec, P.ncells * P.nfields, cfg->seed, x->stream)) != 0)
            return hip_bail(static_cast<hipError_t>(r), "init field");
    }
    x->map.assign(static_cast<size_t>(P.C), 0);
    block_map(P.C, P.S, x->map.data());
    if ((r = upload_plan(x, nullptr, nullptr)) != LB_OK) {
        g_err = x->err;
        return bail(r);
    }
    if ((e = hipStreamSynchronize(x->stream)) != hipSuccess) return hip_bail(e, "hipStreamSynchronize");
    *out = x;
    return LB_OK;
}

int lb_step(lb_ctx* x, int32_t nsteps, int32_t mode) {
    if (!x) return fail(nullptr, LB_E_INVAL, "ctx is NULL");
    if (x->broken) return fail(&x->err, LB_E_STATE, "context unusable: an earlier step failed part-way");
    if (nsteps < 0) return fail(&x->err, LB_E_INVAL, "nsteps must be >= 0");
    if (mode < LB_PLAIN || mode > LB_PERSISTENT_EAGER) return fail(&x->err, LB_E_INVAL, "unknown mode");
    if (forced_failure("step")) return fail(&x->err, LB_E_HIP, "forced failure at step (LBGRID_FAIL_AT)");
    HIP_TRY(x, hipSetDevice(x->device));
    const Plan& p = x->plan;
    if (nsteps == 0) return LB_OK;
    // Every step is counted as soon as all of its launches are enqueued, so that
    // on a failure `steps` still names the buffer and checksum slot the device
    // state is in.  A step that fails after some of its launches (the plain
    // form's per-chunk launches) leaves a partly applied step behind: the
    // context is then marked unusable.
    const int fail_at = forced_launch_failure();
    int launches = 0;
    auto forced = [&]() { return fail_at > 0 && ++launches == fail_at; };
    // every launch moves the field to the other copy: n steps take n launches,
    // or launches_for(n) when balanced launches fuse steps
    auto done = [&](int n, bool balanced) {
        x->steps += n;
        x->window_steps += n;
        x->cur ^= ((balanced ? launches_for(p, n) : n) & 1);
    };
    auto launch_failed = [&](const char* what, int e, bool partial) {
        if (partial) x->broken = true;
        return fail(&x->err, LB_E_HIP, std::string(what) + ": " +
                                           (e ? hipGetErrorString(static_cast<hipError_t>(e))
                                              : "forced launch failure (LBGRID_FAIL_AT)"));
    };
    int rc;
    // Forms that read every workgroup's own copy of the step state need it
    // refreshed after steps launched one workgroup per item.
    const bool own_state = !(p.IG && (mode == LB_PERSISTENT || mode == LB_PERSISTENT_EAGER));
    if (own_state && x->wstate_stale) {
        LAUNCH_TRY(x, launch_seed_state(x->args, static_cast<int>(x->steps & kSlotMask), x->stream));
        x->wstate_stale = false;
    }
    if (!own_state) x->wstate_stale = true;
    if ((mode == LB_PLAIN || mode == LB_PLAIN_GRAPH) && x->items_stale && (rc = upload_items(x)) != LB_OK)
        return rc;
    switch (mode) {
        case LB_PERSISTENT: {
            const int R = x->cfg.graph_steps;
            if (p.IG) {
                // graphs per slot of their first step, retaken when the plan changes
                for (int k = 0; k < kStepSlots; ++k)
                    if (x->items_graph_version[k] != x->plan_version) {
                        if (x->g_items[k]) HIP_TRY(x, hipGraphExecDestroy(x->g_items[k]));
                        if (x->g_items1[k]) HIP_TRY(x, hipGraphExecDestroy(x->g_items1[k]));
                        x->g_items[k] = x->g_items1[k] = nullptr;
                        x->items_graph_version[k] = x->plan_version;
                    }
                for (int i = 0; i < nsteps / R; ++i) {
                    const int sl = static_cast<int>(x->steps & kSlotMask);
                    if (!x->g_items[sl] && (rc = capture(x, LB_PERSISTENT, R, &x->g_items[sl], sl)) != LB_OK)
                        return rc;
                    if (forced()) return launch_failed("hipGraphLaunch", 0, false);
                    if (int e = hipGraphLaunch(x->g_items[sl], x->stream)) return launch_failed("hipGraphLaunch", e, false);
                    done(R, true);
                }
                for (int i = 0; i < nsteps % R;) {
                    const int sl = static_cast<int>(x->steps & kSlotMask);
                    const int n = launch_span(p, nsteps % R - i);
                    if (n >= 2) {   // fused steps of the remainder: one launch, not worth a graph
                        if (forced()) return launch_failed("launch_balanced", 0, false);
                        if (int e = launch_balanced(x, sl, n, x->stream)) return launch_failed("launch_balanced", e, false);
                    } else {
                        if (!x->g_items1[sl] && (rc = capture(x, LB_PERSISTENT, 1, &x->g_items1[sl], sl)) != LB_OK)
                            return rc;
                        if (forced()) return launch_failed("hipGraphLaunch", 0, false);
                        if (int e = hipGraphLaunch(x->g_items1[sl], x->stream)) return launch_failed("hipGraphLaunch", e, false);
                    }
                    done(n, true);
                    i += n;
                }
                break;
            }
            if (nsteps >= R && !x->g_pers && (rc = capture(x, LB_PERSISTENT, R, &x->g_pers)) != LB_OK) return rc;
            if (nsteps % R && !x->g_pers1 && (rc = capture(x, LB_PERSISTENT, 1, &x->g_pers1)) != LB_OK) return rc;
            for (int i = 0; i < nsteps / R; ++i) {
                if (forced()) return launch_failed("hipGraphLaunch", 0, false);
                if (int e = hipGraphLaunch(x->g_pers, x->stream)) return launch_failed("hipGraphLaunch", e, false);
                done(R, true);
            }
            for (int i = 0; i < nsteps % R; ++i) {
                if (forced()) return launch_failed("hipGraphLaunch", 0, false);
                if (int e = hipGraphLaunch(x->g_pers1, x->stream)) return launch_failed("hipGraphLaunch", e, false);
                done(1, true);
            }
            break;
        }
        case LB_PERSISTENT_EAGER:
            for (int i = 0; i < nsteps;) {
                const int n = launch_span(p, nsteps - i);
                if (forced()) return launch_failed("launch_balanced", 0, false);
                if (int e = launch_balanced(x, static_cast<int>(x->steps & kSlotMask), n, x->stream))
                    return launch_failed("launch_balanced", e, false);
                done(n, true);
                i += n;
            }
            break;
        case LB_PLAIN_GRAPH:
            if (x->g_plain && x->plain_graph_version != x->plan_version) {  // grid sizes changed
                HIP_TRY(x, hipGraphExecDestroy(x->g_plain));
                x->g_plain = nullptr;
            }
            if (!x->g_plain) {
                if ((rc = capture(x, LB_PLAIN, 1, &x->g_plain)) != LB_OK) return rc;
                x->plain_graph_version = x->plan_version;
            }
            for (int i = 0; i < nsteps; ++i) {
                if (forced()) return launch_failed("hipGraphLaunch", 0, false);
                if (int e = hipGraphLaunch(x->g_plain, x->stream)) return launch_failed("hipGraphLaunch", e, false);
                done(1, false);
            }
            break;
        default:  // LB_PLAIN: C launches and a finisher per step
            for (int i = 0; i < nsteps; ++i) {
                for (int32_t c = 0; c <= p.C; ++c) {
                    const bool partial = c > 0;   // some of this step's launches are already enqueued
                    if (forced()) return launch_failed(c < p.C ? "launch_plain_chunk" : "launch_finish", 0, partial);
                    const int e = c < p.C ? launch_plain_chunk(x->args, p.prec, p.vec, c,
                                                               x->item_off[c + 1] - x->item_off[c], p.block,
                                                               p.lds, x->stream)
                                          : launch_finish(x->args, x->stream);
                    if (e) return launch_failed(c < p.C ? "launch_plain_chunk" : "launch_finish", e, partial);
                }
                done(1, false);
            }
    }
    return LB_OK;
}

int lb_measure_begin(lb_ctx* x, int32_t source, int32_t reset) {
    if (!x) return fail(nullptr, LB_E_INVAL, "ctx is NULL");
    if (x->broken) return fail(&x->err, LB_E_STATE, "context unusable: an earlier step failed part-way");
    if (source != LB_LOAD_WORK && source != LB_LOAD_TIME) return fail(&x->err, LB_E_INVAL, "unknown load source");
    if (x->measure_pending) return fail(&x->err, LB_E_STATE, "a measurement is pending: call lb_measure_end first");
    const Plan& p = x->plan;
    HIP_TRY(x, hipSetDevice(x->device));
    // one kernel moves the loads and tile work into pinned staging after the
    // window's last step and clears the counters (work, time, busy and tile
    // counters are adjacent in the workspace); an event marks its end
    LAUNCH_TRY(x, launch_measure_out(
                      reinterpret_cast<double*>(x->ws + (source == LB_LOAD_WORK ? p.off_lw : p.off_lt)),
                      reinterpret_cast<double*>(x->ws + p.off_tw), p.C, p.ntiles,
                      reinterpret_cast<double*>(const_cast<char*>(x->staging_dev) + p.st_loads),
                      reinterpret_cast<double*>(const_cast<char*>(x->staging_dev) + p.st_tiles),
                      x->ws + p.off_lw, reset ? p.off_busy + sizeof(double) * busy_slots(p) - p.off_lw : 0,
                      x->stream));
    HIP_TRY(x, hipEventRecord(x->measured_ev, x->stream));
    x->measure_pending = true;
    x->pending_steps = x->window_steps;
    if (reset) x->window_steps = 0;
    return LB_OK;
}

int lb_measure_end(lb_ctx* x, double* loads_out) {
    if (!x) return fail(nullptr, LB_E_INVAL, "ctx is NULL");
    if (!x->measure_pending) return fail(&x->err, LB_E_STATE, "no measurement begun");
    const Plan& p = x->plan;
    HIP_TRY(x, hipSetDevice(x->device));
    if (forced_failure("sync")) return fail(&x->err, LB_E_HIP, "forced failure at sync (LBGRID_FAIL_AT)");
    // poll the event: the measurement sits on the critical path between two
    // windows, and polling returns sooner than a blocking wait on this system
    hipError_t q;
    while ((q = hipEventQuery(x->measured_ev)) == hipErrorNotReady) {
    }
    x->measure_pending = false;
    if (q != hipSuccess) return fail(&x->err, LB_E_HIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
    const double* st = reinterpret_cast<const double*>(x->staging + p.st_loads);
    const double* stt = reinterpret_cast<const double*>(x->staging + p.st_tiles);
    x->measured.assign(st, st + p.C);
    x->tile_measured.assign(stt, stt + p.ntiles);
    x->tile_steps = x->pending_steps;
    x->have_measured = true;
    if (loads_out) std::memcpy(loads_out, x->measured.data(), sizeof(double) * p.C);
    return LB_OK;
}

int lb_measure(lb_ctx* x, int32_t source, double* loads_out, int32_t reset) {
    int rc = lb_measure_begin(x, source, reset);
    if (rc != LB_OK) return rc;
    return lb_measure_end(x, loads_out);
}

int lb_balance_host(const double* loads, const int32_t* old_map, int32_t C, int32_t S,
                    int32_t strategy, double threshold, int32_t* map_out, int32_t* nmigrated) {
    if (C < 0 || S < 1) return fail(nullptr, LB_E_INVAL, "need C >= 0 and S >= 1");
    if (C > 0 && (!loads || !map_out)) return fail(nullptr, LB_E_INVAL, "loads and map_out are required");
    if (strategy != LB_GREEDY && strategy != LB_REFINE && strategy != LB_REFINESWAP &&
        strategy != LB_GREEDY_THEN_REFINESWAP)
        return fail(nullptr, LB_E_INVAL, "unknown strategy");
    if (strategy == LB_GREEDY_THEN_REFINESWAP) strategy = old_map ? LB_REFINESWAP : LB_GREEDY;
    std::vector<int32_t> base(static_cast<size_t>(C));
    if (old_map) {
        for (int32_t c = 0; c < C; ++c) {
            if (old_map[c] < 0 || old_map[c] >= S) return fail(nullptr, LB_E_INVAL, "old_map entry out of range");
            base[c] = old_map[c];
        }
    } else {
        if (strategy != LB_GREEDY) return fail(nullptr, LB_E_INVAL, "refinement needs old_map");
        block_map(C, S, base.data());
    }
    int rc = balance(loads, base.data(), C, S, strategy, threshold, map_out);
    if (rc == -2) return fail(nullptr, LB_E_UNSUPPORTED, "strategy not implemented");
    if (rc != 0) return fail(nullptr, LB_E_INVAL, "invalid loads or threshold (loads must be >= 0, threshold > 0)");
    if (nmigrated) {
        int32_t n = 0;
        for (int32_t c = 0; c < C; ++c) n += (map_out[c] != base[c]);
        *nmigrated = n;
    }
    return LB_OK;
}

int lb_rebalance(lb_ctx* x, int32_t strategy, double threshold, const double* loads,
                 int32_t* map_out, int32_t* nmigrated, double* lam) {
    if (!x) return fail(nullptr, LB_E_INVAL, "ctx is NULL");
    if (x->broken) return fail(&x->err, LB_E_STATE, "context unusable: an earlier step failed part-way");
    const Plan& p = x->plan;
    const double* w = loads;
    if (!w) {
        if (x->measure_pending)
            return fail(&x->err, LB_E_STATE, "a measurement is pending: call lb_measure_end first");
        if (!x->have_measured) return fail(&x->err, LB_E_STATE, "no measured loads: call lb_measure first or pass loads");
        w = x->measured.data();
    }
    const auto t_bal = std::chrono::steady_clock::now();
    std::vector<int32_t> nm(static_cast<size_t>(p.C));
    int32_t mig = 0;
    if (strategy == LB_GREEDY_THEN_REFINESWAP)  // Experiment C: Greedy first, RefineSwap later
        strategy = x->rebalances == 0 ? LB_GREEDY : LB_REFINESWAP;
    int rc = lb_balance_host(w, x->map.data(), p.C, p.S, strategy, threshold, nm.data(), &mig);
    if (rc != LB_OK) {
        x->err = g_err;
        return rc;
    }
    x->host_balance_us +=
        std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t_bal).count();
    const double before = imbalance(w, x->map.data(), p.C, p.S);
    const double after = imbalance(w, nm.data(), p.C, p.S);
    x->map = nm;
    HIP_TRY(x, hipSetDevice(x->device));
    // measured loads come with the measured work of every tile, which cuts the items
    const double* tw = (!loads && !x->tile_measured.empty()) ? x->tile_measured.data() : nullptr;
    if ((rc = upload_plan(x, w, tw)) != LB_OK) return rc;
    ++x->rebalances;
    if (map_out) std::memcpy(map_out, nm.data(), sizeof(int32_t) * p.C);
    if (nmigrated) *nmigrated = mig;
    if (lam) {
        lam[0] = before;
        lam[1] = after;
    }
    return LB_OK;
}

int lb_set_map(lb_ctx* x, const int32_t* map, const double* cost) {
    if (!x) return fail(nullptr, LB_E_INVAL, "ctx is NULL");
    if (x->broken) return fail(&x->err, LB_E_STATE, "context unusable: an earlier step failed part-way");
    if (!map) return fail(&x->err, LB_E_INVAL, "map is NULL");
    const Plan& p = x->plan;
    for (int32_t c = 0; c < p.C; ++c)
        if (map[c] < 0 || map[c] >= p.S) return fail(&x->err, LB_E_INVAL, "map entry out of range");
    if (cost)
        for (int32_t c = 0; c < p.C; ++c)
            if (!(cost[c] >= 0.0)) return fail(&x->err, LB_E_INVAL, "costs must be >= 0");
    x->map.assign(map, map + p.C);
    HIP_TRY(x, hipSetDevice(x->device));
    return upload_plan(x, cost, nullptr);
}

int lb_fields(lb_ctx* x, int32_t field, void* dst, size_t dst_bytes, double* checksum_out) {
    if (!x) return fail(nullptr, LB_E_INVAL, "ctx is NULL");
    if (x->broken) return fail(&x->err, LB_E_STATE, "context unusable: an earlier step failed part-way");
    const Plan& p = x->plan;
    if (field < 0 || field >= p.nfields) return fail(&x->err, LB_E_INVAL, "field index out of range");
    const size_t bytes = static_cast<size_t>(p.ncells) * p.elem;
    if (dst && dst_bytes < bytes) return fail(&x->err, LB_E_NOMEM, "dst too small");
    HIP_TRY(x, hipSetDevice(x->device));
    const char* cur = static_cast<const char*>(x->field[x->cur]) + static_cast<size_t>(field) * bytes;
    if (checksum_out) {
        double* part = reinterpret_cast<double*>(x->ws + p.off_sum);
        LAUNCH_TRY(x, launch_field_sum(cur, p.prec, p.ncells, part, part + kSumBlocks, x->stream));
    }
    if (dst) HIP_TRY(x, hipMemcpyAsync(dst, cur, bytes, hipMemcpyDefault, x->stream));
    int rc = sync(x);
    if (rc != LB_OK) return rc;
    if (checksum_out)
        HIP_TRY(x, hipMemcpy(checksum_out, x->ws + p.off_sum + sizeof(double) * kSumBlocks, sizeof(double),
                             hipMemcpyDeviceToHost));
    return LB_OK;
}

int lb_stats(lb_ctx* x, lb_stats_t* out) {
    if (!x || !out) return fail(x ? &x->err : nullptr, LB_E_INVAL, "ctx and out are required");
    HIP_TRY(x, hipSetDevice(x->device));
    LAUNCH_TRY(x, launch_flush(x->args, x->stream));   // the last step's checksum
    int rc = sync(x);
    if (rc != LB_OK) return rc;
    const Plan& p = x->plan;
    std::memset(out, 0, sizeof(*out));
    out->steps = x->steps;
    out->nchunks = p.C;
    out->ntiles = p.ntiles;
    out->nrows = p.nrows;
    out->nitems = static_cast<int32_t>(x->items.size());
    out->host_balance_us = x->host_balance_us;
    out->busy_slots = busy_slots(x->plan);
    out->host_plan_us = x->host_plan_us;
    out->nslots = p.S;
    out->nqueues = p.Q;
    out->nwg = p.nwg;
    out->block = p.block;
    out->block2 = p.block2;
    out->block3 = p.block3;
    out->tile_x = p.TX;
    out->tile_y = p.TY;
    out->clock_hz = x->clock_hz;
    out->measured_steps = x->window_steps;
    if (x->steps > 0)
        HIP_TRY(x, hipMemcpy(&out->last_checksum,
                             x->ws + p.off_hist + sizeof(double) * ((x->steps - 1) % kHistLen),
                             sizeof(double), hipMemcpyDeviceToHost));
    return LB_OK;
}

int lb_wg_busy(lb_ctx* x, double* out, int32_t n) {
    if (!x || !out) return fail(x ? &x->err : nullptr, LB_E_INVAL, "ctx and out are required");
    const int32_t slots = busy_slots(x->plan);
    if (n < slots) return fail(&x->err, LB_E_NOMEM, "out too small for the busy slots (lb_stats busy_slots)");
    int rc = sync(x);
    if (rc != LB_OK) return rc;
    HIP_TRY(x, hipMemcpy(out, x->ws + x->plan.off_busy, sizeof(double) * slots, hipMemcpyDeviceToHost));
    return LB_OK;
}

int lb_wg_timeline(lb_ctx* x, double* out, int32_t n) {
    if (!x || !out) return fail(x ? &x->err : nullptr, LB_E_INVAL, "ctx and out are required");
    const Plan& p = x->plan;
    if (n < 4 * p.nwg) return fail(&x->err, LB_E_NOMEM, "out too small for 4 * nwg entries");
    int rc = sync(x);
    if (rc != LB_OK) return rc;
    std::vector<uint64_t> t(4 * static_cast<size_t>(p.nwg));
    HIP_TRY(x, hipMemcpy(t.data(), x->ws + p.off_tl, sizeof(uint64_t) * t.size(), hipMemcpyDeviceToHost));
    uint64_t t0 = UINT64_MAX;
    for (int32_t w = 0; w < p.nwg; ++w) t0 = std::min(t0, t[4 * w]);
    for (size_t i = 0; i < t.size(); ++i)
        out[i] = t[i] >= t0 ? static_cast<double>(t[i] - t0) / x->clock_hz * 1e6 : 0.0;
    return LB_OK;
}

int lb_visits(lb_ctx* x, int32_t* out, int32_t n, int32_t reset) {
    if (!x) return fail(nullptr, LB_E_INVAL, "ctx is NULL");
    const Plan& p = x->plan;
    if (out && n < p.nrows) return fail(&x->err, LB_E_NOMEM, "out too small for nrows entries");
    int rc = sync(x);
    if (rc != LB_OK) return rc;
    if (out) HIP_TRY(x, hipMemcpy(out, x->ws + p.off_visits, sizeof(int32_t) * p.nrows, hipMemcpyDeviceToHost));
    if (reset) {
        LAUNCH_TRY(x, launch_zero(x->ws + p.off_visits, sizeof(int32_t) * p.nrows, x->stream));
        return sync(x);
    }
    return LB_OK;
}

int lb_checksums(lb_ctx* x, double* out, int32_t n, int32_t* got) {
    if (!x || !out || !got) return fail(x ? &x->err : nullptr, LB_E_INVAL, "ctx, out and got are required");
    if (x->broken) return fail(&x->err, LB_E_STATE, "context unusable: an earlier step failed part-way");
    HIP_TRY(x, hipSetDevice(x->device));
    LAUNCH_TRY(x, launch_flush(x->args, x->stream));   // the last step's checksum
    int rc = sync(x);
    if (rc != LB_OK) return rc;
    const int64_t avail = std::min<int64_t>(x->steps, kHistLen);
    const int64_t m = std::min<int64_t>(avail, std::max(n, 0));
    std::vector<double> ring(kHistLen);
    HIP_TRY(x, hipMemcpy(ring.data(), x->ws + x->plan.off_hist, sizeof(double) * kHistLen, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < m; ++i) out[i] = ring[(x->steps - m + i) % kHistLen];
    *got = static_cast<int32_t>(m);
    return LB_OK;
}

void lb_destroy(lb_ctx* x) {
    if (!x) return;
    (void)hipSetDevice(x->device);
    if (x->stream || x->cap) (void)hipStreamSynchronize(x->stream);
    if (x->g_pers) (void)hipGraphExecDestroy(x->g_pers);
    if (x->g_pers1) (void)hipGraphExecDestroy(x->g_pers1);
    for (int k = 0; k < kStepSlots; ++k) {
        if (x->g_items[k]) (void)hipGraphExecDestroy(x->g_items[k]);
        if (x->g_items1[k]) (void)hipGraphExecDestroy(x->g_items1[k]);
    }
    if (x->g_plain) (void)hipGraphExecDestroy(x->g_plain);
    if (x->upload_done) (void)hipEventDestroy(x->upload_done);
    if (x->measured_ev) (void)hipEventDestroy(x->measured_ev);
    if (x->staging) (void)hipHostFree(x->staging);
    if (x->cap) (void)hipStreamDestroy(x->cap);
    delete x;
}

const char* lb_last_error(const lb_ctx* x) {
    if (x) return x->err.c_str();
    return g_err.c_str();
}

}  // extern "C"
