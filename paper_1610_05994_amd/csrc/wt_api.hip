// Host runtime behind include/wtree.h: layouts, argument checks, launch
// sequences, handles and query wrappers.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "wt_internal.h"
#include "wtree.h"
#include "wtree_prof.h"

struct wt_tree {
    wt::Layout L;
    uint8_t *tree;         // caller's tree memory
    hipStream_t stream;    // stream the build was enqueued on
    int device;
    uint64_t *d_query;     // lazily allocated scratch for the single queries
    // Huffman-shaped tree: its table (host copy) and the host buffer of the
    // tables copied into the tree memory by the build (kept until wt_free)
    wt::HuffMeta *hm;
    uint8_t *htab;
};

namespace wt {

// ------------------------------------------------------------- profiling --
// While on, each enqueued kernel is bracketed by two events on its stream.
struct ProfEntry {
    wt_prof_rec rec;
    hipEvent_t a, b;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<ProfEntry> g_prof;
static std::vector<hipEvent_t> g_event_pool;

static hipEvent_t prof_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    // Timing only, on the device: without the system-scope fence a record
    // costs no cache writeback and invalidate, which would otherwise stall
    // the stream for several microseconds at every record.
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// Opens a record; returns its index or -1 when profiling is off.
static long prof_begin(hipStream_t st, const char *kernel, uint32_t level, uint32_t width, uint64_t n,
                       uint64_t bytes) {
    if (!g_prof_on) return -1;
    std::lock_guard<std::mutex> g(g_prof_mu);
    ProfEntry e;
    memset(&e.rec, 0, sizeof(e.rec));
    strncpy(e.rec.kernel, kernel, sizeof(e.rec.kernel) - 1);
    e.rec.level = level;
    e.rec.width = width;
    e.rec.n = n;
    e.rec.bytes = bytes;
    e.a = prof_event();
    e.b = prof_event();
    if (!e.a || !e.b) return -1;
    (void)hipEventRecord(e.a, st);
    g_prof.push_back(e);
    return (long)g_prof.size() - 1;
}

static void prof_end(long idx, hipStream_t st) {
    if (idx < 0) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    if ((size_t)idx < g_prof.size()) (void)hipEventRecord(g_prof[idx].b, st);
}

// ---------------------------------------------------------- tuning table --
// Geometry per (mode: single or batched build, width class, levels,
// floor lg n): 0 = the default, kGeomSmall / kGeomMid = one workgroup per
// sequence (64 KB / 160 KB of LDS), 32 / 64 / 128 = tiled level passes with
// that many bytes per lane.  Filled
// by wt_tune_set (the autotuner writes a table that the Python binding
// loads); read by every layout computation, so a footprint and the build
// that uses it must see the same table.
static uint8_t g_tune[2][3][25][41];

static int wclass(uint32_t w) { return w == 1 ? 0 : (w == 2 ? 1 : 2); }
static uint32_t floor_lg(uint64_t n) {
    uint32_t k = 0;
    while (k < 40 && (2ull << k) <= n) k++;
    return k;
}

// The default: short sequences take the smallest one-workgroup build that
// holds them, longer ones 64 bytes per lane.  A one-workgroup geometry that
// cannot hold the sequence falls back to the default.
static uint32_t resolve_geometry(uint32_t v, uint64_t n, uint32_t width) {
    if (v == kGeomSmall || v == kGeomMid) {
        if (n <= one_wg_cap(width, v)) return v;
        v = 0;
    }
    if (v == 0) {
        if (n <= one_wg_cap(width, kGeomSmall)) return kGeomSmall;
        if (n <= one_wg_cap(width, kGeomMid)) return kGeomMid;
        return kDefaultLaneBytes;
    }
    return lane_bytes_valid(width, v) ? v : kDefaultLaneBytes;
}

uint32_t tuned_geometry(uint64_t n, uint32_t sigma, uint32_t width, bool batched) {
    const uint32_t l = levels_for(sigma);
    return resolve_geometry(g_tune[batched ? 1 : 0][wclass(width)][l < 25 ? l : 24][floor_lg(n)], n, width);
}

// Bytes per symbol that hold `bits` bits.
static uint32_t bytes_for(uint32_t bits) { return bits <= 8 ? 1u : (bits <= 16 ? 2u : 4u); }

// Builds of at least this many symbols narrow their symbol orders (smaller
// ones are bound by launches, not bytes, and the anchor tables cost one).
constexpr uint64_t kNarrowMinN = 1ull << 18;

// Narrowed orders of a single binary-tree build (2- and 4-byte symbols):
// T_{i+1} halves the width of T_i as soon as the levels after i fit in half
// of it, where a narrowing pass exists for the width and the lane's symbol
// count E, and where the anchor nodes the half width needs are few beside
// the tiles (a tile over two anchors takes the slower direct split: at most
// one tile in kAnchorTiles may); a width whose 8w bits hold fewer bits than
// the levels gets the per-tile anchor table of level levels - 8w.  The
// narrower order keeps E symbols per lane (the same tiles), or takes 2E
// (tiles of twice the symbols, as many bytes per lane as before) where the
// tuning table runs that width, at this length and number of levels, with
// at least that many symbols per lane, and where most levels of that width
// still take the single-node split at the larger tiles (their nodes average
// kMultiAvgTiles tiles or more; always in a wavelet matrix).  Larger tiles
// move a tile's bytes for less per-tile work, but span more nodes: on deep
// levels the per-node work grows more than that saves.
// A wavelet matrix (one node per level) needs no anchors: its orders narrow
// wherever the widths allow.
constexpr uint64_t kAnchorTiles = 8;
static void narrow_widths(Layout *L, bool matrix) {
    const uint32_t l = L->levels;
    L->narrow = 0;
    for (uint32_t i = 0; i <= kMaxTreeLevels; i++) {
        L->tw[i] = (uint8_t)L->width;
        L->te[i] = (uint8_t)(L->lane_bytes / L->width);
    }
    if (L->small || L->width < 2 || l < 2 || L->n < kNarrowMinN) return;
    for (uint32_t i = 0; i + 1 < l; i++) {
        const uint32_t w = L->tw[i], E = L->te[i];
        const uint32_t half_bits = 8 * (w / 2);
        // (tiles of 64 e symbols, against the anchor nodes of the half width)
        auto few_anchors = [&](uint32_t e) {
            return matrix || half_bits >= l || (kAnchorTiles << (l - half_bits)) <= ceil_div(L->n, 64ull * e);
        };
        const bool halve = w >= 2 && bytes_for(l - (i + 1)) <= w / 2 && narrowing_pass(w, E * w) && few_anchors(E);
        uint32_t en = E;
        if (halve && 2 * E <= 64 && narrowing_pass_doubling(w, E * w) && few_anchors(2 * E)) {
            const uint32_t rest = l - (i + 1);
            const uint32_t want = resolve_geometry(g_tune[0][wclass(w / 2)][rest < 25 ? rest : 24][floor_lg(L->n)],
                                                   L->n, w / 2);
            // the levels of the half width (T_j of w / 2 bytes) whose average
            // node still spans enough doubled tiles for the single-node split
            uint32_t total = 0, single = 0;
            for (uint32_t j = i + 1; j < l && (w / 2 == 1 || bytes_for(l - j) > w / 4); j++) {
                total++;
                single += (matrix || !level_multi(L->n, j, w / 2, E * w)) ? 1u : 0u;
            }
            if (want != kGeomSmall && want != kGeomMid && want >= E * w && 2 * single >= total) en = 2 * E;
        }
        L->tw[i + 1] = (uint8_t)(halve ? w / 2 : w);
        L->te[i + 1] = (uint8_t)(halve ? en : E);
        if (halve) L->narrow = 1;
    }
    for (uint32_t i = l; i <= kMaxTreeLevels; i++) {
        L->tw[i] = L->tw[l - 1];
        L->te[i] = L->te[l - 1];
    }
}

static void plan_narrowing(Layout *L) {
    const uint32_t l = L->levels;
    narrow_widths(L, false);
    if (!L->narrow) return;
    for (uint32_t w = 1; w <= 2; w++) {
        bool used = false;
        for (uint32_t i = 0; i < l; i++) used |= L->tw[i] == w;
        if (!used || 8 * w >= l) continue;
        L->anc_level[w - 1] = l - 8 * w;
        L->ws_tanc[w - 1] = L->work_bytes;
        L->work_bytes += round_up(L->ntiles * 8, 256);
    }
}

void make_layout(uint64_t n, uint32_t sigma, uint32_t width, bool batched, Layout *L) {
    make_layout_geom(n, sigma, width, tuned_geometry(n, sigma, width, batched), L);
    if (!batched) plan_narrowing(L);
}

void make_layout_geom(uint64_t n, uint32_t sigma, uint32_t width, uint32_t geom, Layout *L) {
    memset(L, 0, sizeof(*L));
    for (uint32_t i = 0; i <= kMaxTreeLevels; i++) {  // (no narrowing)
        L->tw[i] = (uint8_t)width;
        L->te[i] = (uint8_t)((geom == kGeomSmall || geom == kGeomMid ? kDefaultLaneBytes : geom) / width);
    }
    const uint32_t l = levels_for(sigma);
    L->n = n;
    L->sigma = sigma;
    L->width = width;
    L->levels = l;
    L->words = round_up(ceil_div(n, 64), 8);
    L->rank_entries = ceil_div(n, 512) + 1;
    L->rank_stride = round_up(L->rank_entries, 8);
    L->small = (geom == kGeomSmall || geom == kGeomMid) ? geom : 0u;
    L->lane_bytes = L->small ? kDefaultLaneBytes : geom;
    L->ntiles = ceil_div(n, tile_syms(width, L->lane_bytes));
    L->nsup = ceil_div(L->ntiles, kSup);

    L->tree_bits_off = kHeaderBytes;
    L->tree_ranks_off = L->tree_bits_off + (uint64_t)l * L->words * 8;
    L->tree_bytes = L->tree_ranks_off + (uint64_t)l * L->rank_stride * 8;

    uint64_t off = 0;
    const uint64_t tbytes = round_up(n * width, 256);
    L->ws_ta = off;
    if (l >= 2) off += tbytes;
    L->ws_tb = off;
    if (l >= 3) off += tbytes;

    L->ws_ctrl = off;
    L->ws_tile_ones = off;
    off += round_up((uint64_t)l * tile_stride(L->ntiles) * 4, 256);
    L->ws_ones = off;
    off += round_up(ones_offset(l) * 8, 256);
    L->ws_fold_cnt = off;
    off += 256;
    L->ws_ctrl_bytes = off - L->ws_ctrl;

    L->ws_sup = off;
    off += round_up((uint64_t)l * L->nsup * 8, 256);
    L->ws_supsum = off;
    off += round_up((L->nsup ? L->nsup : 1) * 8, 256);
    L->ws_zo = off;
    off += round_up(zo_offset(l) * 16, 256);
    L->ws_start = off;
    off += round_up(start_offset(l) * 8, 256);
    L->ws_partials = off;
    off += round_up(kMaxScanBlocks * 8, 256);
    if (width == 1 && l >= 2) {  // a u8 build may fold its last level
        L->fold_ovf_cap = fold_ovf_capacity(L->ntiles, l, tile_syms(width, L->lane_bytes));
        L->ws_fold_own = off;
        off += round_up(2 * L->ntiles * 8, 256);
        L->ws_fold_ovf = off;
        off += round_up(L->fold_ovf_cap * 8, 256);
    }
    L->work_bytes = L->small ? 256 : off;  // the one-workgroup build needs no workspace
}

static SmallJob make_small_job(const Layout &L, const void *S, void *tree) {
    SmallJob j;
    j.S = S;
    j.tree = reinterpret_cast<uint8_t *>(tree);
    j.bits_off = L.tree_bits_off;
    j.ranks_off = L.tree_ranks_off;
    j.n = (uint32_t)L.n;
    j.sigma = L.sigma;
    j.levels = L.levels;
    j.words = (uint32_t)L.words;
    j.rank_entries = (uint32_t)L.rank_entries;
    j.rank_stride = (uint32_t)L.rank_stride;
    j.matrix = L.matrix;
    return j;
}

// 4-ary tree: the binary passes of a tiled build (the one-workgroup build
// writes binary levels only), with the tree holding digit levels and their
// directories and the workspace the directory's workgroup sums.
static uint64_t dir_wgs(uint64_t n) { return ceil_div(ceil_div(n, 512), kDirBlocksPerWG); }

static void make_layout4(uint64_t n, uint32_t sigma, uint32_t width, Layout *L) {
    uint32_t g = tuned_geometry(n, sigma, width, false);
    if (g == kGeomSmall || g == kGeomMid) g = 32;
    // the tables of a binary split over the code padded to an even number of
    // bits (2 L4), read two levels at a time by the four-way passes
    const uint32_t l4 = (levels_for(sigma) + 1) / 2;
    make_layout_geom(n, (uint32_t)(1ull << (2 * l4)), width, g, L);
    L->sigma = sigma;
    L->arity = 4;
    L->levels4 = l4;
    L->dwords = round_up(ceil_div(n, 32), 8);
    L->tree_bits_off = L->tree_ranks_off = 0;  // no binary levels
    L->tree_digits_off = kHeaderBytes;
    L->tree_dir_off = L->tree_digits_off + (uint64_t)L->levels4 * L->dwords * 8;
    L->tree_bytes = L->tree_dir_off + (uint64_t)L->levels4 * L->rank_stride * 32;
    L->ws_dsum = L->work_bytes;
    L->work_bytes += round_up((uint64_t)(L->levels4 ? L->levels4 : 1) * (dir_wgs(n) ? dir_wgs(n) : 1) * 32, 256);
    // four-way passes: their two extra tile counts are cleared with the
    // control area, so they go right after it and the area grows over them
    // (everything that followed the control area moves up)
    const uint64_t stride = tile_stride(L->ntiles);
    const uint64_t qcnt_bytes = round_up(2ull * (L->levels4 ? L->levels4 : 1) * stride * 4, 256);
    const uint64_t ctrl_end = L->ws_ctrl + L->ws_ctrl_bytes;
    uint64_t *after[] = {&L->ws_sup, &L->ws_supsum, &L->ws_zo, &L->ws_start, &L->ws_partials,
                         &L->ws_fold_own, &L->ws_fold_ovf, &L->ws_dsum};
    for (uint64_t *o : after)
        if (*o >= ctrl_end) *o += qcnt_bytes;
    L->ws_qcnt = ctrl_end;
    L->ws_ctrl_bytes += qcnt_bytes;
    L->work_bytes += qcnt_bytes;
    const uint64_t nsup = L->nsup ? L->nsup : 1;
    L->ws_qsup = L->work_bytes;
    L->work_bytes += round_up(2ull * (L->levels4 ? L->levels4 : 1) * nsup * 8, 256);
    L->ws_qsupsum = L->work_bytes;
    L->work_bytes += round_up(3ull * nsup * 8, 256);
    L->ws_qpartials = L->work_bytes;
    const uint64_t top = L->levels >= 2 ? (1ull << (L->levels - 2)) : 1;  // nodes of the last four-way level
    L->work_bytes += round_up(3ull * ceil_div(top, 1024) * 8, 256);
}

// Whether the last level of a build is folded into the pass before it:
// binary u8 trees whose level l-2 pass runs the plain kernel variant (whose
// split paths can emit bits).  The pass then writes the last level's bitmap
// directly, T_{l-1} is never written, the last pass is not run, and the
// last directory comes from the bitmap.  Not for partial trees of a
// buffered build, whose last-level node tables the merge reads.
static bool fold_last_level(const Layout &L, bool partial) {
    const uint32_t l = L.levels;
    return !partial && !L.matrix && L.arity != 4 && L.width == 1 && l >= 2 && L.n > 0 &&
           !level_multi(L.n, l - 2, L.width, L.lane_bytes);
}

// Enqueue every kernel of one build.  Arguments are already validated.
static hipError_t enqueue_build(const void *S, const Layout &L, uint8_t *tree, uint8_t *work, hipStream_t st,
                                bool partial = false) {
    const uint32_t l = L.levels;
    if (L.small) {
        long pr = prof_begin(st, "small", 0, L.width, L.n, L.n * L.width + (L.words + L.rank_stride) * 8 * l);
        hipError_t err = launch_small_one(make_small_job(L, S, tree), L.width, L.small, st);
        prof_end(pr, st);
        return err;
    }
    uint32_t *tree_status = reinterpret_cast<uint32_t *>(tree);
    uint64_t *bits = reinterpret_cast<uint64_t *>(tree + L.tree_bits_off);
    uint64_t *ranks = reinterpret_cast<uint64_t *>(tree + L.tree_ranks_off);
    uint32_t *tile_ones = reinterpret_cast<uint32_t *>(work + L.ws_tile_ones);
    unsigned long long *supsum = reinterpret_cast<unsigned long long *>(work + L.ws_supsum);
    unsigned long long *ones = reinterpret_cast<unsigned long long *>(work + L.ws_ones);
    unsigned long long *sup = reinterpret_cast<unsigned long long *>(work + L.ws_sup);
    ulonglong2 *zo = reinterpret_cast<ulonglong2 *>(work + L.ws_zo);
    uint64_t *start = reinterpret_cast<uint64_t *>(work + L.ws_start);
    uint64_t *partials = reinterpret_cast<uint64_t *>(work + L.ws_partials);

    const bool fold = fold_last_level(L, partial);
    // folded: granules below n get one writer each (the pass or the stitch);
    // the words from the one holding position n on are cleared by ingest
    uint64_t *bits_last = fold ? bits + (uint64_t)(l - 1) * L.words : nullptr;
    long pr = prof_begin(st, "zero", 0, L.width, L.n, L.ws_ctrl_bytes);
    hipError_t err = launch_zero(work + L.ws_ctrl, L.ws_ctrl_bytes, tree_status,
                                 L.n == 0 ? ranks : nullptr, (uint64_t)l * L.rank_stride, st);
    prof_end(pr, st);
    if (err == hipSuccess && L.n == 0 && L.matrix && l)  // the zeros of an empty matrix
        err = launch_zero(tree + kZerosOff, (uint64_t)l * 8, tree_status, nullptr, 0, st);
    if (err != hipSuccess || L.n == 0) return err;

    IngestArgs ia;
    ia.S = S;
    ia.tile_ones0 = l ? tile_ones : nullptr;
    ia.ones0 = ones;
    ia.start0 = l ? start : nullptr;
    ia.tree_status = tree_status;
    ia.n = L.n;
    ia.ntiles = L.ntiles;
    ia.slots0 = level_slots(0);
    ia.sigma = L.sigma;
    ia.check = (L.width < 4 && (uint64_t)L.sigma == (1ull << (8 * L.width))) ? 0u : 1u;
    ia.msb = l ? l - 1 : 0;
    // (folded: the granules wholly past n; the pass and the stitch write the others)
    ia.zero_g = fold ? reinterpret_cast<uint16_t *>(bits_last) + ceil_div(L.n, 16) : nullptr;
    ia.zero_granules = fold ? 4 * L.words - ceil_div(L.n, 16) : 0;
    {
        // contiguous tiles per ingest workgroup: ~8192 workgroups
        uint64_t k = kWaves;
        while (L.ntiles > 8192 * k) k <<= 1;
        ia.tiles_per_block = k;
    }
    pr = prof_begin(st, "ingest", 0, L.width, L.n, L.n * L.width);
    err = launch_ingest(ia, L.width, L.lane_bytes, st);
    prof_end(pr, st);
    if (err != hipSuccess) return err;
    if (l == 0) return hipSuccess;

    uint8_t *tbuf[2] = {work + L.ws_ta, work + L.ws_tb};
    const uint32_t lrun = fold ? l - 1 : l;  // passes to run
    // narrowed orders: T_i has tw[i] bytes per symbol and tiles of te[i]
    // symbols per lane (E, or twice that after a narrowing to 1 byte), so
    // each level has its own tile and superchunk counts
    const bool narrow = L.narrow && !partial && L.arity != 4;
    const uint32_t E = L.lane_bytes / L.width;
    bool anc_ready[2] = {false, false};
    for (uint32_t i = 0; i < lrun; i++) {
        PlanArgs pa;
        pa.start = start + start_offset(i);
        pa.ones = ones + ones_offset(i);
        pa.zo = zo + zo_offset(i);
        pa.start_next = (i + 1 < l) ? start + start_offset(i + 1) : nullptr;
        pa.partials = partials;
        pa.nodes = L.matrix ? 1ull : 1ull << i;  // a matrix level is one node
        // a matrix level is a single node: its counters keep every slot of the
        // level's allocation (level_slots(i) << i >= kSlotSpan entries)
        pa.slots = L.matrix ? kSlotSpan : level_slots(i);
        pa.n = L.n;
        pa.matrix = L.matrix;
        pa.shift = 0;
        const bool big = pa.nodes > kScanChunk;  // one counter slot there
        // (the last level's pass writes only its bitmap and directory: a large
        // last level gets no node tables, except in a buffered build's partial
        // tree, whose last-level node tables are the leaf offsets the merge
        // reads)
        if (big && (i + 1 < l || partial)) {
            pr = prof_begin(st, "plan", i, L.width, L.n, pa.nodes * (8 + 16 + 8 + 16));
            err = launch_plan(pa, st);
            prof_end(pr, st);
            if (err != hipSuccess) return err;
        }
        const uint32_t ei = narrow ? L.te[i] : E;  // symbols per lane of T_i's tiles
        const uint64_t tiles_i = narrow ? ceil_div(L.n, 64ull * ei) : L.ntiles;
        const uint64_t nsup_i = ceil_div(tiles_i, kSup);
        PrepArgs pp;
        pp.tile_ones = tile_ones + (uint64_t)i * tile_stride(L.ntiles);
        pp.supsum = supsum;
        pp.sup = sup + (uint64_t)i * L.nsup;
        pp.ntiles = tiles_i;
        pp.nsup = nsup_i;
        pp.plan = pa;
        pp.plan_here = big ? 0u : 1u;
        pp.sums_here = (nsup_i <= kPrepSups && !big && pa.nodes < kThreads) ? 1u : 0u;
        pr = prof_begin(st, "prep", i, L.width, L.n, tiles_i * 4 + nsup_i * 16);
        err = launch_prep(pp, st);
        prof_end(pr, st);
        if (err != hipSuccess) return err;

        const uint32_t w = narrow ? L.tw[i] : L.width;
        const uint32_t wo = (narrow && i + 1 < l) ? L.tw[i + 1] : w;
        const bool anchored = narrow && !L.matrix && w < L.width && 8 * w < l;
        if (anchored && !anc_ready[w - 1]) {
            // the anchor level's node starts exist since that level's prep
            AnchorArgs an;
            an.start = start + start_offset(L.anc_level[w - 1]);
            an.nodes = 1ull << L.anc_level[w - 1];
            an.n = L.n;
            an.tile = 64ull * ei;  // (a width's levels share one tile geometry)
            an.ntiles = tiles_i;
            an.out = reinterpret_cast<uint2 *>(work + L.ws_tanc[w - 1]);
            pr = prof_begin(st, "anchor", i, w, L.n, tiles_i * 8);
            err = launch_tile_anchor(an, st);
            prof_end(pr, st);
            if (err != hipSuccess) return err;
            anc_ready[w - 1] = true;
        }

        LevelArgs a;
        memset(&a, 0, sizeof(a));
        const bool fold_here = fold && i + 1 == lrun;
        a.tin = (i == 0) ? S : tbuf[(i - 1) & 1];  // T_i for i >= 1 alternates ta, tb
        // (folded: T_{l-1} receives the edge symbols of the split only)
        a.tout = (i + 1 < lrun || fold_here) ? tbuf[i & 1] : nullptr;
        a.bits = bits + (uint64_t)i * L.words;
        a.ranks = ranks + (uint64_t)i * L.rank_stride;
        a.digits = nullptr;
        a.dwords = 0;
        a.dsh = 0;
        a.zo = zo + zo_offset(i);
        a.tile_ones = tile_ones + (uint64_t)i * tile_stride(L.ntiles);
        a.sup = sup + (uint64_t)i * L.nsup;
        a.tile_ones_next = (i + 1 < lrun) ? tile_ones + (uint64_t)(i + 1) * tile_stride(L.ntiles) : nullptr;
        a.ones_next = (i + 1 < lrun) ? ones + ones_offset(i + 1) : nullptr;
        a.nodes_next = L.matrix ? 1ull : 2ull << i;
        a.slots_next = L.matrix ? kSlotSpan : level_slots(i + 1);
        a.n = L.n;
        a.words = L.words;
        a.rank_entries = L.rank_entries;
        a.rank_stride = L.rank_stride;
        a.ntiles = tiles_i;
        a.levels = l;
        a.level = i;
        // (a narrowed symbol keeps its low 8w bits only)
        a.symmask = (uint32_t)((1ull << (8 * w < l ? 8 * w : l)) - 1);
        a.anc_start = anchored ? start + start_offset(L.anc_level[w - 1]) : nullptr;
        a.tile_anc = anchored ? reinterpret_cast<const uint2 *>(work + L.ws_tanc[w - 1]) : nullptr;
        a.matrix = L.matrix;
        a.zeros = L.matrix ? reinterpret_cast<unsigned long long *>(tree + kZerosOff) : nullptr;
        a.bits_next = fold_here ? bits_last : nullptr;
        a.n_out = L.n;
        a.fold_own = fold_here ? reinterpret_cast<uint64_t *>(work + L.ws_fold_own) : nullptr;
        a.fold_ovf = fold_here ? reinterpret_cast<uint64_t *>(work + L.ws_fold_ovf) : nullptr;
        a.fold_ovf_n = fold_here ? reinterpret_cast<unsigned int *>(work + L.ws_fold_cnt) : nullptr;
        a.fold_ovf_cap = fold_here ? L.fold_ovf_cap : 0;
        a.fold_status = tree_status;
        const uint64_t lbytes = L.n * w + ((a.tout && !fold_here) ? L.n * wo : 0) +
                                (a.bits ? L.words * 8 + L.rank_stride * 8 : 0) + (a.digits ? L.dwords * 8 : 0) +
                                (a.bits_next ? L.words * 8 : 0);
        const uint32_t lb = ei * w;  // lane bytes of T_i's tiles
        const uint32_t lbo = (narrow && i + 1 < l) ? L.te[i + 1] * wo : lb;  // and of T_{i+1}'s
        pr = prof_begin(st, "level", i, w, L.n, lbytes);
        err = launch_level(a, w, lb, !L.matrix && wo == w && level_multi(L.n, i, w, lb), wo, lbo, st);
        prof_end(pr, st);
        if (err != hipSuccess) return err;
    }
    if (fold) {
        // the granules the folded pass left to the stitch
        StitchArgs sa;
        sa.t = tbuf[(lrun - 1) & 1];
        sa.own = reinterpret_cast<const uint64_t *>(work + L.ws_fold_own);
        sa.ovf = reinterpret_cast<const uint64_t *>(work + L.ws_fold_ovf);
        sa.ovf_n = reinterpret_cast<const unsigned int *>(work + L.ws_fold_cnt);
        sa.bits16 = reinterpret_cast<uint16_t *>(bits_last);
        sa.nown = 2 * L.ntiles;
        sa.ovf_cap = L.fold_ovf_cap;
        sa.n = L.n;
        sa.sh = 0;
        pr = prof_begin(st, "stitch", l - 1, L.width, L.n, sa.nown * 8);
        err = launch_fold_stitch(sa, st);
        prof_end(pr, st);
        if (err != hipSuccess) return err;
        // the last level's directory from its bitmap; the partial sums use
        // that level's tile-count slot, which the folded pass leaves unused
        BitDirArgs d;
        d.bits = bits_last;
        d.ranks = ranks + (uint64_t)(l - 1) * L.rank_stride;
        d.wsum = reinterpret_cast<unsigned long long *>(tile_ones + (uint64_t)(l - 1) * tile_stride(L.ntiles));
        d.nblk = L.rank_entries - 1;
        d.nwg = ceil_div(d.nblk, kBitDirBlocks);
        d.rank_stride = L.rank_stride;
        pr = prof_begin(st, "bitdir", l - 1, L.width, L.n, L.words * 8 + L.rank_stride * 8);
        err = launch_bitdir(d, st);
        prof_end(pr, st);
    }
    return err;
}

// A 4-ary build: one four-way pass per digit level over the code padded to
// 2 L4 bits (digit level k is binary level 2k of that code), then the digit
// directories (also for n = 0: the level totals and padding).
static hipError_t enqueue_multiary(const void *S, const Layout &L, uint8_t *tree, uint8_t *work, hipStream_t st) {
    const uint32_t L4 = L.levels4, lp = L.levels;  // lp = 2 L4
    uint32_t *tree_status = reinterpret_cast<uint32_t *>(tree);
    uint32_t *tile_ones = reinterpret_cast<uint32_t *>(work + L.ws_tile_ones);
    uint32_t *qcnt = reinterpret_cast<uint32_t *>(work + L.ws_qcnt);
    unsigned long long *ones = reinterpret_cast<unsigned long long *>(work + L.ws_ones);
    unsigned long long *sup = reinterpret_cast<unsigned long long *>(work + L.ws_sup);
    unsigned long long *qsup = reinterpret_cast<unsigned long long *>(work + L.ws_qsup);
    unsigned long long *qsupsum = reinterpret_cast<unsigned long long *>(work + L.ws_qsupsum);
    unsigned long long *qpart = reinterpret_cast<unsigned long long *>(work + L.ws_qpartials);
    ulonglong2 *zo = reinterpret_cast<ulonglong2 *>(work + L.ws_zo);
    uint64_t *start = reinterpret_cast<uint64_t *>(work + L.ws_start);
    const uint64_t stride = tile_stride(L.ntiles), nsup = L.nsup;
    long pr = prof_begin(st, "zero", 0, L.width, L.n, L.ws_ctrl_bytes);
    hipError_t err = launch_zero(work + L.ws_ctrl, L.ws_ctrl_bytes, tree_status, nullptr, 0, st);
    prof_end(pr, st);
    if (err == hipSuccess && L.n > 0 && L4 > 0) {
        QuadIngestArgs ia;
        ia.S = S;
        ia.cnt[0] = tile_ones;
        ia.cnt[1] = qcnt;
        ia.cnt[2] = qcnt + stride;
        ia.ones_a0 = ones + ones_offset(0);
        ia.ones_b1 = ones + ones_offset(1);
        ia.slots_a0 = level_slots(0);
        ia.slots_b1 = level_slots(1);
        ia.start0 = start + start_offset(0);
        ia.tree_status = tree_status;
        ia.n = L.n;
        ia.ntiles = L.ntiles;
        ia.sigma = L.sigma;
        ia.check = (L.width < 4 && (uint64_t)L.sigma == (1ull << (8 * L.width))) ? 0u : 1u;
        ia.levels = lp;
        pr = prof_begin(st, "ingest", 0, L.width, L.n, L.n * L.width);
        err = launch_quad_ingest(ia, L.width, L.lane_bytes, st);
        prof_end(pr, st);
        uint8_t *tbuf[2] = {work + L.ws_ta, work + L.ws_tb};
        for (uint32_t k = 0; k < L4 && err == hipSuccess; k++) {
            const uint32_t i = 2 * k;
            const bool more = k + 1 < L4;
            QuadPrepArgs pp;
            pp.cnt[0] = tile_ones + (uint64_t)i * stride;
            pp.cnt[1] = qcnt + (uint64_t)(2 * k) * stride;
            pp.cnt[2] = qcnt + (uint64_t)(2 * k + 1) * stride;
            for (int j = 0; j < 3; j++) pp.supsum[j] = qsupsum + (uint64_t)j * nsup;
            pp.sup[0] = sup + (uint64_t)i * nsup;
            pp.sup[1] = qsup + (uint64_t)(2 * k) * nsup;
            pp.sup[2] = qsup + (uint64_t)(2 * k + 1) * nsup;
            pp.ntiles = L.ntiles;
            pp.nsup = nsup;
            pp.start = start + start_offset(i);
            pp.ones_a = ones + ones_offset(i);
            pp.ones_b = ones + ones_offset(i + 1);
            pp.slots_a = level_slots(i);
            pp.slots_b = level_slots(i + 1);
            pp.K = zo + zo_offset(i);  // (2 entries per node: the zo space of levels i and i + 1)
            pp.start_next = more ? start + start_offset(i + 2) : nullptr;
            pp.partials = qpart;
            pp.nodes = 1ull << i;
            pp.n = L.n;
            pr = prof_begin(st, "prep", k, L.width, L.n, L.ntiles * 12 + nsup * 48);
            err = launch_quad_prep(pp, st);
            prof_end(pr, st);
            if (err != hipSuccess) break;
            QuadArgs a;
            a.tin = (k == 0) ? S : tbuf[(k - 1) & 1];
            a.tout = more ? tbuf[k & 1] : nullptr;
            a.K = zo + zo_offset(i);
            for (int j = 0; j < 3; j++) {
                a.cnt[j] = pp.cnt[j];
                a.sup[j] = pp.sup[j];
            }
            a.cnt_next[0] = more ? tile_ones + (uint64_t)(i + 2) * stride : nullptr;
            a.cnt_next[1] = more ? qcnt + (uint64_t)(2 * k + 2) * stride : nullptr;
            a.cnt_next[2] = more ? qcnt + (uint64_t)(2 * k + 3) * stride : nullptr;
            a.ones_a_next = more ? ones + ones_offset(i + 2) : nullptr;
            a.ones_b_next = more ? ones + ones_offset(i + 3) : nullptr;
            a.nodes_a_next = 1ull << (i + 2);
            a.slots_a_next = level_slots(i + 2);
            a.nodes_b_next = 1ull << (i + 3);
            a.slots_b_next = level_slots(i + 3);
            a.n = L.n;
            a.ntiles = L.ntiles;
            a.levels = lp;
            a.level = i;
            a.symmask = (uint32_t)((1ull << lp) - 1);
            a.digits = reinterpret_cast<uint64_t *>(tree + L.tree_digits_off) + (uint64_t)k * L.dwords;
            a.dwords = L.dwords;
            const uint64_t qbytes = L.n * L.width * (more ? 2 : 1) + L.dwords * 8;
            pr = prof_begin(st, "quad", k, L.width, L.n, qbytes);
            err = launch_quad(a, L.width, L.lane_bytes, st);
            prof_end(pr, st);
        }
    }
    if (err != hipSuccess) return err;
    DigitDirArgs d;
    d.digits = reinterpret_cast<const uint64_t *>(tree + L.tree_digits_off);
    d.dir = reinterpret_cast<uint64_t *>(tree + L.tree_dir_off);
    d.wsum = reinterpret_cast<unsigned long long *>(work + L.ws_dsum);
    d.n = L.n;
    d.dwords = L.dwords;
    d.dir_stride = L.rank_stride;
    d.nblk = ceil_div(L.n, 512);
    d.wg_per_level = dir_wgs(L.n);
    d.levels = L4;
    pr = prof_begin(st, "digit_dir", 0, L.width, L.n, (uint64_t)L4 * (L.dwords * 8 + L.rank_stride * 32));
    err = launch_digit_dir(d, st);
    prof_end(pr, st);
    return err;
}

static int check_desc(const wt_desc *d) {
    if (!d) return WT_EINVAL;
    if (d->width != 1 && d->width != 2 && d->width != 4) return WT_EINVAL;
    if (d->sigma == 0 || d->sigma > WT_MAX_SIGMA) return WT_EINVAL;
    if (d->width < 4 && (uint64_t)d->sigma > (1ull << (8 * d->width))) return WT_EINVAL;
    if (d->n >= WT_MAX_N) return WT_EINVAL;
    return WT_OK;
}

static TreeView view_of(const wt_tree *t) {
    TreeView v;
    v.bits = reinterpret_cast<const uint64_t *>(t->tree + t->L.tree_bits_off);
    v.ranks = reinterpret_cast<const uint64_t *>(t->tree + t->L.tree_ranks_off);
    v.n = t->L.n;
    v.words = t->L.words;
    v.rank_entries = t->L.rank_entries;
    v.rank_stride = t->L.rank_stride;
    v.sigma = t->L.sigma;
    v.levels = t->L.levels;
    v.zeros = t->L.matrix ? reinterpret_cast<const unsigned long long *>(t->tree + kZerosOff) : nullptr;
    const bool four = t->L.arity == 4;
    v.digits = four ? reinterpret_cast<const uint64_t *>(t->tree + t->L.tree_digits_off) : nullptr;
    v.dir = four ? reinterpret_cast<const uint64_t *>(t->tree + t->L.tree_dir_off) : nullptr;
    v.dwords = t->L.dwords;
    v.levels4 = t->L.levels4;
    if (four) v.bits = v.ranks = nullptr;
    v.huff = nullptr;
    v.hbase = nullptr;
    if (t->hm) {
        v.bits = v.ranks = nullptr;
        v.huff = reinterpret_cast<const HuffMeta *>(t->tree + kHeaderBytes);
        v.hbase = t->tree;
        v.levels = t->hm->levels;
    }
    return v;
}

static wt_tree *new_handle(const Layout &L, void *tree, hipStream_t st) {
    wt_tree *h = new (std::nothrow) wt_tree;
    if (!h) return nullptr;
    h->L = L;
    h->tree = reinterpret_cast<uint8_t *>(tree);
    h->stream = st;
    h->device = 0;
    (void)hipGetDevice(&h->device);
    h->d_query = nullptr;
    h->hm = nullptr;
    h->htab = nullptr;
    return h;
}

// Batched-build workspace: job descriptors, block maps, then one workspace
// slice per sequence.  Sequences are grouped by (width, lane bytes).
constexpr int kClasses = 9;
static int batch_class(uint32_t w, uint32_t lb) { return wclass(w) * 3 + (lb == 32 ? 0 : (lb == 64 ? 1 : 2)); }
static const uint32_t kClassWidth[kClasses] = {1, 1, 1, 2, 2, 2, 4, 4, 4};
static const uint32_t kClassLane[kClasses] = {32, 64, 128, 32, 64, 128, 32, 64, 128};

// Long sequences of a batch are built on their own, each as a single build
// on the batch's stream, where that is faster: the single build brings
// narrowed orders (2- and 4-byte symbols), the folded last level (1-byte
// symbols) and per-level tuning, but pays its own chain of launches, which
// batched sequences share.  So a sequence goes alone
// - with 4-byte symbols, from 2^25 symbols on (narrowing saves more than
//   the chain costs), and
// - from 2^25 symbols of 1 byte or 2^23 of 2 or 4 bytes, when no other
//   sequence of the batch would share its batched launches (none left in its
//   class of width and lane geometry), so that it pays a chain either way.
static const uint32_t kSoloMinLg[3] = {25, 23, 23};
constexpr uint32_t kSoloSharedMinLg = 25;

struct BatchPlan {
    std::vector<Layout> L;
    // per class (width, lane bytes): sequences by levels, descending
    std::vector<uint32_t> order[kClasses];
    std::vector<uint32_t> small[6];  // per (width class, 64 KB / 160 KB): one-workgroup builds
    std::vector<uint32_t> solo;      // long sequences, built as single builds
    uint64_t jobs_off, small_off, map_off[kClasses], sup_off[kClasses], slices_off, total;
    std::vector<uint64_t> slice;     // workspace offset of each sequence's slice
    uint64_t blocks[kClasses], sups[kClasses];
};

static int plan_batch(uint32_t m, const wt_desc *descs, BatchPlan *P) {
    P->L.resize(m);
    // per sequence: its batched class, or one of these
    constexpr int kOneWorkgroup = -1, kAlwaysAlone = -2;
    std::vector<int> cls(m, kOneWorkgroup);
    uint32_t members[kClasses] = {};
    for (uint32_t q = 0; q < m; q++) {
        int rc = check_desc(&descs[q]);
        if (rc != WT_OK) return rc;
        make_layout(descs[q].n, descs[q].sigma, descs[q].width, true, &P->L[q]);
        if (P->L[q].small) {
            P->small[wclass(descs[q].width) * 2 + (P->L[q].small == kGeomMid)].push_back(q);
            continue;
        }
        cls[q] = batch_class(descs[q].width, P->L[q].lane_bytes);
        if (descs[q].width == 4 && descs[q].n >= (1ull << kSoloSharedMinLg)) cls[q] = kAlwaysAlone;
        else members[cls[q]]++;
    }
    for (uint32_t q = 0; q < m; q++) {
        if (cls[q] == kOneWorkgroup) continue;
        const bool solo = cls[q] == kAlwaysAlone ||
                          (members[cls[q]] == 1 && descs[q].n >= (1ull << kSoloMinLg[wclass(descs[q].width)]));
        if (solo) {
            make_layout(descs[q].n, descs[q].sigma, descs[q].width, false, &P->L[q]);
            P->solo.push_back(q);
        } else {
            P->order[cls[q]].push_back(q);
        }
    }
    uint64_t nsmall = 0;
    for (int c = 0; c < 6; c++) nsmall += P->small[c].size();
    P->jobs_off = 0;
    uint64_t off = round_up((uint64_t)(m - nsmall - P->solo.size()) * sizeof(BatchJob), 256);
    P->small_off = off;
    off += round_up(nsmall * sizeof(SmallJob), 256);
    for (int c = 0; c < kClasses; c++) {
        std::vector<uint32_t> &o = P->order[c];
        std::stable_sort(o.begin(), o.end(), [&](uint32_t x, uint32_t y) { return P->L[x].levels > P->L[y].levels; });
        uint64_t nb = 0, ns = 0;
        for (uint32_t q : o) {
            nb += ceil_div(P->L[q].ntiles, kWaves);
            ns += P->L[q].nsup;
        }
        P->blocks[c] = nb;
        P->sups[c] = ns;
        P->map_off[c] = off;
        off += round_up((nb ? nb : 1) * 4, 256);
        P->sup_off[c] = off;
        off += round_up((ns ? ns : 1) * 4, 256);
    }
    P->slices_off = off;
    P->slice.resize(m);
    for (uint32_t q = 0; q < m; q++) {
        P->slice[q] = off;
        if (!P->L[q].small) off += round_up(P->L[q].work_bytes, 256);
    }
    P->total = off;
    return WT_OK;
}

static BatchJob make_job(const Layout &L, const void *S, void *tree, uint8_t *work) {
    BatchJob j;
    memset(&j, 0, sizeof(j));
    j.S = S;
    j.tree = reinterpret_cast<uint8_t *>(tree);
    j.work = work;
    j.n = L.n;
    j.words = L.words;
    j.rank_entries = L.rank_entries;
    j.rank_stride = L.rank_stride;
    j.ntiles = L.ntiles;
    j.nsup = L.nsup;
    j.tree_bits_off = L.tree_bits_off;
    j.tree_ranks_off = L.tree_ranks_off;
    j.ws_ta = L.ws_ta;
    j.ws_tb = L.ws_tb;
    j.ws_ctrl = L.ws_ctrl;
    j.ws_ctrl_bytes = L.ws_ctrl_bytes;
    j.ws_tile_ones = L.ws_tile_ones;
    j.ws_ones = L.ws_ones;
    j.ws_sup = L.ws_sup;
    j.ws_supsum = L.ws_supsum;
    j.ws_zo = L.ws_zo;
    j.ws_start = L.ws_start;
    j.ws_partials = L.ws_partials;
    j.sigma = L.sigma;
    j.width = L.width;
    j.levels = L.levels;
    j.check = (L.width < 4 && (uint64_t)L.sigma == (1ull << (8 * L.width))) ? 0u : 1u;
    j.lane_bytes = L.lane_bytes;
    return j;
}

// ---------------------------------------------------------- buffered build --
// S is read in buffers of b symbols; each becomes a partial tree in the
// workspace, built with a tiled geometry so that its last-level node tables
// (the leaf offsets of the buffer) are left in the partial workspace.
// Staging slots of the buffered build: the copy of buffer q + kStages waits
// until the partial build of buffer q has consumed slot q % kStages, so the
// copies can run that many buffers ahead of the builds.
constexpr int kStages = 4;

struct BufPlan {
    Layout L;          // the final tree
    Layout Lb, Llast;  // a full partial tree and the last (ragged) one
    uint64_t b, nbuf;
    uint64_t stage_bytes, off_stage[kStages], off_pwork, off_ptrees, pstride, off_C, off_csum, off_span, row, wg_per_level;
    uint64_t work_bytes;
};

constexpr uint64_t kMaxBuffers = 1ull << 20;

static int plan_buffered(const wt_desc *d, uint64_t b, BufPlan *P) {
    if (b == 0) return WT_EINVAL;
    memset(P, 0, sizeof(*P));
    make_layout(d->n, d->sigma, d->width, false, &P->L);
    P->b = b < d->n ? b : (d->n ? d->n : 1);
    P->nbuf = d->n ? ceil_div(d->n, P->b) : 1;
    if (P->nbuf > kMaxBuffers) return WT_EINVAL;
    P->stage_bytes = round_up(P->b * d->width, 256);
    P->off_stage[0] = 0;
    if (P->nbuf == 1) {  // one buffer: the ordinary build of the staged copy
        P->off_pwork = P->stage_bytes;
        P->work_bytes = P->off_pwork + P->L.work_bytes;
        return WT_OK;
    }
    uint32_t g = tuned_geometry(P->b, d->sigma, d->width, false);
    if (g == kGeomSmall || g == kGeomMid) g = 32;  // partial trees need node tables
    make_layout_geom(P->b, d->sigma, d->width, g, &P->Lb);
    make_layout_geom(d->n - (P->nbuf - 1) * P->b, d->sigma, d->width, g, &P->Llast);
    const uint32_t l = P->L.levels;
    uint64_t off = 0;
    for (int s = 0; s < kStages; s++) {
        P->off_stage[s] = off;
        off += P->stage_bytes;
    }
    P->off_pwork = off;
    off += P->Lb.work_bytes;
    P->pstride = round_up(P->Lb.tree_bytes, 256);
    P->off_ptrees = off;
    off += P->nbuf * P->pstride;
    P->row = (1ull << l) + 1;
    P->off_C = off;
    off += round_up((P->nbuf + 1) * P->row * 8, 256);
    P->wg_per_level = ceil_div(P->L.words, 1024);  // merge workgroups per level: 1024 words each
    P->off_csum = off;
    off += round_up((uint64_t)(l ? l : 1) * P->wg_per_level * 8, 256);
    P->off_span = off;
    off += round_up((uint64_t)(l ? l : 1) * (P->wg_per_level + 1) * 8, 256);
    P->work_bytes = off;
    return WT_OK;
}

// One non-blocking copy stream per device (default priority) for the
// host-to-device copies of the buffers; it lives until the process ends.
static hipStream_t copy_stream() {
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
        streams[dev] = nullptr;
    return streams[dev];
}

// Copies buffer q of S into staging slot q % kStages (on the copy stream)
// and builds its partial tree on `st`; the copy of buffer q + kStages waits
// until the build of buffer q has consumed the slot.
static hipError_t enqueue_buffered(const uint8_t *S, const BufPlan &P, uint8_t *tree, uint8_t *work, hipStream_t st) {
    const uint64_t w = P.L.width;
    if (P.nbuf == 1) {
        uint8_t *stage = work + P.off_stage[0];
        if (P.L.n == 0) return enqueue_build(stage, P.L, tree, work + P.off_pwork, st);
        hipEvent_t done = nullptr;
        hipError_t err = hipEventCreateWithFlags(&done, hipEventDisableTiming);
        if (err != hipSuccess) return err;
        err = hipMemcpyAsync(stage, S, P.L.n * w, hipMemcpyDefault, st);
        if (err == hipSuccess) err = hipEventRecord(done, st);
        if (err == hipSuccess) err = enqueue_build(stage, P.L, tree, work + P.off_pwork, st);
        if (err == hipSuccess) err = hipEventSynchronize(done);  // S has been read once the call returns
        (void)hipEventDestroy(done);
        return err;
    }
    hipStream_t cs = copy_stream();
    if (!cs) return hipErrorInvalidValue;
    constexpr int kEv = 1 + 2 * kStages;  // start, copied[kStages], used[kStages]
    hipEvent_t ev[kEv] = {};
    hipError_t err = hipSuccess;
    for (int e = 0; e < kEv && err == hipSuccess; e++) err = hipEventCreateWithFlags(&ev[e], hipEventDisableTiming);
    const uint32_t l = P.L.levels;
    unsigned long long *C = reinterpret_cast<unsigned long long *>(work + P.off_C);
    uint8_t *pwork = work + P.off_pwork;
    if (err == hipSuccess) err = hipEventRecord(ev[0], st);  // the workspace is free once st gets here
    if (err == hipSuccess) err = hipStreamWaitEvent(cs, ev[0], 0);
    uint64_t copied = 0;  // buffers whose copy was enqueued
    for (uint64_t q = 0; q < P.nbuf && err == hipSuccess; q++) {
        const int s = (int)(q % kStages);
        const Layout &Lq = (q + 1 == P.nbuf) ? P.Llast : P.Lb;
        uint8_t *stage = work + P.off_stage[s];
        uint8_t *ptree = work + P.off_ptrees + q * P.pstride;
        if (q >= kStages) err = hipStreamWaitEvent(cs, ev[1 + kStages + s], 0);
        if (err == hipSuccess) err = hipMemcpyAsync(stage, S + q * P.b * w, Lq.n * w, hipMemcpyDefault, cs);
        if (err == hipSuccess) copied = q + 1;
        if (err == hipSuccess) err = hipEventRecord(ev[1 + s], cs);
        if (err == hipSuccess) err = hipStreamWaitEvent(st, ev[1 + s], 0);
        if (err == hipSuccess) err = enqueue_build(stage, Lq, ptree, pwork, st, true);
        if (err == hipSuccess && l)
            err = launch_leaf_prefix(reinterpret_cast<const uint64_t *>(pwork + Lq.ws_start) + start_offset(l - 1),
                                     reinterpret_cast<const ulonglong2 *>(pwork + Lq.ws_zo) + zo_offset(l - 1), l, Lq.n,
                                     C + q * P.row, st);
        if (err == hipSuccess && q + kStages < P.nbuf) err = hipEventRecord(ev[1 + kStages + s], st);
    }
    if (err == hipSuccess) {
        MergeArgs a;
        a.C = C;
        a.ptrees = work + P.off_ptrees;
        a.pstride = P.pstride;
        a.pbits_off = P.Lb.tree_bits_off;
        a.pwords = P.Lb.words;
        a.pwords_last = P.Llast.words;
        a.bits = reinterpret_cast<uint64_t *>(tree + P.L.tree_bits_off);
        a.ranks = reinterpret_cast<uint64_t *>(tree + P.L.tree_ranks_off);
        a.tree_status = reinterpret_cast<uint32_t *>(tree);
        a.csum = reinterpret_cast<unsigned long long *>(work + P.off_csum);
        a.span_run = reinterpret_cast<uint64_t *>(work + P.off_span);
        a.n = P.L.n;
        a.words = P.L.words;
        a.rank_stride = P.L.rank_stride;
        a.nblk = ceil_div(P.L.n, 512);
        a.wg_per_level = P.wg_per_level;
        a.row = P.row;
        a.levels = l;
        a.nbuf = (uint32_t)P.nbuf;
        const uint64_t mbytes = (uint64_t)l * (P.L.words * 8 * 2 + P.L.rank_stride * 8);
        long pr = prof_begin(st, "merge", 0, P.L.width, P.L.n, mbytes);
        err = launch_merge(a, st);
        prof_end(pr, st);
    }
    // S has been read once every enqueued copy is done; every event recorded
    // above is complete by then, so they can be released.
    if (copied) {
        hipError_t e2 = hipEventSynchronize(ev[1 + (int)((copied - 1) % kStages)]);
        if (err == hipSuccess) err = e2;
    } else {
        (void)hipStreamSynchronize(cs);
    }
    for (int e = 0; e < kEv; e++)
        if (ev[e]) (void)hipEventDestroy(ev[e]);
    return err;
}

// ------------------------------------------------ Huffman-shaped tree ---
// The code: Huffman's merging of the two lightest items with two FIFO queues
// (the symbols that occur, by count then symbol; the merged items in the
// order they are made), the lighter front first and the symbol queue on
// equal weights; a symbol's length is the depth of its leaf.  Canonical
// codes follow from the lengths.  One symbol alone (or n = 0) gives a tree
// with no levels.
struct HuffPlan {
    HuffMeta m;
    std::vector<uint32_t> code_tab;  // per symbol: length | kHuffPresent | code << 8
    std::vector<uint32_t> syms;      // symbols by (length, symbol)
    uint32_t inner_width;            // bytes per left-aligned code
    Layout inner;                    // level split over the codes (2^L symbols)
    uint64_t tree_bytes, ws_k, ws_work, work_bytes;
};

static int huff_lengths(const uint64_t *counts, uint32_t sigma, std::vector<uint8_t> &len, uint32_t &maxlen) {
    len.assign(sigma, 0);
    maxlen = 0;
    // the symbols that occur, by (count, symbol): a counting sort by count
    // (stable, symbols taken in increasing order) when the counts are small
    // next to the number of symbols, else a sort of the distinct packed keys
    // count << 24 | symbol (count < 2^40, symbol < 2^24)
    uint64_t k = 0, maxc = 0;
    for (uint32_t c = 0; c < sigma; c++)
        if (counts[c]) {
            k++;
            maxc = std::max<uint64_t>(maxc, counts[c]);
        }
    if (k < 2) return WT_OK;
    // items: leaves 0..k-1 (in queue order), merged items k..2k-2, with
    // weights w; up[i] is item i's parent (k < 2^24, so 32 bits hold it).
    // The leaves' weights are the sorted counts, written in order.
    std::vector<uint32_t> leaf(k);
    std::vector<uint64_t> w(2 * k - 1);
    std::vector<uint32_t> up(2 * k - 1);
    if (maxc <= 4 * k + 1024) {
        std::vector<uint32_t> pos(maxc + 2, 0);
        for (uint32_t c = 0; c < sigma; c++)
            if (counts[c]) pos[counts[c] + 1]++;
        for (uint64_t x = 1; x < pos.size(); x++) pos[x] += pos[x - 1];
        for (uint32_t c = 0; c < sigma; c++)
            if (counts[c]) leaf[pos[counts[c]]++] = c;
        // (pos[x] now ends count x's leaves)
        size_t i = 0;
        for (uint64_t x = 1; x <= maxc; x++)
            for (; i < pos[x]; i++) w[i] = x;
    } else {
        std::vector<uint64_t> key;
        key.reserve(k);
        for (uint32_t c = 0; c < sigma; c++)
            if (counts[c]) key.push_back((counts[c] << 24) | c);
        std::sort(key.begin(), key.end());
        for (size_t i = 0; i < k; i++) {
            leaf[i] = (uint32_t)(key[i] & 0xFFFFFFu);
            w[i] = key[i] >> 24;
        }
    }
    size_t lf = 0, mf = k, made = k;
    for (; made < 2 * k - 1; made++) {
        size_t pick[2];
        for (int t = 0; t < 2; t++) {
            const bool from_leaf = lf < k && (mf >= made || w[lf] <= w[mf]);
            pick[t] = from_leaf ? lf++ : mf++;
        }
        w[made] = w[pick[0]] + w[pick[1]];
        up[pick[0]] = up[pick[1]] = (uint32_t)made;
    }
    // depths in place: parents come later, so walking down from the root
    // each item reads its parent's depth where the parent's link was
    up[2 * k - 2] = 0;
    for (size_t i = 2 * k - 2; i-- > 0;) up[i] = up[up[i]] + 1;
    for (size_t i = 0; i < k; i++) {
        len[leaf[i]] = (uint8_t)std::min<uint32_t>(up[i], 255u);
        maxlen = std::max(maxlen, up[i]);
    }
    return WT_OK;
}

static int plan_huffman(const uint64_t *counts, const wt_desc *desc, HuffPlan *P) {
    int rc = check_desc(desc);
    if (rc != WT_OK) return rc;
    if (!counts) return WT_EINVAL;
    const uint32_t sigma = desc->sigma;
    const uint64_t n = desc->n;
    uint64_t total = 0;
    uint32_t distinct = 0, only = 0;
    for (uint32_t c = 0; c < sigma; c++) {
        total += counts[c];
        if (counts[c]) { distinct++; only = c; }
    }
    if (total != n) return WT_EINVAL;  // not the histogram of S
    std::vector<uint8_t> len;
    uint32_t L;
    huff_lengths(counts, sigma, len, L);
    if (L > kHuffMaxLevels) return WT_EINVAL;
    HuffMeta &m = P->m;
    memset(&m, 0, sizeof(m));
    m.n = n;
    m.sigma = sigma;
    m.levels = L;
    m.distinct = distinct;
    m.only = (L == 0 && n > 0) ? only : 0xFFFFFFFFu;
    // canonical codes: by (length, symbol); counts and first codes per length
    P->code_tab.assign(sigma, 0);
    P->syms.clear();
    for (uint32_t c = 0; c < sigma; c++)
        if (counts[c]) P->code_tab[c] = kHuffPresent;  // (length 0 when the tree has no levels)
    // codes per length, then each length's symbols in symbol order (one
    // counting pass), and the occurrences per length for the depth sizes
    uint64_t occ[kHuffMaxLevels + 1] = {0};
    for (uint32_t c = 0; c < sigma; c++)
        if (len[c]) {
            m.count[len[c]]++;
            occ[len[c]] += counts[c];
        }
    uint64_t next = 0;  // first code of the current length
    uint32_t at = 0;
    for (uint32_t l = 1; l <= L; l++) {
        m.first[l] = (uint32_t)next;
        m.start[l] = at;
        at += m.count[l];
        next = (next + m.count[l]) << 1;
    }
    P->syms.assign(at, 0);
    uint32_t fill[kHuffMaxLevels + 1];
    for (uint32_t l = 1; l <= L; l++) fill[l] = 0;
    for (uint32_t c = 0; c < sigma; c++) {
        const uint32_t l = len[c];
        if (!l) continue;
        P->code_tab[c] = l | kHuffPresent | ((m.first[l] + fill[l]) << 8);
        P->syms[m.start[l] + fill[l]] = c;
        fill[l]++;
    }
    // depth sizes: symbols whose code is longer than d
    uint64_t longer = 0;
    for (uint32_t d = L; d-- > 0;) {
        longer += occ[d + 1];
        m.size[d] = longer;
    }
    // tree layout
    uint64_t off = kHeaderBytes + kHuffMetaBytes;
    m.code_off = off;
    off += round_up((uint64_t)sigma * 4, 256);
    m.syms_off = off;
    off += round_up((uint64_t)(P->syms.size() ? P->syms.size() : 1) * 4, 256);
    uint64_t max_words = 0, max_wg = 1;
    for (uint32_t d = 0; d < L; d++) {
        m.bits_off[d] = off;
        const uint64_t words = round_up(ceil_div(m.size[d], 64), 8);
        max_words = std::max(max_words, words);
        off += words * 8;
    }
    for (uint32_t d = 0; d < L; d++) {
        m.dir_off[d] = off;
        m.dir_entries[d] = ceil_div(m.size[d], 512) + 1;
        max_wg = std::max(max_wg, ceil_div(m.dir_entries[d] - 1, kBitDirBlocks));
        off += round_up(m.dir_entries[d], 8) * 8;
    }
    P->tree_bytes = off;
    // workspace: the codes (T_0 of the level split) and the split's own
    // workspace, tiled (the one-workgroup build lists every level in full)
    P->inner_width = L <= 8 ? 1u : (L <= 16 ? 2u : 4u);
    memset(&P->inner, 0, sizeof(P->inner));
    uint64_t w = 0;
    P->ws_k = w;
    if (L > 0) {
        uint32_t g = tuned_geometry(n, 1u << L, P->inner_width, false);
        if (g == kGeomSmall || g == kGeomMid) g = 32;
        make_layout_geom(n, 1u << L, P->inner_width, g, &P->inner);
        w += round_up(n * P->inner_width, 256);
        P->ws_work = w;
        w += round_up(P->inner.work_bytes, 256);
    }
    P->work_bytes = w ? w : 256;
    (void)max_words;
    (void)max_wg;
    return WT_OK;
}

static hipError_t enqueue_huffman(const void *S, const wt_desc *desc, const HuffPlan &P, const uint8_t *htab,
                                  uint64_t htab_bytes, uint8_t *tree, uint8_t *work, hipStream_t st) {
    const HuffMeta &m = P.m;
    const uint32_t L = m.levels;
    const Layout &I = P.inner;
    uint32_t *status = reinterpret_cast<uint32_t *>(tree);
    // status word (and, with levels, the split's counters) cleared, tables in
    long pr = prof_begin(st, "zero", 0, desc->width, m.n, L ? I.ws_ctrl_bytes : 0);
    hipError_t err = L ? launch_zero(work + P.ws_work + I.ws_ctrl, I.ws_ctrl_bytes, status, nullptr, 0, st)
                       : launch_zero(tree, 0, status, nullptr, 0, st);
    prof_end(pr, st);
    if (err == hipSuccess)
        err = hipMemcpyAsync(tree + kHeaderBytes, htab, htab_bytes, hipMemcpyHostToDevice, st);
    if (err != hipSuccess) return err;
    const uint32_t *code_tab = reinterpret_cast<const uint32_t *>(tree + m.code_off);
    uint8_t *K = L ? work + P.ws_k : nullptr;
    pr = prof_begin(st, "huff_map", 0, desc->width, m.n, m.n * (desc->width + (L ? P.inner_width : 0)));
    err = launch_huff_map(S, m.n, desc->width, code_tab, m.sigma, L, K, P.inner_width, status, st);
    prof_end(pr, st);
    if (err != hipSuccess || L == 0) return err;
    // The level split over the left-aligned codes, compacted: level d lists
    // only the n_d symbols still inside the tree (its positions are depth d's
    // bitmap positions).  The node tables of level d + 1 are shifted down by
    // the number of symbols whose code ends at depth d + 1 (they come first
    // in that level's order), so that the split drops them and places the
    // others directly in the next depth's order.
    const uint64_t TILE = tile_syms(I.width, I.lane_bytes);
    uint32_t *tile_ones = reinterpret_cast<uint32_t *>(work + P.ws_work + I.ws_tile_ones);
    unsigned long long *supsum = reinterpret_cast<unsigned long long *>(work + P.ws_work + I.ws_supsum);
    unsigned long long *ones = reinterpret_cast<unsigned long long *>(work + P.ws_work + I.ws_ones);
    unsigned long long *sup = reinterpret_cast<unsigned long long *>(work + P.ws_work + I.ws_sup);
    ulonglong2 *zo = reinterpret_cast<ulonglong2 *>(work + P.ws_work + I.ws_zo);
    uint64_t *start = reinterpret_cast<uint64_t *>(work + P.ws_work + I.ws_start);
    uint64_t *partials = reinterpret_cast<uint64_t *>(work + P.ws_work + I.ws_partials);
    uint8_t *tbuf[2] = {work + P.ws_work + I.ws_ta, work + P.ws_work + I.ws_tb};
    IngestArgs ia;
    ia.S = K;
    ia.tile_ones0 = tile_ones;
    ia.ones0 = ones;
    ia.start0 = start;
    ia.tree_status = status;
    ia.n = m.n;
    ia.ntiles = I.ntiles;
    ia.slots0 = level_slots(0);
    ia.sigma = 1u << L;
    ia.check = 0;
    ia.msb = L - 1;
    ia.zero_g = nullptr;
    ia.zero_granules = 0;
    {
        uint64_t k = kWaves;
        while (I.ntiles > 8192 * k) k <<= 1;
        ia.tiles_per_block = k;
    }
    pr = prof_begin(st, "ingest", 0, I.width, m.n, m.n * I.width);
    err = launch_ingest(ia, I.width, I.lane_bytes, st);
    prof_end(pr, st);
    if (err != hipSuccess) return err;
    const uint64_t stride = tile_stride(I.ntiles);
    for (uint32_t d = 0; d < L; d++) {
        const uint64_t nd = m.size[d];
        const uint64_t nnext = (d + 1 < L) ? m.size[d + 1] : 0;
        const uint64_t ntiles = ceil_div(nd, TILE), nsup = ceil_div(ntiles, kSup);
        PlanArgs pa;
        pa.start = start + start_offset(d);
        pa.ones = ones + ones_offset(d);
        pa.zo = zo + zo_offset(d);
        pa.start_next = (d + 1 < L) ? start + start_offset(d + 1) : nullptr;
        pa.partials = partials;
        pa.nodes = 1ull << d;
        pa.slots = level_slots(d);
        pa.n = nd;
        pa.matrix = 0;
        pa.shift = (d + 1 < L) ? nd - nnext : 0;  // the symbols whose code ends at depth d + 1
        const bool big = pa.nodes > kScanChunk;
        if (big) {
            err = launch_plan(pa, st);
            if (err != hipSuccess) return err;
        }
        PrepArgs pp;
        pp.tile_ones = tile_ones + (uint64_t)d * stride;
        pp.supsum = supsum;
        pp.sup = sup + (uint64_t)d * I.nsup;
        pp.ntiles = ntiles;
        pp.nsup = nsup;
        pp.plan = pa;
        pp.plan_here = big ? 0u : 1u;
        pp.sums_here = (nsup <= kPrepSups && !big && pa.nodes < kThreads) ? 1u : 0u;
        pr = prof_begin(st, "prep", d, I.width, nd, ntiles * 4 + nsup * 16);
        err = launch_prep(pp, st);
        prof_end(pr, st);
        if (err != hipSuccess) return err;
        LevelArgs a;
        memset(&a, 0, sizeof(a));
        a.tin = (d == 0) ? (const void *)K : tbuf[(d - 1) & 1];
        a.tout = (d + 1 < L) ? tbuf[d & 1] : nullptr;
        a.bits = reinterpret_cast<uint64_t *>(tree + m.bits_off[d]);
        a.ranks = reinterpret_cast<uint64_t *>(tree + m.dir_off[d]);
        a.zo = zo + zo_offset(d);
        a.tile_ones = tile_ones + (uint64_t)d * stride;
        a.sup = sup + (uint64_t)d * I.nsup;
        a.tile_ones_next = (d + 1 < L) ? tile_ones + (uint64_t)(d + 1) * stride : nullptr;
        a.ones_next = (d + 1 < L) ? ones + ones_offset(d + 1) : nullptr;
        a.nodes_next = 2ull << d;
        a.slots_next = level_slots(d + 1);
        a.n = nd;
        a.n_out = nnext;
        a.words = round_up(ceil_div(nd, 64), 8);
        a.rank_entries = m.dir_entries[d];
        a.rank_stride = round_up(m.dir_entries[d], 8);
        a.ntiles = ntiles;
        a.levels = L;
        a.level = d;
        a.symmask = (uint32_t)((1ull << L) - 1);
        const uint64_t lbytes = nd * I.width + nnext * I.width + a.words * 8 + a.rank_stride * 8;
        pr = prof_begin(st, "level", d, I.width, nd, lbytes);
        // (the plain variant: every destination comes from the node tables)
        err = launch_level(a, I.width, I.lane_bytes, false, I.width, I.lane_bytes, st);
        prof_end(pr, st);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

// ------------------------------------------------ no-allocation build ---
// Workspace of wt_build_noalloc: a file-scope device array, one copy on
// every device the library runs on, held until the process ends.  In host
// code its name is not a device address: the address of the current
// device's copy comes from hipGetSymbolAddress, taken once per device on the
// first call there, and only that pointer reaches the kernels.
static __device__ __align__(256) uint8_t scratch[WT_NOALLOC_WORK_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static uint8_t *g_scratch[kMaxDevices];

static int scratch_on_current_device(uint8_t **p) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return WT_EDEVICE;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) return WT_EDEVICE;
        g_scratch[dev] = reinterpret_cast<uint8_t *>(ptr);
    }
    *p = g_scratch[dev];
    return WT_OK;
}

}  // namespace wt

using namespace wt;

extern "C" {

int wt_histogram(const void *d_S, const wt_desc *desc, uint64_t *d_counts, void *stream) {
    int rc = check_desc(desc);
    if (rc != WT_OK) return rc;
    if (!d_counts || (desc->n > 0 && !d_S) || ((uintptr_t)d_counts & 7)) return WT_EINVAL;
    return launch_histogram(d_S, desc->n, desc->width, desc->sigma, reinterpret_cast<unsigned long long *>(d_counts),
                            reinterpret_cast<hipStream_t>(stream)) == hipSuccess
               ? WT_OK
               : WT_EDEVICE;
}

int wt_huffman_footprint(const uint64_t *counts, const wt_desc *desc, uint64_t *tree_bytes, uint64_t *work_bytes) {
    HuffPlan P;
    int rc = plan_huffman(counts, desc, &P);
    if (rc != WT_OK) return rc;
    if (tree_bytes) *tree_bytes = P.tree_bytes;
    if (work_bytes) *work_bytes = P.work_bytes;
    return WT_OK;
}

int wt_build_huffman(const void *d_S, const wt_desc *desc, const uint64_t *counts, void *d_tree, uint64_t tree_bytes,
                     void *d_work, uint64_t work_bytes, void *stream, wt_tree **out) {
    if (out) *out = nullptr;
    if (!out) return WT_EINVAL;
    HuffPlan P;
    int rc = plan_huffman(counts, desc, &P);
    if (rc != WT_OK) return rc;
    if (!d_tree || !d_work || (desc->n > 0 && !d_S)) return WT_EINVAL;
    if (((uintptr_t)d_S & 15) || ((uintptr_t)d_tree & 255) || ((uintptr_t)d_work & 255)) return WT_EINVAL;
    if (tree_bytes < P.tree_bytes || work_bytes < P.work_bytes) return WT_ENOMEM;
    // the tables as they sit in the tree memory from kHeaderBytes on
    const uint64_t tab_bytes = P.m.syms_off + P.syms.size() * 4 - kHeaderBytes;
    uint8_t *htab = new (std::nothrow) uint8_t[tab_bytes];
    HuffMeta *hm = new (std::nothrow) HuffMeta(P.m);
    Layout hl;
    memset(&hl, 0, sizeof(hl));
    hl.n = desc->n;
    hl.sigma = desc->sigma;
    hl.width = desc->width;
    hl.levels = P.m.levels;
    hl.tree_bytes = P.tree_bytes;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    wt_tree *h = (htab && hm) ? new_handle(hl, d_tree, st) : nullptr;
    if (!h) {
        delete[] htab;
        delete hm;
        return WT_ENOMEM;
    }
    memset(htab, 0, tab_bytes);
    memcpy(htab, &P.m, sizeof(HuffMeta));
    memcpy(htab + (P.m.code_off - kHeaderBytes), P.code_tab.data(), P.code_tab.size() * 4);
    if (!P.syms.empty()) memcpy(htab + (P.m.syms_off - kHeaderBytes), P.syms.data(), P.syms.size() * 4);
    h->hm = hm;
    h->htab = htab;
    if (enqueue_huffman(d_S, desc, P, htab, tab_bytes, reinterpret_cast<uint8_t *>(d_tree),
                        reinterpret_cast<uint8_t *>(d_work), st) != hipSuccess) {
        wt_free(h);
        return WT_EDEVICE;
    }
    *out = h;
    return WT_OK;
}

int wt_huffman_levels(const wt_tree *t, uint32_t *levels, uint64_t *sizes, uint64_t *bits_off, uint64_t *dir_off,
                      uint64_t *dir_entries, uint32_t *code_table) {
    if (!t || !t->hm) return WT_EINVAL;
    const HuffMeta &m = *t->hm;
    if (levels) *levels = m.levels;
    for (uint32_t d = 0; d < m.levels; d++) {
        if (sizes) sizes[d] = m.size[d];
        if (bits_off) bits_off[d] = m.bits_off[d];
        if (dir_off) dir_off[d] = m.dir_off[d];
        if (dir_entries) dir_entries[d] = m.dir_entries[d];
    }
    if (code_table)
        memcpy(code_table, t->htab + (m.code_off - kHeaderBytes), (uint64_t)m.sigma * 4);
    return WT_OK;
}

int wt_build_noalloc(const void *d_S, const wt_desc *desc, void *d_tree, uint64_t tree_bytes, void *stream) {
    int rc = check_desc(desc);
    if (rc != WT_OK) return rc;
    if (!d_tree || (desc->n > 0 && !d_S)) return WT_EINVAL;
    if (((uintptr_t)d_S & 15) || ((uintptr_t)d_tree & 255)) return WT_EINVAL;
    Layout L;
    make_layout(desc->n, desc->sigma, desc->width, false, &L);
    if (tree_bytes < L.tree_bytes || L.work_bytes > WT_NOALLOC_WORK_BYTES) return WT_ENOMEM;
    uint8_t *work = nullptr;
    rc = scratch_on_current_device(&work);
    if (rc != WT_OK) return rc;
    return enqueue_build(d_S, L, reinterpret_cast<uint8_t *>(d_tree), work, reinterpret_cast<hipStream_t>(stream)) ==
                   hipSuccess
               ? WT_OK
               : WT_EDEVICE;
}

int wt_footprint(const wt_desc *desc, uint64_t *tree_bytes, uint64_t *work_bytes) {
    int rc = check_desc(desc);
    if (rc != WT_OK) return rc;
    Layout L;
    make_layout(desc->n, desc->sigma, desc->width, false, &L);
    if (tree_bytes) *tree_bytes = L.tree_bytes;
    if (work_bytes) *work_bytes = L.work_bytes;
    return WT_OK;
}

static int build_one(const void *d_S, const wt_desc *desc, void *d_tree, uint64_t tree_bytes, void *d_work,
                     uint64_t work_bytes, void *stream, wt_tree **out, uint32_t matrix) {
    if (out) *out = nullptr;
    int rc = check_desc(desc);
    if (rc != WT_OK) return rc;
    if (!out || !d_tree || !d_work || (desc->n > 0 && !d_S)) return WT_EINVAL;
    if (((uintptr_t)d_S & 15) || ((uintptr_t)d_tree & 255) || ((uintptr_t)d_work & 255)) return WT_EINVAL;
    Layout L;
    make_layout(desc->n, desc->sigma, desc->width, false, &L);
    L.matrix = matrix;
    if (matrix) narrow_widths(&L, true);  // (the footprint's workspace still holds it)
    if (tree_bytes < L.tree_bytes || work_bytes < L.work_bytes) return WT_ENOMEM;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    wt_tree *h = new_handle(L, d_tree, st);
    if (!h) return WT_ENOMEM;
    if (enqueue_build(d_S, L, reinterpret_cast<uint8_t *>(d_tree), reinterpret_cast<uint8_t *>(d_work), st) !=
        hipSuccess) {
        delete h;
        return WT_EDEVICE;
    }
    *out = h;
    return WT_OK;
}

int wt_build(const void *d_S, const wt_desc *desc, void *d_tree, uint64_t tree_bytes, void *d_work,
             uint64_t work_bytes, void *stream, wt_tree **out) {
    return build_one(d_S, desc, d_tree, tree_bytes, d_work, work_bytes, stream, out, 0u);
}

int wt_build_matrix(const void *d_S, const wt_desc *desc, void *d_tree, uint64_t tree_bytes, void *d_work,
                    uint64_t work_bytes, void *stream, wt_tree **out) {
    return build_one(d_S, desc, d_tree, tree_bytes, d_work, work_bytes, stream, out, 1u);
}

int wt_multiary_footprint(const wt_desc *desc, uint64_t *tree_bytes, uint64_t *work_bytes) {
    int rc = check_desc(desc);
    if (rc != WT_OK) return rc;
    Layout L;
    make_layout4(desc->n, desc->sigma, desc->width, &L);
    if (tree_bytes) *tree_bytes = L.tree_bytes;
    if (work_bytes) *work_bytes = L.work_bytes;
    return WT_OK;
}

int wt_build_multiary(const void *d_S, const wt_desc *desc, void *d_tree, uint64_t tree_bytes, void *d_work,
                      uint64_t work_bytes, void *stream, wt_tree **out) {
    if (out) *out = nullptr;
    int rc = check_desc(desc);
    if (rc != WT_OK) return rc;
    if (!out || !d_tree || !d_work || (desc->n > 0 && !d_S)) return WT_EINVAL;
    if (((uintptr_t)d_S & 15) || ((uintptr_t)d_tree & 255) || ((uintptr_t)d_work & 255)) return WT_EINVAL;
    Layout L;
    make_layout4(desc->n, desc->sigma, desc->width, &L);
    if (tree_bytes < L.tree_bytes || work_bytes < L.work_bytes) return WT_ENOMEM;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    wt_tree *h = new_handle(L, d_tree, st);
    if (!h) return WT_ENOMEM;
    if (enqueue_multiary(d_S, L, reinterpret_cast<uint8_t *>(d_tree), reinterpret_cast<uint8_t *>(d_work), st) !=
        hipSuccess) {
        delete h;
        return WT_EDEVICE;
    }
    *out = h;
    return WT_OK;
}

int wt_multiary_levels(const wt_tree *t, uint32_t *levels, const uint64_t **d_digits, uint64_t *words_per_level,
                       const uint64_t **d_dir, uint64_t *dir_stride) {
    if (!t || t->L.arity != 4) return WT_EINVAL;
    if (levels) *levels = t->L.levels4;
    if (d_digits) *d_digits = reinterpret_cast<const uint64_t *>(t->tree + t->L.tree_digits_off);
    if (words_per_level) *words_per_level = t->L.dwords;
    if (d_dir) *d_dir = reinterpret_cast<const uint64_t *>(t->tree + t->L.tree_dir_off);
    if (dir_stride) *dir_stride = t->L.rank_stride;
    return WT_OK;
}

int wt_matrix_zeros(const wt_tree *t, uint64_t *zeros) {
    if (!t || !zeros || !t->L.matrix) return WT_EINVAL;
    if (t->L.levels == 0) return WT_OK;
    if (hipStreamSynchronize(t->stream) != hipSuccess) return WT_EDEVICE;
    if (hipMemcpy(zeros, t->tree + kZerosOff, t->L.levels * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess)
        return WT_EDEVICE;
    return WT_OK;
}

int wt_buffered_footprint(const wt_desc *desc, uint64_t buffer_syms, uint64_t *tree_bytes, uint64_t *work_bytes) {
    int rc = check_desc(desc);
    if (rc != WT_OK) return rc;
    BufPlan P;
    if ((rc = plan_buffered(desc, buffer_syms, &P)) != WT_OK) return rc;
    if (tree_bytes) *tree_bytes = P.L.tree_bytes;
    if (work_bytes) *work_bytes = P.work_bytes;
    return WT_OK;
}

int wt_build_buffered(const void *S, const wt_desc *desc, uint64_t buffer_syms, void *d_tree, uint64_t tree_bytes,
                      void *d_work, uint64_t work_bytes, void *stream, wt_tree **out) {
    if (out) *out = nullptr;
    int rc = check_desc(desc);
    if (rc != WT_OK) return rc;
    if (!out || !d_tree || !d_work || (desc->n > 0 && !S)) return WT_EINVAL;
    if (((uintptr_t)d_tree & 255) || ((uintptr_t)d_work & 255)) return WT_EINVAL;
    BufPlan P;
    if ((rc = plan_buffered(desc, buffer_syms, &P)) != WT_OK) return rc;
    if (tree_bytes < P.L.tree_bytes || work_bytes < P.work_bytes) return WT_ENOMEM;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    wt_tree *h = new_handle(P.L, d_tree, st);
    if (!h) return WT_ENOMEM;
    if (enqueue_buffered(reinterpret_cast<const uint8_t *>(S), P, reinterpret_cast<uint8_t *>(d_tree),
                         reinterpret_cast<uint8_t *>(d_work), st) != hipSuccess) {
        delete h;
        return WT_EDEVICE;
    }
    *out = h;
    return WT_OK;
}

int wt_batch_footprint(uint32_t m, const wt_desc *descs, uint64_t *work_bytes) {
    if (m > 0 && !descs) return WT_EINVAL;
    BatchPlan P;
    int rc = plan_batch(m, descs, &P);
    if (rc != WT_OK) return rc;
    if (work_bytes) *work_bytes = P.total;
    return WT_OK;
}

int wt_build_batch(uint32_t m, const void *const *d_S, const wt_desc *descs, void *const *d_trees,
                   const uint64_t *tree_bytes, void *d_work, uint64_t work_bytes, void *stream, wt_tree **out) {
    if (!out || (m > 0 && (!d_S || !descs || !d_trees || !tree_bytes || !d_work))) return WT_EINVAL;
    for (uint32_t q = 0; q < m; q++) out[q] = nullptr;
    if (m == 0) return WT_OK;
    BatchPlan P;
    int rc = plan_batch(m, descs, &P);
    if (rc != WT_OK) return rc;
    if (work_bytes < P.total) return WT_ENOMEM;
    if ((uintptr_t)d_work & 255) return WT_EINVAL;
    for (uint32_t q = 0; q < m; q++) {
        if (!d_trees[q] || (descs[q].n > 0 && !d_S[q])) return WT_EINVAL;
        if (((uintptr_t)d_S[q] & 15) || ((uintptr_t)d_trees[q] & 255)) return WT_EINVAL;
        if (tree_bytes[q] < P.L[q].tree_bytes) return WT_ENOMEM;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    uint8_t *work = reinterpret_cast<uint8_t *>(d_work);

    // job descriptors, class by class (levels descending inside a class)
    std::vector<BatchJob> jobs;
    jobs.reserve(m);
    uint32_t first[kClasses];
    uint32_t maxl = 0;
    for (int c = 0; c < kClasses; c++) {
        first[c] = (uint32_t)jobs.size();
        uint64_t blk = 0, sup = 0;
        for (uint32_t q : P.order[c]) {
            BatchJob j = make_job(P.L[q], d_S[q], d_trees[q], work + P.slice[q]);
            j.blk_base = blk;
            j.sup_base = sup;
            blk += ceil_div(P.L[q].ntiles, kWaves);
            sup += P.L[q].nsup;
            jobs.push_back(j);
            maxl = std::max(maxl, P.L[q].levels);
        }
    }
    BatchJob *d_jobs = reinterpret_cast<BatchJob *>(work + P.jobs_off);
    // (pageable source: the call returns once the descriptors are staged)
    if (!jobs.empty() &&
        hipMemcpyAsync(d_jobs, jobs.data(), jobs.size() * sizeof(BatchJob), hipMemcpyHostToDevice, st) != hipSuccess)
        return WT_EDEVICE;
    // short sequences: one workgroup each, one launch per width
    std::vector<SmallJob> sjobs;
    uint32_t sfirst[7];
    for (int c = 0; c < 6; c++) {
        sfirst[c] = (uint32_t)sjobs.size();
        for (uint32_t q : P.small[c]) sjobs.push_back(make_small_job(P.L[q], d_S[q], d_trees[q]));
    }
    sfirst[6] = (uint32_t)sjobs.size();
    SmallJob *d_sjobs = reinterpret_cast<SmallJob *>(work + P.small_off);
    if (!sjobs.empty() &&
        hipMemcpyAsync(d_sjobs, sjobs.data(), sjobs.size() * sizeof(SmallJob), hipMemcpyHostToDevice, st) != hipSuccess)
        return WT_EDEVICE;
    // long sequences: single builds, first in the stream
    for (uint32_t q : P.solo)
        if (enqueue_build(d_S[q], P.L[q], reinterpret_cast<uint8_t *>(d_trees[q]), work + P.slice[q], st) !=
            hipSuccess)
            return WT_EDEVICE;
    static const uint32_t kWidthOf[3] = {1, 2, 4};
    for (int c = 0; c < 6; c++) {
        const uint32_t cnt = sfirst[c + 1] - sfirst[c];
        if (!cnt) continue;
        uint64_t nsym = 0, bytes = 0;
        for (uint32_t q : P.small[c]) {
            nsym += P.L[q].n;
            bytes += P.L[q].n * P.L[q].width + (P.L[q].words + P.L[q].rank_stride) * 8 * P.L[q].levels;
        }
        long pr = prof_begin(st, (c & 1) ? "batch_mid" : "batch_small", 0, kWidthOf[c / 2], nsym, bytes);
        hipError_t e = launch_small_batch(d_sjobs + sfirst[c], cnt, kWidthOf[c / 2], (c & 1) ? kGeomMid : kGeomSmall, st);
        prof_end(pr, st);
        if (e != hipSuccess) return WT_EDEVICE;
    }

    BatchClass cls[kClasses];
    for (int c = 0; c < kClasses; c++) {
        cls[c].jobs = d_jobs + first[c];
        cls[c].blk_map = reinterpret_cast<uint32_t *>(work + P.map_off[c]);
        cls[c].sup_map = reinterpret_cast<uint32_t *>(work + P.sup_off[c]);
        cls[c].njobs = (uint32_t)P.order[c].size();
    }
    const uint32_t *widths = kClassWidth;
    hipError_t err = hipSuccess;
    for (int c = 0; c < kClasses && err == hipSuccess; c++) {
        if (!cls[c].njobs) continue;
        long pr = prof_begin(st, "batch_setup", 0, widths[c], 0, 0);
        uint64_t max_ctrl = 0;
        for (uint32_t q : P.order[c]) max_ctrl = std::max(max_ctrl, P.L[q].ws_ctrl_bytes);
        err = launch_batch_setup(cls[c], max_ctrl, st);
        prof_end(pr, st);
    }
    for (int c = 0; c < kClasses && err == hipSuccess; c++) {
        if (!cls[c].njobs) continue;
        uint64_t nsym = 0;
        for (uint32_t q : P.order[c]) nsym += P.L[q].n;
        long pr = prof_begin(st, "batch_ingest", 0, widths[c], nsym, nsym * widths[c]);
        err = launch_batch_ingest(cls[c], widths[c], kClassLane[c], P.blocks[c], st);
        prof_end(pr, st);
    }
    for (uint32_t i = 0; i < maxl && err == hipSuccess; i++) {
        for (int c = 0; c < kClasses && err == hipSuccess; c++) {
            // the sequences still building level i are a prefix of the class
            uint32_t active = 0;
            uint64_t blocks = 0, sups = 0, nsym = 0, bytes = 0, nsym_multi = 0;
            for (uint32_t q : P.order[c]) {
                const Layout &L = P.L[q];
                if (L.levels <= i) break;
                active++;
                if (level_multi(L.n, i, L.width, L.lane_bytes)) nsym_multi += L.n;
                blocks += ceil_div(L.ntiles, kWaves);
                sups += L.nsup;
                nsym += L.n;
                bytes += L.n * L.width * (i + 1 < L.levels ? 2 : 1) + L.words * 8 + L.rank_stride * 8;
            }
            if (!active) continue;
            long pr = prof_begin(st, "batch_level", i, widths[c], nsym, bytes);
            // the staged split where most of the level's symbols sit in short nodes
            err = launch_batch_level(cls[c], widths[c], kClassLane[c], 2 * nsym_multi >= nsym, i, active, blocks, sups,
                                     st);
            prof_end(pr, st);
        }
    }
    if (err != hipSuccess) return WT_EDEVICE;
    for (uint32_t q = 0; q < m; q++) {
        wt_tree *h = new_handle(P.L[q], d_trees[q], st);
        if (!h) {
            for (uint32_t r = 0; r < q; r++) { delete out[r]; out[r] = nullptr; }
            return WT_ENOMEM;
        }
        out[q] = h;
    }
    return WT_OK;
}

int wt_debug_write_counters(void *d_counts, const void *d_base, uint64_t bytes) {
    if (((uintptr_t)d_base & 1) || (bytes & 1)) return WT_EINVAL;
#ifdef WT_WRITE_CHECK
    uint32_t *c = static_cast<uint32_t *>(d_counts);
    const uint64_t base = (uint64_t)(uintptr_t)d_base, span = c ? bytes : 0;
    hipError_t e = write_check_build(c, base, span);
    if (e == hipSuccess) e = write_check_small(c, base, span);
    if (e == hipSuccess) e = write_check_buffered(c, base, span);
    if (e == hipSuccess) e = write_check_quad(c, base, span);
    return e == hipSuccess ? WT_OK : WT_EDEVICE;
#else
    (void)d_counts;
    return WT_EINVAL;
#endif
}

int wt_tree_status(const wt_tree *t) {
    if (!t) return WT_EINVAL;
    if (hipStreamSynchronize(t->stream) != hipSuccess) return WT_EDEVICE;
    uint32_t flag = 0;
    if (hipMemcpy(&flag, t->tree, sizeof(flag), hipMemcpyDeviceToHost) != hipSuccess) return WT_EDEVICE;
    return (flag & 1u) ? WT_ERANGE : ((flag & 2u) ? WT_EDEVICE : WT_OK);
}

void wt_free(wt_tree *t) {
    if (!t) return;
    if (t->d_query) (void)hipFree(t->d_query);
    delete t->hm;
    delete[] t->htab;
    delete t;
}

int wt_levels(const wt_tree *t, uint32_t *levels, const uint64_t **d_bitmaps, uint64_t *words_per_level,
              const uint64_t **d_ranks, uint64_t *rank_stride, uint64_t *rank_entries) {
    // a 4-ary tree has digit levels (wt_multiary_levels), a Huffman-shaped
    // tree levels of different sizes (wt_huffman_levels)
    if (!t || t->L.arity == 4 || t->hm) return WT_EINVAL;
    if (levels) *levels = t->L.levels;
    if (d_bitmaps) *d_bitmaps = reinterpret_cast<const uint64_t *>(t->tree + t->L.tree_bits_off);
    if (words_per_level) *words_per_level = t->L.words;
    if (d_ranks) *d_ranks = reinterpret_cast<const uint64_t *>(t->tree + t->L.tree_ranks_off);
    if (rank_stride) *rank_stride = t->L.rank_stride;
    if (rank_entries) *rank_entries = t->L.rank_entries;
    return WT_OK;
}

int wt_access_batch(const wt_tree *t, const uint64_t *d_i, uint32_t *d_sym, uint64_t m, void *stream) {
    if (!t || (m > 0 && (!d_i || !d_sym))) return WT_EINVAL;
    return launch_access(view_of(t), d_i, d_sym, m, reinterpret_cast<hipStream_t>(stream)) == hipSuccess
               ? WT_OK : WT_EDEVICE;
}

int wt_rank_batch(const wt_tree *t, const uint32_t *d_c, const uint64_t *d_i, uint64_t *d_r, uint64_t m,
                  void *stream) {
    if (!t || (m > 0 && (!d_c || !d_i || !d_r))) return WT_EINVAL;
    return launch_rank(view_of(t), d_c, d_i, d_r, m, reinterpret_cast<hipStream_t>(stream)) == hipSuccess
               ? WT_OK : WT_EDEVICE;
}

int wt_select_batch(const wt_tree *t, const uint32_t *d_c, const uint64_t *d_j, uint64_t *d_pos, uint64_t m,
                    void *stream) {
    if (!t || (m > 0 && (!d_c || !d_j || !d_pos))) return WT_EINVAL;
    return launch_select(view_of(t), d_c, d_j, d_pos, m, reinterpret_cast<hipStream_t>(stream)) == hipSuccess
               ? WT_OK : WT_EDEVICE;
}

int wt_query_multi_footprint(uint32_t ntrees, uint64_t *work_bytes) {
    if (!work_bytes) return WT_EINVAL;
    *work_bytes = round_up((uint64_t)(ntrees ? ntrees : 1) * sizeof(TreeView), 256);
    return WT_OK;
}

int wt_query_multi(uint32_t ntrees, const wt_tree *const *trees, const uint32_t *d_tree, const uint8_t *d_kind,
                   const uint32_t *d_c, const uint64_t *d_x, uint64_t *d_out, uint64_t m, void *d_work,
                   uint64_t work_bytes, void *stream) {
    if (m == 0) return WT_OK;
    if (!trees || ntrees == 0 || !d_tree || !d_kind || !d_c || !d_x || !d_out || !d_work) return WT_EINVAL;
    if (((uintptr_t)d_work & 15) || work_bytes < (uint64_t)ntrees * sizeof(TreeView)) return WT_ENOMEM;
    std::vector<TreeView> views(ntrees);
    for (uint32_t k = 0; k < ntrees; k++) {
        if (!trees[k]) return WT_EINVAL;
        views[k] = view_of(trees[k]);
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // (pageable source: the call returns once the layouts are staged)
    if (hipMemcpyAsync(d_work, views.data(), ntrees * sizeof(TreeView), hipMemcpyHostToDevice, st) != hipSuccess)
        return WT_EDEVICE;
    return launch_query_multi(reinterpret_cast<const TreeView *>(d_work), ntrees, d_tree, d_kind, d_c, d_x, d_out, m,
                              st) == hipSuccess ? WT_OK : WT_EDEVICE;
}

// Single queries: argument 0 of the scratch holds the query, 2 the answer.
static int single_query(const wt_tree *t, int kind, uint32_t c, uint64_t x, uint64_t *ans) {
    wt_tree *h = const_cast<wt_tree *>(t);
    if (!h->d_query && hipMalloc(reinterpret_cast<void **>(&h->d_query), 64) != hipSuccess) {
        h->d_query = nullptr;
        return WT_EDEVICE;
    }
    uint64_t host[4] = {x, (uint64_t)c, 0, 0};
    if (hipMemcpyAsync(h->d_query, host, 32, hipMemcpyHostToDevice, h->stream) != hipSuccess) return WT_EDEVICE;
    const TreeView v = view_of(t);
    hipError_t err;
    uint32_t *cptr = reinterpret_cast<uint32_t *>(h->d_query + 1);
    if (kind == 0) err = launch_access(v, h->d_query, reinterpret_cast<uint32_t *>(h->d_query + 2), 1, h->stream);
    else if (kind == 1) err = launch_rank(v, cptr, h->d_query, h->d_query + 2, 1, h->stream);
    else err = launch_select(v, cptr, h->d_query, h->d_query + 2, 1, h->stream);
    if (err != hipSuccess) return WT_EDEVICE;
    if (hipMemcpyAsync(host, h->d_query, 32, hipMemcpyDeviceToHost, h->stream) != hipSuccess) return WT_EDEVICE;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return WT_EDEVICE;
    *ans = kind == 0 ? (uint64_t)(uint32_t)host[2] : host[2];
    return WT_OK;
}

int wt_access(const wt_tree *t, uint64_t i, uint32_t *sym) {
    if (!t || !sym || i >= t->L.n) return WT_EINVAL;
    uint64_t a = 0;
    int rc = single_query(t, 0, 0, i, &a);
    if (rc == WT_OK) *sym = (uint32_t)a;
    return rc;
}

int wt_rank(const wt_tree *t, uint32_t c, uint64_t i, uint64_t *r) {
    if (!t || !r || c >= t->L.sigma || i > t->L.n) return WT_EINVAL;
    return single_query(t, 1, c, i, r);
}

int wt_select(const wt_tree *t, uint32_t c, uint64_t j, uint64_t *pos) {
    if (!t || !pos || c >= t->L.sigma) return WT_EINVAL;
    uint64_t a = 0;
    int rc = single_query(t, 2, c, j, &a);
    if (rc != WT_OK) return rc;
    if (a == ~0ull) return WT_ENOTFOUND;
    *pos = a;
    return WT_OK;
}

static bool tune_key_ok(uint32_t mode, uint32_t width, uint32_t levels, uint32_t lg_n) {
    return mode <= 1 && (width == 1 || width == 2 || width == 4) && levels >= 1 && levels <= 24 &&
           levels <= 8 * width && lg_n <= 40;
}

int wt_tune_set(uint32_t mode, uint32_t width, uint32_t levels, uint32_t lg_n, uint32_t geometry) {
    if (!tune_key_ok(mode, width, levels, lg_n)) return WT_EINVAL;
    if (geometry != 0 && geometry != kGeomSmall && geometry != kGeomMid && !lane_bytes_valid(width, geometry))
        return WT_EINVAL;
    g_tune[mode][wclass(width)][levels][lg_n] = (uint8_t)geometry;
    return WT_OK;
}

int wt_tune_get(uint32_t mode, uint32_t width, uint32_t levels, uint32_t lg_n, uint32_t *geometry) {
    if (!tune_key_ok(mode, width, levels, lg_n) || !geometry) return WT_EINVAL;
    *geometry = resolve_geometry(g_tune[mode][wclass(width)][levels][lg_n], 1ull << lg_n, width);
    return WT_OK;
}

int wt_prof_enable(int on) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto &e : g_prof) {
        g_event_pool.push_back(e.a);
        g_event_pool.push_back(e.b);
    }
    g_prof.clear();
    g_prof_on = on != 0;
    return WT_OK;
}

int wt_prof_read(wt_prof_rec *out, uint64_t max, uint64_t *count) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto &e : g_prof) {
        if (hipEventSynchronize(e.b) != hipSuccess) return WT_EDEVICE;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess) return WT_EDEVICE;
        e.rec.ms = ms;
    }
    if (out)
        for (uint64_t k = 0; k < max && k < g_prof.size(); k++) out[k] = g_prof[k].rec;
    if (count) *count = g_prof.size();
    return WT_OK;
}

const char *wt_strerror(int s) {
    switch (s) {
        case WT_OK: return "success";
        case WT_EINVAL: return "invalid argument";
        case WT_ERANGE: return "symbol out of range (>= sigma)";
        case WT_ENOMEM: return "tree or workspace smaller than the footprint";
        case WT_ENOTFOUND: return "no such occurrence";
        case WT_EDEVICE: return "HIP runtime error";
        default: return "unknown status";
    }
}

}  // extern "C"
