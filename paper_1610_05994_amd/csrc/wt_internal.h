// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wt {

// Level pass geometry: one wave owns one tile of 64 lanes x 64 bytes of
// symbols, i.e. 4096 / width symbols (4096, 2048 or 1024), always a
// multiple of 512; a workgroup holds kWaves independent tiles.
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr uint64_t kTileBytes = 64 * 64;
__host__ __device__ constexpr uint64_t tile_syms(uint32_t width) { return kTileBytes / width; }
// Tiles per superchunk of the tile-count scan (four counts per lane).
constexpr uint64_t kSup = kThreads;
// Levels whose node offsets come straight from the first-pass histogram.
constexpr uint32_t kTopBits = 12;
// LDS words of the ingest histogram: every bin has 8192 / nbins copies
// (lane L adds into copy L % copies), spreading the hot bins of skewed data
// over banks.
constexpr uint32_t kHistWords = 8192;
// Tiles spanning at most this many nodes aggregate next-level counts in LDS.
constexpr uint32_t kNodeCap = 128;
// Entries of the node-offset scan handled by one workgroup.
constexpr uint64_t kScanChunk = 4096;
constexpr uint64_t kMaxScanBlocks = (1ull << 23) / kScanChunk;  // sigma <= 2^24

constexpr uint64_t kHeaderBytes = 256;

__host__ __device__ static inline uint64_t round_up(uint64_t x, uint64_t m) { return (x + m - 1) / m * m; }
__host__ __device__ static inline uint64_t ceil_div(uint64_t x, uint64_t m) { return (x + m - 1) / m; }

static inline uint32_t levels_for(uint32_t sigma) {
    uint32_t l = 0;
    while ((1ull << l) < (uint64_t)sigma) l++;
    return l;
}

// Byte layout of one tree (in caller memory) and of one build's workspace.
struct Layout {
    uint64_t n;
    uint32_t sigma, width, levels, top_bits;
    uint64_t words;         // W: bitmap words per level
    uint64_t rank_entries;  // K
    uint64_t rank_stride;   // round_up(K, 8)
    uint64_t ntiles;
    // tree offsets
    uint64_t tree_bits_off, tree_ranks_off, tree_bytes;
    // workspace offsets
    uint64_t ws_ta, ws_tb;              // next-level symbol buffers
    uint64_t ws_ctrl, ws_ctrl_bytes;    // zeroed at the start of a build
    uint64_t ws_tile_ones;              // levels x ntiles x u32: ones per tile of T_i
    uint64_t ws_hist;                   // 2^top_bits x u64
    uint64_t ws_ones;                   // ones counts for levels >= top_bits
    uint64_t ws_sup;                    // levels x nsup x u64: superchunk prefixes
    uint64_t ws_done;                   // levels x u32: finished superchunk-sum workgroups
    uint64_t ws_zo;                     // per level 2^i x (u64, u64)
    uint64_t ws_start;                  // start offsets for levels >= top_bits
    uint64_t ws_partials;               // scan partial sums
    uint64_t nsup;                      // superchunks per level
    uint64_t work_bytes;
    // per-level table offsets (entries), level < 32
    uint64_t ones_off[32], zo_off[32], start_off[32];
};

void make_layout(uint64_t n, uint32_t sigma, uint32_t width, Layout *L);

// Arguments of one level pass.
struct LevelArgs {
    const void *tin;
    void *tout;                       // null on the last level
    uint64_t *bits;                   // level bitmap
    uint64_t *ranks;                  // level rank directory
    const ulonglong2 *zo;             // per node: (zero base, one base)
    const uint32_t *tile_ones;        // ones per tile of this level
    const unsigned long long *sup;    // exclusive prefix of the superchunks of tile_ones
    uint32_t *tile_ones_next;         // ones per tile of the next level (accumulated), or null
    unsigned long long *ones_next;    // next-level ones per node (accumulated), or null
    uint64_t n, words, rank_entries, rank_stride, ntiles;
    uint32_t levels, level, symmask;
};

struct IngestArgs {
    const void *S;
    unsigned long long *hist;
    uint32_t *tile_ones0;   // ones of level 0 per tile (null when there is no level)
    uint64_t tiles_per_block;  // a multiple of kWaves dividing kSup
    uint32_t *tree_status;
    uint64_t n, ntiles;
    uint32_t sigma, symmask, hshift, nbins, copies, msb;
};

struct TopArgs {
    const unsigned long long *hist;
    ulonglong2 *zo;        // base of the zo arena (level i at zo_off[i])
    uint64_t *start_h;     // start offsets of level top_bits (if it exists)
    uint64_t n;
    uint32_t h, levels;
    uint64_t zo_off[32];
};

struct PlanArgs {
    const uint64_t *start;     // level i node starts (2^i + 1)
    const unsigned long long *ones;  // level i ones per node (2^i)
    ulonglong2 *zo;            // level i output
    uint64_t *start_next;      // level i+1 starts (null on the last level)
    uint64_t *partials;
    uint64_t nodes, n;
};

// kernel launchers (wt_build.hip)
hipError_t launch_zero(void *p, uint64_t bytes, uint32_t *tree_status, uint64_t *tree_ranks,
                       uint64_t tree_ranks_count, hipStream_t s);
hipError_t launch_ingest(const IngestArgs &a, uint32_t width, hipStream_t s);
hipError_t launch_supsum(const uint32_t *tile_ones, unsigned long long *sup, uint32_t *done, uint64_t ntiles,
                         hipStream_t s);
hipError_t launch_top(const TopArgs &a, hipStream_t s);
hipError_t launch_plan(const PlanArgs &a, hipStream_t s);
hipError_t launch_level(const LevelArgs &a, uint32_t width, hipStream_t s);

// query launchers (wt_query.hip)
struct TreeView {
    const uint64_t *bits;
    const uint64_t *ranks;
    uint64_t n, words, rank_entries, rank_stride;
    uint32_t sigma, levels;
};
hipError_t launch_access(const TreeView &t, const uint64_t *i, uint32_t *sym, uint64_t m,
                         hipStream_t s);
hipError_t launch_rank(const TreeView &t, const uint32_t *c, const uint64_t *i, uint64_t *r,
                       uint64_t m, hipStream_t s);
hipError_t launch_select(const TreeView &t, const uint32_t *c, const uint64_t *j,
                         uint64_t *pos, uint64_t m, hipStream_t s);

}  // namespace wt
