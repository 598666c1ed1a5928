// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wt {

// Level pass geometry: one wave owns one tile of 64 lanes x B bytes of
// symbols (B = lane_bytes: 32, 64 or 128; B / width <= 64), i.e.
// 64 * B / width symbols, always a multiple of 512; a workgroup holds kWaves
// independent tiles.  B is picked per (width, levels, lg n) by the tuning
// table (wt_tune_set).
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr uint32_t kDefaultLaneBytes = 64;
__host__ __device__ constexpr uint64_t tile_syms(uint32_t width, uint32_t lane_bytes) {
    return 64ull * lane_bytes / width;
}
static inline bool lane_bytes_valid(uint32_t width, uint32_t lb) {
    return (lb == 32 || lb == 64 || lb == 128) && lb / width <= 64;
}
// Short sequences: one workgroup builds every level in LDS (two symbol
// buffers and a 16-bit rank per position).  Two sizes: kGeomSmall, 512
// threads in under 64 KB (two workgroups per CU), and kGeomMid, 1024 threads
// in up to 160 KB (the whole LDS of a CU).  The tuning table selects them
// with these geometry codes.
constexpr uint32_t kGeomSmall = 1;
constexpr uint32_t kGeomMid = 2;
__host__ __device__ constexpr int one_wg_threads(uint32_t geom) { return geom == kGeomMid ? 1024 : 512; }
__host__ __device__ constexpr uint32_t one_wg_cap(uint32_t width, uint32_t geom) {
    return geom == kGeomMid ? (width == 1 ? 32768u : (width == 2 ? 26624u : 15360u))
                            : (width == 1 ? 15360u : (width == 2 ? 10240u : 6144u));
}
// Entries per level of the per-tile counts: a multiple of 4, so that a lane
// reads four consecutive counts with one 16-byte load.
__host__ __device__ constexpr uint64_t tile_stride(uint64_t ntiles) { return (ntiles + 3) / 4 * 4; }
// Tree header: status word at byte 0; for a wavelet matrix, the zeros of
// every level (u64) from byte kZerosOff (24 levels fit the 256-byte header).
constexpr uint64_t kZerosOff = 8;
// Tiles per superchunk of the tile-count scan (four counts per lane).
constexpr uint64_t kSup = kThreads;
constexpr uint64_t kPrepSups = 8;  // superchunks whose sums the prep takes itself
// Node ones counters of shallow levels are spread over slots so that the
// tiles adding into them do not pile onto a few addresses: level i keeps
// max(1, kSlotSpan >> i) copies of its 2^i counters (picked by tile).
constexpr uint64_t kSlotSpan = 4096;
__host__ __device__ constexpr uint64_t level_slots(uint32_t i) {
    return (kSlotSpan >> i) > 1 ? (kSlotSpan >> i) : 1;
}
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
constexpr uint32_t kMaxTreeLevels = 24;  // lg WT_MAX_SIGMA

struct Layout {
    uint64_t n;
    uint32_t sigma, width, levels, lane_bytes;
    uint32_t small;         // 0, or kGeomSmall / kGeomMid: built by one workgroup (no workspace)
    uint32_t matrix;        // a wavelet matrix rather than a wavelet tree
    uint32_t arity;         // 4: a 4-ary tree (digit levels and per-digit directories), else binary
    uint32_t levels4;       // 4-ary levels: ceil(levels / 2)
    uint64_t dwords;        // 4-ary: 64-bit words per digit level (32 digits each, padded to 8)
    uint64_t tree_digits_off, tree_dir_off;  // 4-ary: digit levels, then directories (4 u64 per entry)
    uint64_t ws_dsum;       // 4-ary: per level and directory workgroup, four digit counts (u64)
    // four-way split passes: per digit level the tile counts of b and a & b
    // (inside the control area), their superchunk prefixes, the superchunk
    // sums of the three counts, the scan partials of large levels
    uint64_t ws_qcnt, ws_qsup, ws_qsupsum, ws_qpartials;
    uint64_t words;         // W: bitmap words per level
    uint64_t rank_entries;  // K
    uint64_t rank_stride;   // round_up(K, 8)
    uint64_t ntiles;
    uint64_t nsup;          // superchunks per level
    // tree offsets
    uint64_t tree_bits_off, tree_ranks_off, tree_bytes;
    // workspace offsets
    uint64_t ws_ta, ws_tb;              // next-level symbol buffers
    uint64_t ws_ctrl, ws_ctrl_bytes;    // zeroed at the start of a build
    uint64_t ws_tile_ones;              // levels x ntiles x u32: ones per tile of T_i
    uint64_t ws_supsum;                 // nsup x u64: per-superchunk ones of the current level
    uint64_t ws_ones;                   // per level: slots x 2^i node ones counters (u64)
    uint64_t ws_sup;                    // levels x nsup x u64: superchunk prefixes
    uint64_t ws_zo;                     // per level 2^i x (u64, u64)
    uint64_t ws_start;                  // per level 2^i + 1 node starts (u64)
    uint64_t ws_partials;               // scan partial sums
    // folded last level (u8): the record count (inside the control area),
    // two owner records per tile, and the direct path's records
    uint64_t ws_fold_cnt, ws_fold_own, ws_fold_ovf, fold_ovf_cap;
    // Narrowed symbol orders (single binary-tree builds of 2- and 4-byte
    // symbols): T_i keeps only the low 8 tw[i] bits of every symbol, which
    // hold the bits of the levels still to come.  The node of a symbol then
    // takes its high bits from the position: the anchor level of a width w
    // is levels - 8w, and the node of the anchor level holding a position
    // (its start table is that level's) gives them; ws_tanc[w - 1] holds, per
    // tile, the anchor nodes of its first and last position.
    uint32_t narrow;                    // some T_i is narrower than the input
    uint8_t tw[kMaxTreeLevels + 1];     // bytes per symbol of T_i
    uint8_t te[kMaxTreeLevels + 1];     // symbols per lane of T_i's tiles (64 te[i] symbols a tile)
    uint32_t anc_level[2];              // anchor level of widths 1 and 2 (0: none)
    uint64_t ws_tanc[2];
    uint64_t work_bytes;
};

void make_layout(uint64_t n, uint32_t sigma, uint32_t width, bool batched, Layout *L);
// The same for a given geometry code (lane bytes, kGeomSmall or kGeomMid; a
// one-workgroup code must hold n).
void make_layout_geom(uint64_t n, uint32_t sigma, uint32_t width, uint32_t geom, Layout *L);
uint32_t tuned_geometry(uint64_t n, uint32_t sigma, uint32_t width, bool batched);

// One short sequence for the one-workgroup build.
struct SmallJob {
    const void *S;
    uint8_t *tree;  // status word at offset 0, wavelet-matrix zeros at kZerosOff
    uint64_t bits_off, ranks_off;
    uint32_t n, sigma, levels, words, rank_entries, rank_stride;
    uint32_t matrix;
};
hipError_t launch_small_one(const SmallJob &j, uint32_t width, uint32_t geom, hipStream_t s);
hipError_t launch_small_batch(const SmallJob *d_jobs, uint32_t count, uint32_t width, uint32_t geom, hipStream_t s);

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
    unsigned long long *ones_next;    // next-level ones per node, slot-spread (accumulated)
    uint64_t nodes_next, slots_next;
    uint64_t n, words, rank_entries, rank_stride, ntiles;
    // positions of the next order (T_{i+1}): n, or fewer when the node
    // tables map the symbols of some children below 0 (those children are
    // dropped: a Huffman-shaped tree's leaves)
    uint64_t n_out;
    uint32_t levels, level, symmask;
    // wavelet matrix: one node per level; zeros[level] receives z_i
    uint32_t matrix;
    unsigned long long *zeros;
    // 4-ary tree: digit level written from T_i when non-null (digit of x is
    // (x >> dsh) & 3); the binary bitmap and directory are then not written
    uint64_t *digits;
    uint64_t dwords;
    uint32_t dsh;
    // last level folded into this pass (u8 trees, level l-2, single-node and
    // direct split paths only): the bitmap of level i + 1 receives bit sh - 1
    // of every symbol at its T_{i+1} position, as 16-bit granules (16
    // positions, 16-aligned) with one writer each; null otherwise.  A
    // granule wholly inside one run of a tile's split leaves the pass as one
    // 16-bit store.  The others are shared between runs: the symbols of
    // every edge chunk are stored at their positions in tout (T_{i+1}, not
    // otherwise written), and the run holding a granule's first position
    // records it (fold_own: two records per tile, one per run, ~0 for none;
    // the direct path appends to fold_ovf), so that k_fold_stitch writes it
    // once, after the pass.
    uint64_t *bits_next;
    uint64_t *fold_own;
    uint64_t *fold_ovf;
    unsigned int *fold_ovf_n;
    uint64_t fold_ovf_cap;
    uint32_t *fold_status;            // bit 1 set if fold_ovf would overflow (never, by its sizing)
    // narrowed T_i (its symbols' low 8W bits, W the pass's width, fewer bits
    // than the levels; symmask keeps those bits): the node of a symbol x at
    // position p is (anchor(p) << (8W - nsh)) | (x >> nsh), anchor(p) the
    // node of level levels - 8W holding p (node starts anc_start); tile_anc
    // gives every tile's first and last anchor.  Null otherwise.
    const uint64_t *anc_start;
    const uint2 *tile_anc;
};

// Anchor nodes of every tile (narrowed orders): out[t] = the nodes of the
// anchor level holding tile t's first and last position.
struct AnchorArgs {
    const uint64_t *start;            // the anchor level's node starts (nodes + 1)
    uint64_t nodes, n, tile, ntiles;
    uint2 *out;
};
hipError_t launch_tile_anchor(const AnchorArgs &a, hipStream_t s);

// Write-counting debug build: each translation unit that stores bitmap or
// digit words sets its own copy of the counted span (wt_check.h).
#ifdef WT_WRITE_CHECK
hipError_t write_check_build(uint32_t *cnt, uint64_t base, uint64_t bytes);
hipError_t write_check_small(uint32_t *cnt, uint64_t base, uint64_t bytes);
hipError_t write_check_buffered(uint32_t *cnt, uint64_t base, uint64_t bytes);
hipError_t write_check_quad(uint32_t *cnt, uint64_t base, uint64_t bytes);
#endif

// The granules of a folded last level that the pass recorded: one thread
// per record reads the granule's 16 symbols from T_{l-1} and writes its 16
// bits (positions >= n as zero).
struct StitchArgs {
    const uint8_t *t;                 // T_{l-1} (edge symbols at their positions)
    const uint64_t *own;              // nown records (~0: none)
    const uint64_t *ovf;              // direct-path records, *ovf_n of them (at most ovf_cap)
    const unsigned int *ovf_n;
    uint16_t *bits16;                 // the last level's bitmap as 16-bit granules
    uint64_t nown, ovf_cap, n;
    uint32_t sh;                      // bit of the last level (0)
};
hipError_t launch_fold_stitch(const StitchArgs &a, hipStream_t s);
// Records the direct path of a folded pass can append: tiles spanning
// several nodes number fewer than the nodes of level l-2 (at most 2^(l-2)),
// and such a tile's destinations hold at most TILE/16 + (its runs: two per
// node) multiples of 16.
static inline uint64_t fold_ovf_capacity(uint64_t ntiles, uint32_t levels, uint64_t tile) {
    const uint64_t nodes = levels >= 2 ? (1ull << (levels - 2)) : 1ull;
    const uint64_t tiles = ntiles < nodes ? ntiles : nodes;
    return tiles * (tile / 16 + 2 * nodes + 1);
}

// Rank directory of one bitmap level from its words (entry k = ones before
// position 512k for k < nblk, entry nblk = all ones, zero padding up to
// rank_stride); wsum holds nwg = ceil(nblk / kBitDirBlocks) partial sums.
constexpr uint64_t kBitDirBlocks = 256;
struct BitDirArgs {
    const uint64_t *bits;            // words = 8 * nblk
    uint64_t *ranks;
    unsigned long long *wsum;
    uint64_t nblk, nwg, rank_stride;
};
hipError_t launch_bitdir(const BitDirArgs &a, hipStream_t s);

struct IngestArgs {
    const void *S;
    uint32_t *tile_ones0;              // ones of level 0 per tile
    unsigned long long *ones0;         // ones of the root, slot-spread
    uint64_t *start0;                  // node starts of level 0: {0, n}
    uint32_t *tree_status;
    uint64_t n, ntiles, tiles_per_block, slots0;
    uint32_t sigma, check, msb;
    uint16_t *zero_g;                  // zero_granules 16-bit granules cleared on the way, or null
    uint64_t zero_granules;
};

// Node tables of one level (see k_plan_* and k_prep).
struct PlanArgs {
    const uint64_t *start;             // level i node starts (2^i + 1)
    const unsigned long long *ones;    // level i ones per node, `slots` copies
    ulonglong2 *zo;                    // level i output
    uint64_t *start_next;              // level i+1 starts (null on the last level)
    uint64_t *partials;
    uint64_t nodes, slots, n;
    uint32_t matrix;                   // wavelet matrix: the next level is again one node [0, n)
    // subtracted from every next-level position (zo and start_next): the
    // next level then lists only the children at or after that position
    // (Huffman-shaped tree: its leaves at the next depth come first); 0 else
    uint64_t shift;
};

struct PrepArgs {
    const uint32_t *tile_ones;           // this level's ones per tile
    unsigned long long *supsum;          // per-superchunk sums (k_supsum output)
    unsigned long long *sup;             // their exclusive prefixes (k_prep output)
    uint64_t ntiles, nsup;
    PlanArgs plan;
    uint32_t plan_here;                  // node tables built here (levels up to kScanChunk nodes)
    uint32_t sums_here;                  // superchunk sums taken here from tile_ones (no k_supsum):
                                         // at most kPrepSups superchunks, plan_here, fewer than kThreads nodes
};

// One sequence of a batched build as the batch kernels see it (its layout,
// with the per-level table offsets derived on the device).
struct BatchJob {
    const void *S;
    uint8_t *tree;
    uint8_t *work;
    uint64_t n, words, rank_entries, rank_stride, ntiles, nsup;
    uint64_t tree_bits_off, tree_ranks_off;
    uint64_t ws_ta, ws_tb, ws_ctrl, ws_ctrl_bytes, ws_tile_ones, ws_ones, ws_sup, ws_supsum, ws_zo, ws_start;
    uint64_t ws_partials;
    uint64_t blk_base;  // first workgroup of this sequence in its class's tile map
    uint64_t sup_base;  // first workgroup of this sequence in its class's superchunk map
    uint32_t sigma, width, levels, check, lane_bytes;
};

// Sequences that share one symbol width, sorted by level count (descending),
// so the sequences still building level i are always a prefix.
struct BatchClass {
    const BatchJob *jobs;
    uint32_t *blk_map;  // tile workgroup -> sequence
    uint32_t *sup_map;  // superchunk workgroup -> sequence
    uint32_t njobs;
};

// Per-level table offsets (entries) shared by the host layout and the device.
__host__ __device__ constexpr uint64_t zo_offset(uint32_t i) { return (1ull << i) - 1; }
__host__ __device__ constexpr uint64_t start_offset(uint32_t i) { return (1ull << i) - 1 + i; }
// sum of level_slots(k) << k over k < i: kSlotSpan per level up to the
// level where one slot remains, then 2^k
__host__ __device__ inline uint64_t ones_offset(uint32_t i) {
    constexpr uint32_t kFull = 12;  // kSlotSpan >> 12 == 1
    static_assert((kSlotSpan >> kFull) == 1, "slot span");
    return (i <= kFull + 1) ? (uint64_t)kSlotSpan * i
                            : (uint64_t)kSlotSpan * (kFull + 1) + ((1ull << i) - (1ull << (kFull + 1)));
}

// kernel launchers (wt_build.hip)
// Zeroes `bytes` at p, count2 words at p2 (when non-null) and the status word.
hipError_t launch_zero(void *p, uint64_t bytes, uint32_t *tree_status, uint64_t *p2, uint64_t count2, hipStream_t s);
hipError_t launch_ingest(const IngestArgs &a, uint32_t width, uint32_t lane_bytes, hipStream_t s);
hipError_t launch_prep(const PrepArgs &a, hipStream_t s);  // k_supsum, then k_prep
hipError_t launch_plan(const PlanArgs &a, hipStream_t s);
// out_width: bytes per symbol of T_{i+1}: width, or width / 2 (a narrowing
// pass; lane_bytes 64 or 128, never multi); out_lane_bytes: lane bytes of
// T_{i+1}'s tiles (lane_bytes, or for a narrowing pass lane_bytes / 2 or,
// doubling the symbols per lane, lane_bytes)
hipError_t launch_level(const LevelArgs &a, uint32_t width, uint32_t lane_bytes, bool multi, uint32_t out_width,
                        uint32_t out_lane_bytes, hipStream_t s);
// Whether a narrowing pass exists for this width and lane size.
__host__ __device__ constexpr bool narrowing_pass(uint32_t width, uint32_t lane_bytes) {
    return (width == 4 || width == 2) && (lane_bytes == 64 || lane_bytes == 128);
}
// Whether one also exists that doubles the symbols per lane of T_{i+1}.
__host__ __device__ constexpr bool narrowing_pass_doubling(uint32_t width, uint32_t lane_bytes) {
    return (width == 4 || width == 2) && lane_bytes == 64;
}
// Level passes take the staged split of tiles spanning a few nodes where the
// average node is shorter than this many tiles.
constexpr uint64_t kMultiAvgTiles = 8;
__host__ __device__ constexpr bool level_multi(uint64_t n, uint32_t level, uint32_t width, uint32_t lane_bytes) {
    return (n >> level) < kMultiAvgTiles * tile_syms(width, lane_bytes);
}
hipError_t launch_batch_setup(const BatchClass &c, uint64_t max_ctrl_bytes, hipStream_t s);
hipError_t launch_batch_ingest(const BatchClass &c, uint32_t width, uint32_t lane_bytes, uint64_t blocks,
                               hipStream_t s);
hipError_t launch_batch_level(const BatchClass &c, uint32_t width, uint32_t lane_bytes, bool multi, uint32_t level,
                              uint32_t active, uint64_t blocks, uint64_t sups, hipStream_t s);

// Buffered build (wt_buffered.hip): merge of the partial trees of nbuf
// buffers into one tree.
struct MergeArgs {
    unsigned long long *C;           // (nbuf + 1) rows of `row` = 2^l + 1 leaf offsets
    const uint8_t *ptrees;           // partial trees, pstride bytes apart (status word first)
    uint64_t pstride, pbits_off;     // partial tree stride and bitmap offset
    uint64_t pwords, pwords_last;    // bitmap words per level of a full / the last partial tree
    uint64_t *bits;                  // final bitmaps, `words` per level
    uint64_t *ranks;                 // final rank directories, `rank_stride` per level
    uint32_t *tree_status;           // final status word
    unsigned long long *csum;        // per level, wg_per_level workgroup sums
    uint64_t *span_run;              // per level, wg_per_level + 1 first runs of the merge spans
    uint64_t n, words, rank_stride, nblk, wg_per_level, row;
    uint32_t levels, nbuf;
};
hipError_t launch_leaf_prefix(const uint64_t *start_last, const ulonglong2 *zo_last, uint32_t levels, uint64_t nq,
                              unsigned long long *row, hipStream_t s);
hipError_t launch_merge(const MergeArgs &a, hipStream_t s);  // column prefix, merge, rank directory, status

// 4-ary tree directories (wt_multiary.hip): entry k of a level holds the
// counts of digits 0..3 in positions [0, min(512 k, n)).
struct DigitDirArgs {
    const uint64_t *digits;         // levels x dwords words
    uint64_t *dir;                  // levels x dir_stride entries x 4 counts
    unsigned long long *wsum;       // levels x wg_per_level x 4 counts
    uint64_t n, dwords, dir_stride, nblk, wg_per_level;
    uint32_t levels;
};
constexpr uint64_t kDirBlocksPerWG = 256;  // 512-position blocks per directory workgroup
hipError_t launch_digit_dir(const DigitDirArgs &a, hipStream_t s);

// Huffman-shaped tree (wt_huffman.hip, wt_api.hip, wt_query.hip).  Its
// tree memory starts with the 256-byte header (status word first), then this
// table at kHeaderBytes, then the per-symbol code table, the symbols in code
// order, the depth bitmaps and their directories.  Depth d holds size[d] =
// n_d positions (the symbols whose code is longer than d); in the order of
// the first d bits of the left-aligned codes over all of S, those positions
// come after the n - n_d symbols whose code ends by depth d.
constexpr uint32_t kHuffMaxLevels = 24;
constexpr uint64_t kHuffMetaBytes = 1280;
struct HuffMeta {
    uint64_t n;
    uint32_t sigma, levels, distinct, only;     // only: the one symbol of S when levels = 0 and n > 0
    uint64_t size[kHuffMaxLevels];              // n_d
    uint64_t bits_off[kHuffMaxLevels];          // byte offsets from the tree base
    uint64_t dir_off[kHuffMaxLevels];
    uint64_t dir_entries[kHuffMaxLevels];       // ceil(n_d / 512) + 1
    uint32_t first[kHuffMaxLevels + 1];         // canonical: first code of each length (right-aligned)
    uint32_t count[kHuffMaxLevels + 1];         // codes of each length
    uint32_t start[kHuffMaxLevels + 1];         // their first index in the code-ordered symbol list
    uint64_t code_off, syms_off;                // byte offsets of the two tables
};
static_assert(sizeof(HuffMeta) <= kHuffMetaBytes, "Huffman table size");
// code table entry of a symbol: bits 0-4 its code length, bit 7 set when the
// symbol occurs, bits 8-31 its code (right-aligned)
constexpr uint32_t kHuffPresent = 0x80u;

hipError_t launch_histogram(const void *S, uint64_t n, uint32_t width, uint32_t sigma, unsigned long long *counts,
                            hipStream_t s);
// K[j] = code of S[j] left-aligned to `levels` bits, stored at width wout;
// status bit 0 for a symbol >= sigma or absent from the code table
hipError_t launch_huff_map(const void *S, uint64_t n, uint32_t width, const uint32_t *code_tab, uint32_t sigma,
                           uint32_t levels, void *K, uint32_t wout, uint32_t *status, hipStream_t s);


// Four-way split (wt_quad.hip): one pass over T_i writes T_{i+2}, the
// symbols of every level-i node stably split into its four grandchildren by
// the two bits below the node prefix, the digit d = 2a + b (a = bit l-1-i, b =
// bit l-2-i).  Per tile of T_i the pass needs the counts of a, of b and of
// a & b (prefix-summed over tiles: A(p), B(p), AB(p) = the counts before
// position p); per node v the table K(v) = (K0, K1, K2, K3) with
//   destination of digit 0 at p: K0 + p - A(p) - B(p) + AB(p)
//   digit 1: K1 + B(p) - AB(p),  digit 2: K2 + A(p) - AB(p),  digit 3: K3 + AB(p).
// Node counts come in the binary counters of levels i (a-ones per level-i
// node) and i + 1 (b-ones per level-(i+1) node 2v + a).
struct QuadArgs {
    const void *tin;
    void *tout;                        // T_{i+2} (null: no next order)
    const ulonglong2 *K;               // per node: (K0, K1), (K2, K3)
    const uint32_t *cnt[3];            // per tile of T_i: counts of a, b, a & b
    const unsigned long long *sup[3];  // their superchunk prefixes
    uint32_t *cnt_next[3];             // the same for T_{i+2} (accumulated), or null
    unsigned long long *ones_a_next;   // level i+2: a'-ones per node (slot-spread), or null
    unsigned long long *ones_b_next;   // level i+3: b'-ones per node 2g + a' (slot-spread), or null
    uint64_t nodes_a_next, slots_a_next, nodes_b_next, slots_b_next;
    uint64_t n, ntiles;
    uint32_t levels, level, symmask;   // level = i (even for a 4-ary tree's digit level i / 2)
    // 4-ary tree: digit level i / 2 (32 digits per word), or null
    uint64_t *digits;
    uint64_t dwords;
};
hipError_t launch_quad(const QuadArgs &a, uint32_t width, uint32_t lane_bytes, hipStream_t s);

// Node tables of a four-way level: superchunk prefixes of the three tile
// counts, K(v) for the 2^i nodes of level i, and the node starts of level
// i + 2 (four per node).
struct QuadPrepArgs {
    const uint32_t *cnt[3];
    unsigned long long *supsum[3];     // scratch: per-superchunk sums
    unsigned long long *sup[3];        // output: their exclusive prefixes
    uint64_t ntiles, nsup;
    const uint64_t *start;             // level i node starts (nodes + 1)
    const unsigned long long *ones_a;  // level i a-ones, slots_a copies
    const unsigned long long *ones_b;  // level i+1 b-ones (2 nodes per level-i node), slots_b copies
    uint64_t slots_a, slots_b;
    ulonglong2 *K;                     // output: 2 per node
    uint64_t *start_next;              // output: level i+2 starts (4 nodes + 1), or null
    unsigned long long *partials;      // scratch: 3 per chunk of kScanChunk nodes
    uint64_t nodes, n;
};
hipError_t launch_quad_prep(const QuadPrepArgs &a, hipStream_t s);

// Counts of the first four-way level straight from S: per tile of S the
// counts of a, b, a & b (the two top bits of l), the root's a-ones and the
// b-ones of the two level-1 nodes; symbols >= sigma flagged.
struct QuadIngestArgs {
    const void *S;
    uint32_t *cnt[3];
    unsigned long long *ones_a0;       // slots_a0 copies of 1 node
    unsigned long long *ones_b1;       // slots_b1 copies of 2 nodes
    uint64_t slots_a0, slots_b1;
    uint64_t *start0;                  // {0, n}
    uint32_t *tree_status;
    uint64_t n, ntiles;
    uint32_t sigma, check, levels;
};
hipError_t launch_quad_ingest(const QuadIngestArgs &a, uint32_t width, uint32_t lane_bytes, hipStream_t s);

// query launchers (wt_query.hip)
struct TreeView {
    const uint64_t *bits;
    const uint64_t *ranks;
    const unsigned long long *zeros;  // wavelet matrix: zeros of every level (else null)
    uint64_t n, words, rank_entries, rank_stride;
    uint32_t sigma, levels;
    // 4-ary tree (digits non-null): levels4 digit levels of dwords words and
    // their directories (rank_stride entries of four counts each)
    const uint64_t *digits;
    const uint64_t *dir;
    uint64_t dwords;
    uint32_t levels4;
    // Huffman-shaped tree (non-null): its table and tree base (device)
    const HuffMeta *huff;
    const uint8_t *hbase;
};
hipError_t launch_access(const TreeView &t, const uint64_t *i, uint32_t *sym, uint64_t m,
                         hipStream_t s);
hipError_t launch_rank(const TreeView &t, const uint32_t *c, const uint64_t *i, uint64_t *r,
                       uint64_t m, hipStream_t s);
hipError_t launch_select(const TreeView &t, const uint32_t *c, const uint64_t *j,
                         uint64_t *pos, uint64_t m, hipStream_t s);
hipError_t launch_query_multi(const TreeView *d_views, uint32_t ntrees, const uint32_t *tree, const uint8_t *kind,
                              const uint32_t *c, const uint64_t *x, uint64_t *out, uint64_t m, hipStream_t s);

}  // namespace wt
