/*
 * wtree.h -- C ABI of the MI355X wavelet-tree construction library.
 *
 * Problem (Fuentes-Sepulveda et al., "Parallel Construction of Wavelet Trees
 * on Multicore Architectures", Section 2.3 problem statement, Section 2.2
 * definitions): given a sequence S of n symbols over the alphabet [0, sigma),
 * build the pointerless wavelet tree -- one n-bit bitmap per level, l =
 * ceil(lg sigma) levels -- in which level i lists, node after node in prefix
 * order, bit (l-1-i) of every symbol, the symbols of a node (those sharing
 * their top i bits, Proposition 1) keeping their input order.  Each level also
 * gets a rank directory.  The construction runs on the GPU; queries are
 * provided for verification and serving.
 *
 * Conventions (the paper does not fix them):
 *  - symbols are 0-based, stored as unsigned 8-, 16- or 32-bit integers
 *    (width 1, 2 or 4 bytes); 1 <= sigma <= min(2^(8*width), 2^24);
 *  - non-power-of-two alphabets split by bit prefix over l bits (nodes whose
 *    codes are >= sigma are simply empty);
 *  - positions are 0-based; rank(c, i) counts occurrences in [0, i) for
 *    i in [0, n]; select(c, j) takes a 1-based j and returns a 0-based
 *    position;
 *  - bitmap words are 64-bit, position p of a level sits in word p/64 at bit
 *    p%64 (least significant bit first); each level owns
 *    W = round_up(ceil(n/64), 8) words and every bit at a position >= n is 0;
 *  - the rank directory of a level holds K = ceil(n/512) + 1 absolute 64-bit
 *    counts R[k] = ones in positions [0, min(512k, n)) in a slot of
 *    round_up(K, 8) entries whose padding entries are 0.
 *
 * Memory and ownership:
 *  - every pointer named d_* is device memory of the current HIP device;
 *  - the caller owns the input, the tree memory and the workspace, sized by
 *    wt_footprint / wt_batch_footprint; the library owns only the small host
 *    handle (wt_tree) returned by a build and released by wt_free;
 *  - all work is enqueued on the given stream (a hipStream_t passed as
 *    void*, NULL = the null stream) and is asynchronous: the input must stay
 *    valid and unmodified until the stream has passed the build, and the
 *    tree is complete once the stream has passed it;
 *  - the workspace may be reused for another build once the stream has
 *    passed the previous one; tree memory holds the finished tree;
 *  - the input must be 16-byte aligned (any torch allocation is).
 *
 * Errors: every int-returning function returns a status below; no exception
 * or abort crosses the ABI.  A symbol >= sigma is found on the device, after
 * the call has returned: wt_tree_status reports it (WT_ERANGE) once the
 * stream has passed the build; the bitmaps of such a build are unspecified.
 */
#ifndef WTREE_H
#define WTREE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    WT_OK = 0,
    WT_EINVAL = 1,     /* bad argument (null pointer, width, sigma, size, alignment) */
    WT_ERANGE = 2,     /* some symbol is >= sigma */
    WT_ENOMEM = 3,     /* tree or workspace smaller than the footprint */
    WT_ENOTFOUND = 4,  /* select beyond the number of occurrences */
    WT_EDEVICE = 5     /* a HIP runtime call failed */
};

#define WT_MAX_SIGMA (1u << 24)
#define WT_MAX_N (1ull << 40)

typedef struct wt_tree wt_tree; /* opaque host handle */

typedef struct wt_desc {
    uint64_t n;     /* number of symbols, 0 <= n < WT_MAX_N */
    uint32_t sigma; /* alphabet size, 1 <= sigma <= WT_MAX_SIGMA */
    uint32_t width; /* bytes per stored symbol: 1, 2 or 4 */
} wt_desc;

/*
 * Bytes of tree memory and of workspace that wt_build needs for *desc (the
 * memory question of Section 4.3: the tree itself is l n-bit levels plus
 * their rank directories, the workspace two n-symbol order buffers and the
 * per-level node tables).  Pure host computation (no device call).
 */
int wt_footprint(const wt_desc *desc, uint64_t *tree_bytes, uint64_t *work_bytes);

/*
 * Build the wavelet tree of d_S (desc->n symbols of desc->width bytes) into
 * d_tree (tree_bytes >= the footprint), using d_work (work_bytes >= the
 * footprint) as scratch, on `stream`.  On WT_OK *out receives a new handle
 * describing the tree (release it with wt_free); on error *out is NULL and
 * nothing was enqueued.  Follows the per-level construction of Section 3.1
 * (count, prefix sum, stable fill per level; Algorithm pwt) and the
 * segment-count / offset-scan idea of Section 3.2 (Algorithm dd), organised
 * for the GPU as described in the library's design notes.
 */
int wt_build(const void *d_S, const wt_desc *desc, void *d_tree, uint64_t tree_bytes,
             void *d_work, uint64_t work_bytes, void *stream, wt_tree **out);

/*
 * Wavelet matrix of S (a variant the paper names as future work, Section 5;
 * built from its standard definition): A_0 = S, level i's bitmap is bit
 * (l-1-i) of A_i position by position, and A_{i+1} is A_i stably
 * partitioned by that bit over the whole level (zeros first).  Same
 * arguments, footprint (wt_footprint), memory rules and bitmap / rank
 * directory layout as wt_build; the zeros z_i of every level are kept in
 * the tree header and returned by wt_matrix_zeros.  All queries below accept
 * a matrix handle and answer for S (access / rank / select walk the levels
 * with z_i: bit b at p continues at rank0(p), or z_i + rank1(p)).
 */
int wt_build_matrix(const void *d_S, const wt_desc *desc, void *d_tree, uint64_t tree_bytes,
                    void *d_work, uint64_t work_bytes, void *stream, wt_tree **out);

/*
 * zeros[i] = z_i for the levels i of a wavelet matrix (host array of
 * `levels` entries); waits for the build's stream.  WT_EINVAL for a tree
 * handle.
 */
int wt_matrix_zeros(const wt_tree *tree, uint64_t *zeros);

/*
 * 4-ary wavelet tree of S (multiary trees, whose nodes have more than two
 * children, are future work in Section 5; this is the one-pointer-per-level
 * representation with fan-out 4).  With l = ceil(lg sigma), symbols are read
 * as codes of L4 = ceil(l / 2) base-4 digits (a zero bit on top when l is
 * odd).  Digit level i lists, node after node, digit i of every symbol
 * (bits 2(L4-1-i) + 1 and 2(L4-1-i)); the node of s at level i is
 * s >> 2(L4-i) and the symbols of a node keep their input order.
 *
 * Layout (tree memory of wt_multiary_footprint bytes): the 256-byte header
 * (status word first); then L4 digit levels of round_up(ceil(n/32), 8)
 * 64-bit words, digit p in word p/32 at bits 2(p%32) and 2(p%32)+1, every
 * digit at a position >= n zero; then L4 directories of round_up(K, 8)
 * entries, K = ceil(n/512) + 1, each entry four u64 counts: entry k holds
 * the number of digits 0, 1, 2, 3 in positions [0, min(512k, n)); padding
 * entries are zero.  Same arguments, memory rules and status reporting as
 * wt_build; the workspace is wt_multiary_footprint's.  The queries below
 * accept a 4-ary handle (digit walks: the child of digit d of node [b, e)
 * follows the digits smaller than d of [b, e) at the next level); wt_levels
 * does not (WT_EINVAL), wt_multiary_levels gives the digit levels instead.
 */
int wt_multiary_footprint(const wt_desc *desc, uint64_t *tree_bytes, uint64_t *work_bytes);
int wt_build_multiary(const void *d_S, const wt_desc *desc, void *d_tree, uint64_t tree_bytes,
                      void *d_work, uint64_t work_bytes, void *stream, wt_tree **out);
int wt_multiary_levels(const wt_tree *tree, uint32_t *levels, const uint64_t **d_digits,
                       uint64_t *words_per_level, const uint64_t **d_dir, uint64_t *dir_stride);

/*
 * Buffered build (the extension for inputs that do not fit, Section 5, on
 * Algorithm dd of Section 3.2 and Function mergeBA): S is read in buffers of
 * buffer_syms symbols; each buffer is copied to the device and built as a
 * partial tree without using the rest of S, the partial trees' node offsets
 * are combined by prefix sums over the buffers, and the partial bitmaps are
 * concatenated into the final levels, whose rank directories are then
 * written.  The tree is the one wt_build produces (same layout and
 * queries).
 *
 * S may be host memory (page-locked memory lets the copies of the next
 * buffers overlap the build of the current one; pageable memory works too)
 * or device memory, any alignment.  The device holds four staging buffers, one
 * partial-build workspace, the partial trees (about the size of the final
 * tree's bitmaps) and an offset table of (buffers + 1) x (2^l + 1) u64, so
 * the workspace grows with n l / 8 + (n / buffer_syms) 2^l * 8 bytes rather
 * than with n * width.  With n <= buffer_syms it is one ordinary build of a
 * staged copy.  The call returns once every symbol of S has been read (S may
 * then be reused); the partial builds still in flight and the merge complete
 * on `stream`.  WT_EINVAL for buffer_syms = 0 or more than 2^20 buffers.
 */
int wt_buffered_footprint(const wt_desc *desc, uint64_t buffer_syms, uint64_t *tree_bytes,
                          uint64_t *work_bytes);
int wt_build_buffered(const void *S, const wt_desc *desc, uint64_t buffer_syms, void *d_tree,
                      uint64_t tree_bytes, void *d_work, uint64_t work_bytes, void *stream,
                      wt_tree **out);

/*
 * Workspace bytes that wt_build_batch needs for the m sequences descs[0..m).
 * Tree memory of sequence q is its own wt_footprint tree_bytes.  (Which
 * long sequences are built alone depends on the whole batch, so the figure
 * for a batch is not always at most the sum of its members' figures.)
 */
int wt_batch_footprint(uint32_t m, const wt_desc *descs, uint64_t *work_bytes);

/*
 * Huffman-shaped wavelet tree (compressed wavelet trees are future work in
 * Section 5; the paper gives no definition, so this is the standard one): the
 * tree's shape is the code tree of a Huffman code for the symbol counts of S.
 * A symbol that occurs is a leaf at the depth of its code length, reached by
 * its code bits (0 = left); every internal node lists, for the symbols of its
 * subtree in input order, their next code bit.  Depth d's bitmap is the
 * concatenation, left to right, of the bitmaps of the internal nodes at depth
 * d: n_d bits, n_d = the number of symbols whose code is longer than d.  The
 * code is fixed as follows: lengths by Huffman's merging with two
 * first-in first-out queues (the symbols that occur, by count then symbol;
 * the merged items in the order they are made), the lighter front first and
 * the symbol queue on equal weights; canonical codes from the lengths
 * (symbols by length then symbol, each code the previous plus one, shifted
 * left by the increase in length).  A single distinct symbol (or n = 0)
 * gives a tree with no levels.  Codes longer than 24 bits are not supported
 * (WT_EINVAL).
 *
 * wt_histogram writes the sigma symbol counts of d_S (u64, device memory of
 * 8 * sigma bytes, 8-byte aligned) on `stream`; symbols >= sigma are not
 * counted.  The caller copies them to the host and passes them to
 * wt_huffman_footprint (tree and workspace bytes) and wt_build_huffman; the
 * counts must add up to n (else WT_EINVAL) and be those of S (a symbol that
 * occurs with a zero count, or >= sigma, is reported as WT_ERANGE by
 * wt_tree_status).  The build enqueues a copy of its code tables (host memory
 * owned by the handle: release the handle only after the stream has passed
 * the build) and the kernels on `stream`.
 *
 * Layout of the tree memory: the 256-byte header (status word first), a
 * 1280-byte table (sizes and byte offsets of every depth, canonical code
 * bounds), a u32 per symbol (bits 0-4 its code length, bit 7 set if it
 * occurs, bits 8-31 its code), the symbols in code order, then the depth
 * bitmaps (depth d: round_up(ceil(n_d/64), 8) words, position p in word p/64
 * at bit p%64, bits past n_d zero) and their directories (round_up(K_d, 8)
 * entries, K_d = ceil(n_d/512) + 1, entry k = ones in [0, min(512k, n_d))).
 * wt_huffman_levels gives, per depth, n_d and the byte offsets of its bitmap
 * and directory in the tree memory, K_d, and (optionally, sigma entries) the
 * code table.  The access / rank / select entry points accept the handle
 * (walks over the depths; a leaf is recognised by its canonical code).
 */
int wt_histogram(const void *d_S, const wt_desc *desc, uint64_t *d_counts, void *stream);
int wt_huffman_footprint(const uint64_t *counts, const wt_desc *desc, uint64_t *tree_bytes, uint64_t *work_bytes);
int wt_build_huffman(const void *d_S, const wt_desc *desc, const uint64_t *counts, void *d_tree,
                     uint64_t tree_bytes, void *d_work, uint64_t work_bytes, void *stream, wt_tree **out);
int wt_huffman_levels(const wt_tree *tree, uint32_t *levels, uint64_t *sizes, uint64_t *bits_off,
                      uint64_t *dir_off, uint64_t *dir_entries, uint32_t *code_table);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): wt_build
 * with the workspace taken from a fixed device array inside the library
 * (WT_NOALLOC_WORK_BYTES on each device, held until the process ends)
 * instead of d_work.  No device or host memory is allocated and no handle is
 * returned: the tree lands in d_tree (tree_bytes >= wt_footprint's
 * tree_bytes) with the layout above, and its status word (the first 32 bits
 * of d_tree: 0 = success, bit 0 = some symbol >= sigma) is valid once the
 * stream has passed the build.  WT_ENOMEM when wt_footprint's work_bytes
 * for *desc exceed WT_NOALLOC_WORK_BYTES (for example u8 inputs above about
 * 2^25 symbols), WT_EINVAL as for wt_build, WT_EDEVICE if the array's
 * address cannot be read on the current device (done once per device, on
 * the first call there).  The array is shared by every call on a device and
 * keeps the last build's contents: builds that overlap on one device (other
 * streams, other threads) race and must be serialised by the caller.
 * Profiling (wt_prof_enable) must be off.
 */
#define WT_NOALLOC_WORK_BYTES (64ull << 20)
int wt_build_noalloc(const void *d_S, const wt_desc *desc, void *d_tree, uint64_t tree_bytes, void *stream);

/*
 * Build m independent trees in one batched launch sequence on `stream`: the
 * construction of wt_build (Sections 3.1 and 3.2) for many sequences at
 * once, the segments of all of them sharing each launch the way Algorithm
 * dd's segments share the cores.
 * d_S[q], descs[q], d_trees[q] (of tree_bytes[q] bytes) describe sequence q;
 * sequences may mix lengths, alphabets and widths.  Long sequences, which
 * fill the device by themselves, are built in the same call as wt_build
 * would build them, on the same stream: those of at least 2^25 4-byte
 * symbols, and those of at least 2^25 1-byte or 2^23 2- or 4-byte symbols
 * that no other sequence of the batch would share batched launches with.
 * Every tree is the one wt_build produces.  out[q]
 * receives the handle of tree q (each released with wt_free).  On error no
 * handle is returned; argument errors (WT_EINVAL, and WT_ENOMEM for short
 * tree or work memory) are found before anything is enqueued.
 */
int wt_build_batch(uint32_t m, const void *const *d_S, const wt_desc *descs,
                   void *const *d_trees, const uint64_t *tree_bytes, void *d_work,
                   uint64_t work_bytes, void *stream, wt_tree **out);

/*
 * Waits for the stream of the build, then returns WT_OK, WT_ERANGE (some
 * symbol >= sigma) or WT_EDEVICE.
 */
int wt_tree_status(const wt_tree *tree);

/* Release the host handle (the caller's tree memory is untouched). */
void wt_free(wt_tree *tree);

/*
 * Write counting, for verification (callers: tests and debugging only).
 * The library promises that every word of a level bitmap (or 4-ary digit
 * level) is stored by exactly one writer, with no atomics on the bitmaps.
 * In the write-counting build of the library (libwtree_check.so, compiled
 * with WT_WRITE_CHECK), every later store of bitmap or digit words that
 * falls in [d_base, d_base + bytes) adds one to the 32-bit counter of each
 * 16-bit granule it covers: d_counts holds bytes / 2 counters, in device
 * memory the caller owns and clears.  A build kept the promise when every
 * granule of its bitmaps counts exactly 1, padding words included.  d_counts
 * null stops the counting.  Call it with no build in flight (it writes a
 * device variable synchronously).  Returns WT_OK, WT_EINVAL (d_base or
 * bytes odd, or the product build, which counts nothing) or WT_EDEVICE.
 */
int wt_debug_write_counters(void *d_counts, const void *d_base, uint64_t bytes);

/*
 * The one-pointer-per-level representation of Section 2.2 (one n-bit bitmap
 * per level, addressed from a single pointer).  Layout of a built tree:
 * number of levels, device pointer to level 0's
 * bitmap (level i starts words_per_level * i words later) and to level 0's
 * rank directory (level i starts rank_stride * i entries later), and the
 * number of meaningful rank entries per level (K = ceil(n/512) + 1).
 */
int wt_levels(const wt_tree *tree, uint32_t *levels, const uint64_t **d_bitmaps,
              uint64_t *words_per_level, const uint64_t **d_ranks, uint64_t *rank_stride,
              uint64_t *rank_entries);

/*
 * Batched queries (Section 2.2 access / rank / select, evaluated by walking
 * the levels with rank and select on the bitmaps).  m queries, device
 * arrays, enqueued on `stream` after whatever the stream already holds.
 *  - access: d_sym[k] = S[d_i[k]];            d_i[k] >= n gives 0xFFFFFFFF
 *  - rank:   d_r[k] = occurrences of d_c[k] in S[0, d_i[k]);  d_i[k] > n or
 *            d_c[k] >= sigma gives UINT64_MAX
 *  - select: d_pos[k] = 0-based position of the d_j[k]-th (1-based)
 *            occurrence of d_c[k]; UINT64_MAX if there is none
 */
int wt_access_batch(const wt_tree *tree, const uint64_t *d_i, uint32_t *d_sym, uint64_t m,
                    void *stream);
int wt_rank_batch(const wt_tree *tree, const uint32_t *d_c, const uint64_t *d_i,
                  uint64_t *d_r, uint64_t m, void *stream);
int wt_select_batch(const wt_tree *tree, const uint32_t *d_c, const uint64_t *d_j,
                    uint64_t *d_pos, uint64_t m, void *stream);

/*
 * Mixed queries over many trees in one launch (for serving).  Query k asks
 * tree trees[d_tree[k]] (d_tree[k] < ntrees): d_kind[k] = 0 access(d_x[k]),
 * 1 rank(d_c[k], d_x[k]), 2 select(d_c[k], d_x[k]); d_out[k] receives the
 * symbol, the count or the position, with UINT64_MAX wherever the per-tree
 * calls above return their out-of-range value (and for an unknown kind or
 * tree index).  d_work is device memory of wt_query_multi_footprint(ntrees)
 * bytes (16-byte aligned) into which the trees' layouts are copied on
 * `stream`; it must stay untouched until the stream has passed the queries.
 * The trees must be complete by the time the stream reaches the queries
 * (same stream as their builds, or synchronised).
 */
int wt_query_multi_footprint(uint32_t ntrees, uint64_t *work_bytes);
int wt_query_multi(uint32_t ntrees, const wt_tree *const *trees, const uint32_t *d_tree,
                   const uint8_t *d_kind, const uint32_t *d_c, const uint64_t *d_x, uint64_t *d_out,
                   uint64_t m, void *d_work, uint64_t work_bytes, void *stream);

/*
 * Single queries for verification: they run the batched kernels on the
 * build's stream and wait for the answer.  WT_EINVAL for i out of range or
 * c >= sigma, WT_ENOTFOUND for a select with no such occurrence.
 */
int wt_access(const wt_tree *tree, uint64_t i, uint32_t *sym);
int wt_rank(const wt_tree *tree, uint32_t c, uint64_t i, uint64_t *r);
int wt_select(const wt_tree *tree, uint32_t c, uint64_t j, uint64_t *pos);

/* Static text for a status code. */
const char *wt_strerror(int status);

/*
 * Tile geometry of the level pass (the segment size of the domain
 * decomposition, Section 3.2, here the unit of work of one wavefront: 64
 * lanes x lane_bytes bytes of symbols).  lane_bytes is 32, 64 or 128 with
 * lane_bytes / width <= 64; 0 restores the default (64).  The setting is kept
 * per (mode, width, levels, floor(lg n)) for the whole process -- mode 0 for
 * wt_footprint / wt_build, mode 1 for a sequence of wt_batch_footprint /
 * wt_build_batch; 1 <= levels <= min(24, 8 * width), lg_n <= 40 -- and read
 * whenever a layout is computed.  The tree does not depend on it (every
 * geometry builds the same bits); the workspace size does, so change it only
 * between builds and take footprints after the change.  Not thread-safe
 * against concurrent builds.  WT_EINVAL for an invalid key or value.
 */
int wt_tune_set(uint32_t mode, uint32_t width, uint32_t levels, uint32_t lg_n, uint32_t lane_bytes);
int wt_tune_get(uint32_t mode, uint32_t width, uint32_t levels, uint32_t lg_n, uint32_t *lane_bytes);

#ifdef __cplusplus
}
#endif

#endif /* WTREE_H */
