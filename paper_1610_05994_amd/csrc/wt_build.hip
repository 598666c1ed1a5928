// Wavelet-tree construction kernels for gfx950 (CDNA4, wave64).
//
// The build follows the per-level construction of Section 3.1 (Algorithm
// pwt: count the symbols of every node, prefix-sum the counts into node
// offsets, then place every symbol's level bit at its node's running offset
// in input order) and the segment idea of Section 3.2 (Algorithm dd: local
// counts per segment, a prefix sum over segments turning local offsets into
// global ones).  It is organised for the GPU as a level split:
//
//   T_0 = S;  T_{i+1} = T_i stably partitioned, inside every level-i node,
//   by the level-i bit (zeros first).
//
// T_i is S stably sorted by its top i bits (Proposition 1: the node of s at
// level i is s >> (l-i)), so level i's bitmap is simply bit (l-1-i) of T_i,
// position by position: a 64-position word is built by one wave from 64
// consecutive symbols and has exactly one writer (no atomics on bitmaps).
// (The last level of a u8 tree can instead come out of the pass before it,
// as 16-position granules with one writer each: see LevelArgs::bits_next.)
//
// Segments are tiles of kTile consecutive positions of T_i.  The ones count
// of every tile of level i is known before level i runs: level 0's come from
// the ingest pass, and the pass of level i-1, which knows where every symbol
// lands in T_i, adds up the level-i bits per destination tile.  A small scan
// turns them into the rank of each tile's first position, so a level pass
// needs no inter-tile communication at all.  One level pass, in one read of
// T_i, writes:
//   * the bitmap words of the tile,
//   * the rank directory entries at the multiples of 512 inside the tile,
//   * the stable split into T_{i+1}: with O1(v) the ones before node v and
//     rank1(p) the ones before position p,
//       bit 0 at p  ->  p - rank1(p) + O1(v)
//       bit 1 at p  ->  start_{i+1}(2v+1) - O1(v) + rank1(p)
//     staged in LDS so that the global stores are aligned 16-byte chunks,
//   * the ones of level i+1 per destination tile and per level-(i+1) node
//     (the node sizes of the next level: Algorithm pwt's counting step,
//     done for level i+1 while level i is split).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wt_check.h"
#include "wt_internal.h"

namespace wt {

namespace {

#include "wt_wave.h"

// ------------------------------------------------------------- zero fill --

// Zeroes `words` 8-byte words at p (8-byte aligned): a leading word when p
// is not 16-byte aligned, then two words per store, then a trailing word.
__device__ __forceinline__ void zero_words(uint64_t *p, uint64_t words) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    if (words && ((uintptr_t)p & 15u)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) p[0] = 0;
        p++;
        words--;
    }
    const uint64_t pairs = words / 2;
    ulonglong2 *q = reinterpret_cast<ulonglong2 *>(p);
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < pairs; k += stride)
        q[k] = make_ulonglong2(0ull, 0ull);
    if ((words & 1) && blockIdx.x == 0 && threadIdx.x == 0) p[words - 1] = 0;
}

__global__ void k_zero(uint64_t *p, uint64_t words, uint32_t *tree_status, uint64_t *p2, uint64_t count2) {
    zero_words(p, words);
    if (p2) zero_words(p2, count2);
    if (blockIdx.x == 0 && threadIdx.x == 0) *tree_status = 0;
}

// ---------------------------------------------------------------- ingest --
// Reads S once: flags symbols >= sigma, and counts the ones of level 0 (the
// most significant of the l bits) per tile and in total.  Every later
// node count is produced by the level pass before it.

// u8 level bits in "spread" order, without multiplies: dword q of a lane
// holds symbols 4q..4q+3 in its bytes m = 0..3; bit sh of byte m lands on
// bit 8m + (q mod 8) of the 32-bit half q / 8 (a rotation by sh - q mod 8
// brings every byte's level bit to that column at once, one mask keeps
// them).  Two full-rate operations per dword.
template <int B>
__device__ __forceinline__ typename MaskT<B>::T level_bits_spread(const uint4 (&raw)[B / 16], uint32_t sh) {
    typedef typename MaskT<B>::T M;
    constexpr int D = B / 4;
    uint32_t h[(D + 7) / 8];
#pragma unroll
    for (int i = 0; i < (D + 7) / 8; i++) h[i] = 0;
#pragma unroll
    for (int q = 0; q < D; q++) {
        const uint4 &c = raw[q / 4];
        const uint32_t d = (q % 4 == 0) ? c.x : (q % 4 == 1) ? c.y : (q % 4 == 2) ? c.z : c.w;
        const uint32_t r = (uint32_t)(q % 8);
        h[q / 8] |= __builtin_amdgcn_alignbit(d, d, (sh - r) & 31u) & (0x01010101u << r);
    }
    M m = h[0];
#pragma unroll
    for (int i = 1; i < (D + 7) / 8; i++) m |= (M)h[i] << (32 * i);
    return m;
}

// A lane's level bits for the split: the spread order for u8, else the
// symbol order.
template <int W, int B>
__device__ __forceinline__ typename MaskT<B / W>::T level_bits_split(const uint4 (&raw)[B / 16], uint32_t sh) {
    if constexpr (W == 1) return level_bits_spread<B>(raw, sh);
    else return level_bits<W, B>(raw, sh);
}

// Bit of symbol k of a lane in the split's order.
template <int W>
__host__ __device__ constexpr int level_bit_pos(int k) {
    return (W == 1) ? 32 * (k / 32) + 8 * (k % 4) + (k % 32) / 4 : k;
}

// Spread order -> symbol order in each 32-bit half: bit 8m + r moves to
// 4r + m (a 4 x 8 bit-matrix transpose), as four exchanges of index bits
// (4 <-> 2, 3 <-> 1, 2 <-> 0, 1 <-> 0), each one delta swap.
__device__ __forceinline__ uint32_t spread_half_order(uint32_t x) {
    uint32_t t;
    t = ((x >> 12) ^ x) & 0x0000F0F0u;
    x ^= t ^ (t << 12);
    t = ((x >> 6) ^ x) & 0x00CC00CCu;
    x ^= t ^ (t << 6);
    t = ((x >> 3) ^ x) & 0x0A0A0A0Au;
    x ^= t ^ (t << 3);
    t = ((x >> 1) ^ x) & 0x22222222u;
    x ^= t ^ (t << 1);
    return x;
}

template <typename M>
__device__ __forceinline__ M spread_order(M m) {
    if (sizeof(M) == 8)
        return (M)spread_half_order((uint32_t)m) | ((M)spread_half_order((uint32_t)((uint64_t)m >> 32)) << 32);
    return (M)spread_half_order((uint32_t)m);
}

// Bit sh of the 16 u8 symbols of a 16-byte chunk, symbol k at bit k.  The
// spread gather puts symbol 4j + b at bit 8b + j; folding each byte pair
// into one byte and keeping bytes 0 and 2 leaves it at bit 4b + j, and two
// delta swaps (index bits 3 <-> 1, 2 <-> 0) transpose that 4 x 4 matrix.
__device__ __forceinline__ uint32_t chunk_bits16(const uint4 &v, uint32_t sh) {
    uint32_t h = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint32_t d = (j == 0) ? v.x : (j == 1) ? v.y : (j == 2) ? v.z : v.w;
        h |= __builtin_amdgcn_alignbit(d, d, (sh - (uint32_t)j) & 31u) & (0x01010101u << j);
    }
    const uint32_t f = h | (h >> 4);
    uint32_t x = (f & 0xFFu) | ((f >> 8) & 0xFF00u);
    uint32_t t = ((x >> 6) ^ x) & 0x00CCu;
    x ^= t ^ (t << 6);
    t = ((x >> 3) ^ x) & 0x0A0Au;
    x ^= t ^ (t << 3);
    return x;
}

// Stable split of one lane's symbols into LDS: zeros to zc, zc+1, ...,
// ones to oc, oc+1, ...  kFull: all E symbols are valid (no guards).  The
// level bits come in the order of level_bit_pos.  The staged symbols are
// WO-byte (their low bytes: WO < W narrows them).
template <int W, int B, int WO, bool kFull>
__device__ __forceinline__ void stage_split(typename ElemT<WO>::T *s_stage, const uint4 (&raw)[B / 16],
                                            typename MaskT<B / W>::T mb, uint32_t zc, uint32_t oc, int nval) {
    typedef typename ElemT<WO>::T T;
    constexpr int E = B / W;
    // With zp the next zero slot and D = (next one slot - zp) + k, symbol k
    // goes to zp + b * (D - k); zp advances on a zero, D by 2 on a one (one
    // 24-bit multiply-add per symbol; slots < 2^24).  The empty asm keeps D
    // an opaque register, so the compiler keeps this two-operation update
    // instead of rebuilding D from a ones count.
    T *zp = s_stage + zc;
    uint32_t D = oc - zc;
#pragma unroll
    for (int k = 0; k < E; k++) {
        if (kFull || k < nval) {
            const uint32_t b = (uint32_t)(mb >> level_bit_pos<W>(k)) & 1u;
            const int q = (k * W) >> 2;
            const uint4 &c = raw[q / 4];
            const uint32_t d = (q % 4 == 0) ? c.x : (q % 4 == 1) ? c.y : (q % 4 == 2) ? c.z : c.w;
            // the store keeps the low WO bytes of x (or, for the third byte of
            // a dword, the d16_hi form picks it), so no masking is needed
            uint32_t x;
            if (W == 4) x = d;
            else if (W == 2) x = (k & 1) ? (d >> 16) : d;
            else x = ((k & 3) == 1 || (k & 3) == 3) ? (d >> 8) : d;
            if (W == 1 && (k & 3) >= 2) x >>= 16;
            zp[__umul24(b, D - (uint32_t)k)] = (T)x;
            zp += b ^ 1u;
            D += 2u * b;
            asm volatile("" : "+v"(D));
        }
    }
}

// Number of symbols of a 16-byte chunk whose bit sh2 is set.
template <int W>
__device__ __forceinline__ uint32_t chunk_bit_count(const uint4 &v, uint32_t sh2) {
    const uint32_t lowbits = (W == 1) ? 0x01010101u : (W == 2) ? 0x00010001u : 1u;
    return __popc((v.x >> sh2) & lowbits) + __popc((v.y >> sh2) & lowbits) + __popc((v.z >> sh2) & lowbits) +
           __popc((v.w >> sh2) & lowbits);
}

// One tile of the ingest pass, run by one wave, from its loaded symbols:
// returns the tile's level-0 ones (when they are counted) and sets bad if a
// symbol is >= sigma.
template <int W, int B>
__device__ __forceinline__ uint32_t ingest_tile(const IngestArgs &a, uint64_t t, const uint4 (&raw)[B / 16], int nval,
                                                bool &bad) {
    constexpr int E = B / W;
    const int lane = threadIdx.x & 63;
    if (a.check) {
#pragma unroll
        for (int k = 0; k < E; k++) bad |= (k < nval) && (raw_elem<W, B>(raw, k) >= a.sigma);
    }
    uint32_t ones = 0;
    if (a.tile_ones0) {
        // symbols past n load as 0, so they add no ones
        const typename MaskT<E>::T mb = level_bits_split<W, B>(raw, a.msb);  // (any order for a count)
        ones = wave_sum32((E == 64) ? (uint32_t)__popcll((uint64_t)mb) : (uint32_t)__popc((uint32_t)mb));
        if (lane == 0) a.tile_ones0[t] = ones;
    }
    return ones;
}

// Ends an ingest wave: reports bad symbols, adds the root's ones.
__device__ __forceinline__ void ingest_finish(const IngestArgs &a, bool bad, unsigned long long ones_acc,
                                              uint64_t slot) {
    const int lane = threadIdx.x & 63;
    if (__any(bad) && lane == 0) atomicOr(a.tree_status, 1u);
    if (a.tile_ones0 && lane == 0 && ones_acc) atomicAdd(&a.ones0[slot % a.slots0], ones_acc);
}

template <int W, int B>
__global__ __launch_bounds__(kThreads) void k_ingest(IngestArgs a) {
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.start0) {
        a.start0[0] = 0;
        a.start0[1] = a.n;
    }
    // this workgroup's tiles: [t0, t1); wave wv takes every kWaves-th one
    const uint64_t t0 = (uint64_t)blockIdx.x * a.tiles_per_block;
    const uint64_t t1 = (t0 + a.tiles_per_block < a.ntiles) ? t0 + a.tiles_per_block : a.ntiles;
    // two tiles per step, both loaded before either is counted, so that a
    // wave keeps two tiles' loads in flight
    constexpr int E = B / W;
    constexpr uint64_t TILE = tile_syms(W, B);
    const uint64_t lofs = (uint64_t)(threadIdx.x & 63) * E;
    bool bad = false;
    unsigned long long ones_acc = 0;
    for (uint64_t t = t0 + wv; t < t1; t += 2 * kWaves) {
        const uint64_t u = t + kWaves;
        uint4 ra[B / 16], rb[B / 16];
        const int na = load_lane<W, B>(a.S, t * TILE + lofs, a.n, ra);
        const int nb = (u < t1) ? load_lane<W, B>(a.S, u * TILE + lofs, a.n, rb) : 0;
        ones_acc += ingest_tile<W, B>(a, t, ra, na, bad);
        if (u < t1) ones_acc += ingest_tile<W, B>(a, u, rb, nb, bad);
    }
    ingest_finish(a, bad, ones_acc, (uint64_t)blockIdx.x * kWaves + wv);
    // (a pass that only reads has write bandwidth to spare)
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.zero_granules;
         k += (uint64_t)gridDim.x * blockDim.x) {
        a.zero_g[k] = 0;
        note_write(&a.zero_g[k], 2);
    }
}

// ----------------------------------------------------------- node tables --
// For level i with node starts start_i and ones counts ones_i (the sum of
// the counter slots):
//   O1 = exclusive scan of ones_i (ones before each node),
//   zo_i(v) = (O1(v), start_i(v+1) - ones_i(v) - O1(v)),
//   start_{i+1}(2v) = start_i(v), start_{i+1}(2v+1) = start_i(v+1) - ones_i(v).
// Small levels are done by one workgroup of k_prep; levels above kScanChunk
// nodes (one counter slot) by k_plan_reduce / _partials / _apply.

// Node tables for entries [b0, b0 + kScanChunk) given the ones before b0;
// ov[v - b0] holds the ones of node v.  Returns the ones of the chunk.
// The thread's start entries of a chunk (entries k0 .. k0 + 16 and the one
// before), loaded together; the table stores may alias them, which would
// otherwise serialise one load per node.
struct ChunkStarts {
    uint64_t first;
    uint64_t next[kScanChunk / kThreads];
};

__device__ __forceinline__ void load_chunk_starts(const PlanArgs &a, uint64_t b0, ChunkStarts &cs) {
    const uint64_t per = kScanChunk / kThreads;
    const uint64_t k0 = b0 + threadIdx.x * per;
    cs.first = (k0 < a.nodes) ? a.start[k0] : 0ull;
#pragma unroll
    for (uint64_t q = 0; q < per; q++) cs.next[q] = (k0 + q < a.nodes) ? a.start[k0 + q + 1] : 0ull;
}

// Node tables for entries [b0, b0 + kScanChunk) given the ones before b0 and
// the thread's start entries; ov[v - b0] holds the ones of node v.  Returns
// the ones of the chunk.
__device__ __forceinline__ unsigned long long plan_chunk_with(const PlanArgs &a, const unsigned long long *ov,
                                                              uint64_t b0, unsigned long long before,
                                                              const ChunkStarts &cs) {
    __shared__ unsigned long long s_w[kWaves];
    const uint64_t per = kScanChunk / kThreads;  // 16 consecutive entries per thread
    const uint64_t k0 = b0 + threadIdx.x * per;
    unsigned long long loc[kScanChunk / kThreads];
    unsigned long long tsum = 0;
#pragma unroll
    for (uint64_t q = 0; q < per; q++) {
        loc[q] = (k0 + q < a.nodes) ? ov[k0 + q - b0] : 0ull;
        tsum += loc[q];
    }
    unsigned long long tot;
    unsigned long long o1 = block_excl_scan64(tsum, s_w, &tot) + before;
#pragma unroll
    for (uint64_t q = 0; q < per; q++) {
        const uint64_t v = k0 + q;
        if (v < a.nodes) {
            const unsigned long long ones = loc[q];
            const uint64_t s_next = cs.next[q];
            a.zo[v] = make_ulonglong2(o1 - a.shift, s_next - ones - o1 - a.shift);
            if (a.start_next && !a.matrix) {
                a.start_next[2 * v] = ((q == 0) ? cs.first : cs.next[q - 1]) - a.shift;
                a.start_next[2 * v + 1] = s_next - ones - a.shift;
            }
            o1 += ones;
        }
    }
    if (a.start_next && b0 == 0 && threadIdx.x == 0) {
        if (a.matrix) a.start_next[0] = 0;
        a.start_next[a.matrix ? 1 : 2 * a.nodes] = a.n - a.shift;
    }
    return tot;
}

__device__ __forceinline__ unsigned long long plan_chunk(const PlanArgs &a, const unsigned long long *ov, uint64_t b0,
                                                         unsigned long long before) {
    ChunkStarts cs;
    load_chunk_starts(a, b0, cs);
    return plan_chunk_with(a, ov, b0, before, cs);
}

// Chunk b of a level's nodes: partials[b] = its ones.
__device__ __forceinline__ void plan_reduce_chunk(const PlanArgs &a, uint64_t b) {
    __shared__ unsigned long long s_w[kWaves];
    const uint64_t b0 = b * kScanChunk;
    unsigned long long sum = 0;
    for (uint64_t k = b0 + threadIdx.x; k < b0 + kScanChunk && k < a.nodes; k += kThreads) sum += a.ones[k];
    sum = wave_sum64(sum);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kWaves; w++) t += s_w[w];
        a.partials[b] = t;
    }
}

// Exclusive scan of the nblocks (<= kMaxScanBlocks) partials, in place.
__device__ __forceinline__ void plan_scan_partials(const PlanArgs &a, uint64_t nblocks) {
    __shared__ unsigned long long s_w[kWaves];
    const uint64_t per = ceil_div(nblocks, kThreads);  // a few consecutive entries per thread
    const uint64_t k0 = threadIdx.x * per;
    unsigned long long sum = 0;
    for (uint64_t q = 0; q < per; q++)
        if (k0 + q < nblocks) sum += a.partials[k0 + q];
    unsigned long long tot;
    unsigned long long off = block_excl_scan64(sum, s_w, &tot);
    for (uint64_t q = 0; q < per; q++) {
        if (k0 + q < nblocks) {
            const unsigned long long v = a.partials[k0 + q];
            a.partials[k0 + q] = off;
            off += v;
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_plan_reduce(PlanArgs a) { plan_reduce_chunk(a, blockIdx.x); }

__global__ __launch_bounds__(kThreads) void k_plan_partials(PlanArgs a, uint64_t nblocks) {
    plan_scan_partials(a, nblocks);
}

__global__ __launch_bounds__(kThreads) void k_plan_apply(PlanArgs a) {
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanChunk;
    plan_chunk(a, a.ones + b0, b0, a.partials[blockIdx.x]);
}

// ------------------------------------------------------ per-level prep ---
// k_supsum: workgroup c adds up the kSup tile counts of superchunk c.
// k_prep (one workgroup): sup[c] = ones in all tiles before superchunk c,
// and, for levels of at most kScanChunk nodes, the level's node tables.

// Workgroup: supsum[c] = ones of the kSup tiles of superchunk c.
__device__ __forceinline__ void supsum_one(const uint32_t *tile_ones, uint64_t ntiles, uint64_t c,
                                           unsigned long long *supsum) {
    __shared__ uint32_t s_w[kWaves];
    const uint32_t tid = threadIdx.x;
    const uint64_t t = c * kSup + tid;
    const uint32_t v = wave_sum32(t < ntiles ? tile_ones[t] : 0u);
    if ((tid & 63) == 0) s_w[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        unsigned long long tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; w++) tot += s_w[w];
        supsum[c] = tot;
    }
}

__global__ __launch_bounds__(kThreads) void k_supsum(PrepArgs a) { supsum_one(a.tile_ones, a.ntiles, blockIdx.x, a.supsum); }

// Sum of the counter slots q = g, g + step, ... of node v (loads batched).
__device__ __forceinline__ unsigned long long slot_sum(const unsigned long long *ones, uint64_t nodes,
                                                       uint64_t slots, uint64_t v, uint64_t g, uint64_t step) {
    unsigned long long c = 0;
    uint64_t q = g;
    for (; q + 15 * step < slots; q += 16 * step) {
        unsigned long long x[16];
#pragma unroll
        for (int r = 0; r < 16; r++) x[r] = ones[(q + r * step) * nodes + v];
#pragma unroll
        for (int r = 0; r < 16; r++) c += x[r];
    }
    for (; q < slots; q += step) c += ones[q * nodes + v];
    return c;
}

// Workgroup: superchunk prefixes, then (when plan_here) the node tables of
// the level, kScanChunk nodes at a time.
__device__ __forceinline__ void prep_level(const PrepArgs &a) {
    __shared__ unsigned long long s_w[kWaves];
    __shared__ unsigned long long s_n[kScanChunk];
    const uint32_t tid = threadIdx.x;
    if (a.nsup <= kThreads && a.plan_here && a.plan.nodes < kThreads) {
        // A small level (every level of sequences up to 2^28 u8 symbols):
        // the superchunk sums, the node counter slots and the start entries
        // are all loaded up front, so the step waits for memory once.  With
        // sums_here the superchunk sums come from the tile counts directly
        // (thread t holds tile t of every superchunk), and no k_supsum ran.
        const PlanArgs &p = a.plan;
        const uint64_t cn = p.nodes, groups = kThreads / cn, v = tid % cn, g = tid / cn;
        uint32_t tc[kPrepSups];
#pragma unroll
        for (uint64_t q = 0; q < kPrepSups; q++) {
            const uint64_t t = q * kSup + tid;
            tc[q] = (a.sums_here && q < a.nsup && t < a.ntiles) ? a.tile_ones[t] : 0u;
        }
        unsigned long long sv = (!a.sums_here && tid < a.nsup) ? a.supsum[tid] : 0ull;
        unsigned long long x[16];  // slots * nodes <= kSlotSpan: 16 slots per thread
#pragma unroll
        for (uint64_t q = 0; q < 16; q++) {
            const uint64_t sl = g + q * groups;
            x[q] = (sl < p.slots) ? p.ones[sl * p.nodes + v] : 0ull;
        }
        ChunkStarts cs;
        load_chunk_starts(p, 0, cs);
        if (a.sums_here) {
            // superchunk q's sum: its 256 tile counts over the workgroup
            __shared__ uint32_t s_q[kWaves][kPrepSups];
#pragma unroll
            for (uint64_t q = 0; q < kPrepSups; q++) {
                const uint32_t w = wave_sum32(tc[q]);  // (each count < 2^16: a superchunk sum fits 32 bits)
                if ((tid & 63) == 0) s_q[tid >> 6][q] = w;
            }
            __syncthreads();
            if (tid < kPrepSups) {
                unsigned long long t = 0;
#pragma unroll
                for (int w = 0; w < kWaves; w++) t += s_q[w][tid];
                sv = (tid < a.nsup) ? t : 0ull;
            }
        }
        unsigned long long tot;
        const unsigned long long ex = block_excl_scan64(sv, s_w, &tot);
        if (tid < a.nsup) a.sup[tid] = ex;
        if (tid < cn) s_n[tid] = 0;
        __syncthreads();
        unsigned long long c = 0;
#pragma unroll
        for (uint64_t q = 0; q < 16; q++) c += x[q];
        for (uint64_t sl = g + 16 * groups; sl < p.slots; sl += groups) c += p.ones[sl * p.nodes + v];
        if (c) atomicAdd(&s_n[v], c);
        __syncthreads();
        plan_chunk_with(p, s_n, 0, 0, cs);
        return;
    }
    unsigned long long carry = 0;
    for (uint64_t c0 = 0; c0 < a.nsup; c0 += kThreads) {
        const uint64_t c = c0 + tid;
        const unsigned long long v = (c < a.nsup) ? a.supsum[c] : 0ull;
        unsigned long long tot;
        const unsigned long long ex = block_excl_scan64(v, s_w, &tot);
        if (c < a.nsup) a.sup[c] = carry + ex;
        carry += tot;
    }
    if (!a.plan_here) return;
    const PlanArgs &p = a.plan;
    unsigned long long before = 0;
    for (uint64_t b0 = 0; b0 < p.nodes; b0 += kScanChunk) {
        // add up the node counter slots of this chunk, then scan it
        const uint64_t cn = (p.nodes - b0 < kScanChunk) ? p.nodes - b0 : kScanChunk;
        for (uint64_t v = tid; v < cn; v += kThreads) s_n[v] = 0;
        __syncthreads();
        if (cn >= kThreads) {
            for (uint64_t v = tid; v < cn; v += kThreads) s_n[v] = slot_sum(p.ones, p.nodes, p.slots, b0 + v, 0, 1);
        } else {
            // kThreads / nodes threads per node, then one LDS add per thread
            const uint64_t groups = kThreads / cn;
            const uint64_t v = tid % cn, g = tid / cn;
            const unsigned long long c = slot_sum(p.ones, p.nodes, p.slots, b0 + v, g, groups);
            if (c) atomicAdd(&s_n[v], c);
        }
        __syncthreads();
        before += plan_chunk(p, s_n, b0, before);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void k_prep(PrepArgs a) { prep_level(a); }

// ----------------------------------------------------------- level pass ---

// Tiles spanning fewer than kRunNodes nodes (several nodes, e.g. at deep
// levels) are staged in LDS as runs, one per (node, bit), each placed at
// the 16-byte phase of its destination so that it leaves in aligned chunks.
constexpr uint32_t kRunNodes = 16;

struct MultiTables {
    uint32_t key[kRunNodes + 1];     // node's first tile position << 16 | tile ones before it
    uint32_t st[2 * kRunNodes];      // run r = 2j + b: first staging slot
    uint32_t len[2 * kRunNodes];     // symbols in the run
    uint32_t blk[2 * kRunNodes + 1]; // first 16-byte staging block of the run; [2 span] = blocks in all
    uint32_t cnt[4 * kRunNodes];     // next-level ones per (run, destination-tile parity)
    uint32_t tix[4 * kRunNodes];     // that destination tile
    unsigned long long g[2 * kRunNodes];  // destination of the run's first symbol
};
constexpr uint32_t kMultiTablesBytes = (uint32_t)((sizeof(MultiTables) + 15) / 16 * 16);

template <int W, int B, int WO = W>
__host__ __device__ constexpr uint32_t multi_stage_elems() {
    // every run wastes fewer than CH slots at each end (CH: WO-byte symbols
    // per chunk; WO <= W stages in no more bytes than W)
    return (uint32_t)tile_syms(W, B) + 2 * kRunNodes * 2 * (16 / WO);
}

// LDS bytes of one wave of a level pass: staging of the split (zeros at
// [a0, a0+Z), ones at [a1, a1+O) with a1 + O <= TILE + 3*CH - 3), or, for
// tiles spanning many nodes, next-level counters per (node, bit,
// destination-tile parity); with M, also the run tables and staging of a
// tile spanning a few nodes.  (M is only used for deep levels: the larger
// LDS slice lowers occupancy.)
// LDS of a wave: without M, the single-node staging or the direct path's
// counters; with M (no direct path), the single-node staging, or the run
// tables and staging of the few-nodes split, or the dense split's staging
// (one tile, or two with the symbol copy), whichever is largest.
// The dense split of a single build keeps an LDS copy of the tile beside its
// staging only where that fits in the slice the other paths need anyway;
// elsewhere it reads the symbols back from T_i (just loaded, so from the
// cache) and the slice, and with it the variant's occupancy, is set by the
// other paths.  (The batched passes always keep the copy: their staged
// launches are short, and the reads' latency showed more than occupancy.)
template <int W, int B>
__host__ __device__ constexpr bool dense_lds_copy() {
    constexpr uint32_t split = (uint32_t)(tile_syms(W, B) + 4 * (16 / W)) * W;
    constexpr uint32_t multi = kMultiTablesBytes + multi_stage_elems<W, B>() * W;
    return 2u * (uint32_t)tile_syms(W, B) * W <= (split > multi ? split : multi);
}

template <int W, int B, bool M, bool kCopy>
__host__ __device__ constexpr uint32_t level_wave_bytes() {
    constexpr uint32_t split = (uint32_t)(tile_syms(W, B) + 4 * (16 / W)) * W;
    constexpr uint32_t counters = 2u * 4u * kNodeCap * 4u;
    constexpr uint32_t multi = kMultiTablesBytes + multi_stage_elems<W, B>() * W;
    constexpr uint32_t dense = (kCopy ? 2u : 1u) * (uint32_t)tile_syms(W, B) * W;
    constexpr uint32_t plain = split > counters ? split : counters;
    constexpr uint32_t m1 = split > multi ? split : multi;
    constexpr uint32_t m2 = m1 > dense ? m1 : dense;
    return M ? (m2 > counters ? m2 : counters) : plain;  // (M: the direct path takes tiles over two anchors)
}

// Split of a tile whose symbols span nodes vf..vl (fewer than kRunNodes):
// the symbols of node vf + j with bit b form run r = 2j + b, contiguous in
// T_{i+1}.  With pf / r1f the tile position and tile ones before the node's
// first symbol, a symbol at tile position p with r tile ones before it sits
// at offset (p - pf) - (r - r1f) of its zero run or r - r1f of its one run;
// the runs start at base + pf - R + O1(v) and start_{i+1}(2v+1) - O1(v) + R
// (R = prefix + r1f, the rank of the node's first symbol), as in the
// single-node case.  Runs are staged in LDS at their destination's 16-byte
// phase and written out in aligned chunks; next-level ones are counted per
// chunk.
template <int W, int B, int WO, bool kOptNodes>
__device__ __forceinline__ void stage_multi(const LevelArgs &a, const uint4 (&raw)[B / 16],
                                            typename MaskT<B / W>::T mb, int nval, uint32_t lr1, uint32_t agg,
                                            unsigned long long prefix, uint64_t base, uint64_t nvalid, uint32_t vf,
                                            uint32_t vl, uint32_t nsh, uint32_t nbase, uint8_t *s_wave,
                                            typename ElemT<WO>::T *tout, bool counting, uint32_t sh2,
                                            unsigned long long *ones_next) {
    typedef typename ElemT<WO>::T T;  // staged and written symbols
    constexpr int E = B / W;
    constexpr uint32_t CH = 16 / WO;
    constexpr uint64_t TILE = tile_syms(W, B);
    constexpr uint32_t kStage = multi_stage_elems<W, B, WO>();
    const int lane = threadIdx.x & 63;
    MultiTables *tb = reinterpret_cast<MultiTables *>(s_wave);
    T *s_stage = reinterpret_cast<T *>(s_wave + kMultiTablesBytes);
    const uint32_t span = vl - vf + 1;  // nodes of the tile, some possibly empty
    const uint32_t nruns = 2 * span;

    for (uint32_t q = lane; q <= span; q += 64)
        tb->key[q] = (q == span) ? (((uint32_t)nvalid << 16) | agg) : 0xFFFFFFFFu;
    for (uint32_t q = lane; q < 4 * span; q += 64) tb->cnt[q] = 0;
    wave_sync();
    // first symbol of every node present in the tile
    {
        uint32_t vprev = wave_prev_lane(nbase + ((raw_elem<W, B>(raw, E - 1) & a.symmask) >> nsh), 0xFFFFFFFFu);
        uint32_t r = lr1;
#pragma unroll
        for (int k = 0; k < E; k++) {
            if (k < nval) {
                const uint32_t v = nbase + ((raw_elem<W, B>(raw, k) & a.symmask) >> nsh);
                if (v != vprev && v - vf < span) tb->key[v - vf] = (((uint32_t)lane * E + k) << 16) | r;
                vprev = v;
                r += (uint32_t)(mb >> k) & 1u;
            }
        }
    }
    wave_sync();
    // runs of node j = lane: an empty node takes the next node's key (length 0)
    {
        uint32_t key = ((uint32_t)lane <= span) ? tb->key[lane] : 0xFFFFFFFFu;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t t = __shfl_down(key, d, 64);
            if (lane + d < 64) key = t < key ? t : key;
        }
        const uint32_t knext = __shfl_down(key, 1, 64);
        uint32_t len0 = 0, len1 = 0, nb0 = 0, nb1 = 0;
        unsigned long long g0 = 0, g1 = 0;
        if ((uint32_t)lane < span) {
            const uint32_t pf = key >> 16, r1f = key & 0xFFFFu;
            len1 = (knext & 0xFFFFu) - r1f;
            len0 = ((knext >> 16) - pf) - len1;
            if (len0 + len1) {
                const ulonglong2 zo = a.zo[vf + lane];
                const unsigned long long R = prefix + r1f;
                g0 = base + pf - R + zo.x;
                g1 = zo.y + R;
                nb0 = len0 ? (uint32_t)((g0 % CH + len0 + CH - 1) / CH) : 0u;
                nb1 = len1 ? (uint32_t)((g1 % CH + len1 + CH - 1) / CH) : 0u;
            }
        }
        const uint32_t incl = wave_incl_scan(nb0 + nb1);
        const uint32_t b0 = incl - nb0 - nb1;
        if ((uint32_t)lane < span) {
            tb->st[2 * lane] = b0 * CH + (uint32_t)(g0 % CH);
            tb->len[2 * lane] = len0;
            tb->g[2 * lane] = g0;
            tb->blk[2 * lane] = b0;
            tb->st[2 * lane + 1] = (b0 + nb0) * CH + (uint32_t)(g1 % CH);
            tb->len[2 * lane + 1] = len1;
            tb->g[2 * lane + 1] = g1;
            tb->blk[2 * lane + 1] = b0 + nb0;
        }
        if (lane == 63) tb->blk[nruns] = incl;
    }
    wave_sync();
    // stage every symbol in its run
    {
        uint32_t r = lr1, jc = 0xFFFFFFFFu, st0 = 0, st1 = 0, pf = 0, r1f = 0;
#pragma unroll
        for (int k = 0; k < E; k++) {
            if (k < nval) {
                const uint32_t x = raw_elem<W, B>(raw, k) & a.symmask;
                const uint32_t j = nbase + (x >> nsh) - vf;
                const uint32_t b = (uint32_t)(mb >> k) & 1u;
                if (j != jc && j < span) {
                    jc = j;
                    const uint32_t key = tb->key[j];
                    pf = key >> 16;
                    r1f = key & 0xFFFFu;
                    st0 = tb->st[2 * j];
                    st1 = tb->st[2 * j + 1];
                }
                if (j < span) {
                    const uint32_t p = (uint32_t)lane * E + k;
                    const uint32_t idx = b ? st1 + (r - r1f) : st0 + (p - pf) - (r - r1f);
                    if (idx < kStage) s_stage[idx] = (T)x;
                }
                r += b;
            }
        }
    }
    wave_sync();
    // write the runs out, one 16-byte staging block per lane and step: first
    // every block lying wholly inside its run, then the partial first / last
    // blocks of the runs, one per lane (nruns < 32), so that no per-symbol
    // loop runs under divergence in the block loop
    auto add_ones = [&](uint32_t run, unsigned long long gfirst, uint32_t ones) {
        if (counting && ones) {
            const uint64_t dt = gfirst / TILE;  // a block's symbols share one destination tile
            const uint32_t key = 2 * run + (uint32_t)(dt & 1);
            atomicAdd(&tb->cnt[key], ones);
            tb->tix[key] = (uint32_t)dt;
        }
    };
    const uint32_t nblk = tb->blk[nruns];
    for (uint32_t blk = (uint32_t)lane; blk < nblk; blk += 64) {
        uint32_t lo = 0, hi = nruns - 1;  // last run whose first block is <= blk
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (tb->blk[mid] <= blk) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t st = tb->st[lo], len = tb->len[lo];
        const unsigned long long g = tb->g[lo];
        const uint32_t s = blk * CH;
        if (s + CH > kStage) continue;  // (only with inconsistent tables)
        if (!(s >= st && s + CH <= st + len && g + (s - st) + CH <= a.n_out)) continue;  // partial: below
        const uint4 v = *reinterpret_cast<const uint4 *>(&s_stage[s]);
        const unsigned long long gfirst = g + (s - st);
        *reinterpret_cast<uint4 *>(tout + gfirst) = v;
        add_ones(lo, gfirst, counting ? chunk_bit_count<WO>(v, sh2) : 0u);
    }
    {
        const uint32_t run = (uint32_t)lane >> 1;
        if (run < nruns) {
            const uint32_t st = tb->st[run], len = tb->len[run];
            const unsigned long long g = tb->g[run];
            const uint32_t bfirst = tb->blk[run], bend = tb->blk[run + 1];
            const uint32_t blk = (lane & 1) ? bend - 1 : bfirst;
            const uint32_t s = blk * CH;
            const bool take = len > 0 && bend > bfirst && !((lane & 1) && bend - 1 == bfirst) && s + CH <= kStage;
            if (take && !(s >= st && s + CH <= st + len && g + (s - st) + CH <= a.n_out)) {
                const uint4 v = *reinterpret_cast<const uint4 *>(&s_stage[s]);
                uint32_t ones = 0;
#pragma unroll
                for (int e = 0; e < (int)CH; e++) {
                    const uint32_t q = s + e;
                    if (q >= st && q < st + len && g + (q - st) < a.n_out) {
                        const uint32_t x = chunk_elem<WO>(v, e);
                        tout[g + (q - st)] = (T)x;
                        ones += (x >> sh2) & 1u;
                    }
                }
                add_ones(run, g + ((s > st ? s : st) - st), ones);
            }
        }
    }
    if (!counting) return;
    wave_sync();
    for (uint32_t q = lane; q < 4 * span; q += 64) {
        const uint32_t c = tb->cnt[q];
        if (c) {
            const uint32_t r = q >> 1;
            atomicAdd(&a.tile_ones_next[tb->tix[q]], c);
            if (!kOptNodes || ones_next)
                atomicAdd(&ones_next[2ull * (vf + (r >> 1)) + (r & 1u)], (unsigned long long)c);
        }
    }
}

// Split of a tile spanning many nodes vf..vl (at least kRunNodes).  Nodes
// strictly between vf and vl lie inside the tile, and so do their two
// children in T_{i+1} (zeros then ones, in the node's own positions): with
// [ps, pe) the node's tile positions and rs / re the tile ones before ps /
// pe, a symbol at p with r tile ones before it goes to
//     bit 0: p - r + rs,      bit 1: pe - (re - r)
// (the node-local form of the destinations, Section 3.1).  Those symbols are
// staged in LDS at their own tile positions and leave as one aligned block;
// their children's next-level ones are stored once per node (atomics only
// for nodes crossing lanes).  The two edge nodes vf and vl may extend past
// the tile and use the node tables; their next-level ones are counted per
// (node, bit, destination-tile parity).  Node starts and their tile ranks
// travel between lanes as (position << 16 | rank) in a prefix maximum and a
// suffix minimum.
template <int W, int B, int WO, bool kCopy, bool kOptNodes>
__device__ __forceinline__ void split_dense(const LevelArgs &a, const uint4 (&raw)[B / 16],
                                            typename MaskT<B / W>::T mb, int nval, uint32_t lr1, uint32_t agg,
                                            unsigned long long prefix, uint64_t base, uint64_t nvalid, uint64_t t,
                                            uint32_t vf, uint32_t vl, uint32_t nsh, uint32_t nbase, uint8_t *s_wave,
                                            typename ElemT<WO>::T *tout, bool counting, uint32_t sh2,
                                            unsigned long long *ones_next) {
    typedef typename ElemT<W>::T T;    // symbols read
    typedef typename ElemT<WO>::T TO;  // symbols staged and written
    typedef typename MaskT<B / W>::T Mk;
    constexpr int E = B / W;
    constexpr uint32_t CH = 16 / WO;
    constexpr uint64_t TILE = tile_syms(W, B);
    const int lane = threadIdx.x & 63;
    TO *s_stage = reinterpret_cast<TO *>(s_wave);
    const uint32_t p0 = (uint32_t)lane * E;
    const uint32_t nv = (uint32_t)nvalid;
    // The per-symbol loops run rolled (unrolled, they held too many
    // registers): over an LDS copy of the lane's symbols behind the staging
    // area where it fits the variant's slice, else over T_i itself, which the
    // wave has just loaded (only positions below n are read there).
    const T *s_sym;
    if constexpr (kCopy) {
        T *c = reinterpret_cast<T *>(s_wave + TILE * W) + p0;
#pragma unroll
        for (int q = 0; q < B / 16; q++) reinterpret_cast<uint4 *>(c)[q] = raw[q];
        s_sym = c;
    } else {
        s_sym = reinterpret_cast<const T *>(a.tin) + base + p0;
    }

    // node starts of this lane
    Mk fm = 0;
    {
        uint32_t vprev = wave_prev_lane(nbase + ((raw_elem<W, B>(raw, E - 1) & a.symmask) >> nsh), 0xFFFFFFFFu);
#pragma unroll 2
        for (int k = 0; k < E; k++) {
            if (k < nval) {
                const uint32_t v = nbase + (((uint32_t)s_sym[k] & a.symmask) >> nsh);
                if (v != vprev) fm |= (Mk)1 << k;
                vprev = v;
            }
        }
    }
    // (position << 16 | tile rank) of the lane's last and first node start
    uint32_t last_pk = 0, first_pk = 0xFFFFFFFFu;
    if (fm) {
        const int kl = (E == 64) ? 63 - __clzll((unsigned long long)fm) : 31 - __clz((uint32_t)fm);
        const int kf = (E == 64) ? __ffsll((unsigned long long)fm) - 1 : __ffs((uint32_t)fm) - 1;
        const uint32_t rl = lr1 + ((E == 64) ? (uint32_t)__popcll((unsigned long long)mb & ((1ull << kl) - 1ull))
                                             : (uint32_t)__popc((uint32_t)mb & ((1u << kl) - 1u)));
        const uint32_t rf = lr1 + ((E == 64) ? (uint32_t)__popcll((unsigned long long)mb & ((1ull << kf) - 1ull))
                                             : (uint32_t)__popc((uint32_t)mb & ((1u << kf) - 1u)));
        last_pk = ((p0 + kl) << 16) | rl;
        first_pk = ((p0 + kf) << 16) | rf;
    }
    // node start before the lane (position 0 always starts one) and node end
    // after it (or the tile end, nvalid with all the tile's ones)
    const uint32_t start_in = wave_prev_lane(wave_incl_max(last_pk), 0u);
    uint32_t end_in;
    {
        const uint32_t rev = ~(uint32_t)__shfl(first_pk, 63 - lane, 64);
        const uint32_t ex = wave_prev_lane(wave_incl_max(rev), 0u);
        end_in = ~(uint32_t)__shfl(ex, 63 - lane, 64);
        if (end_in == 0xFFFFFFFFu) end_in = (nv << 16) | agg;
    }
    // interior block of the tile: from the second node start to the last one
    const uint32_t sec = (lane == 0) ? (((uint64_t)fm >> 1) ? (uint32_t)__builtin_ctzll((uint64_t)fm >> 1) + 1 : nv)
                                     : (fm ? (first_pk >> 16) : nv);
    const uint32_t ia_u = ~(uint32_t)__builtin_amdgcn_readlane((int)wave_incl_max(~sec), 63);  // lane minimum
    // last node start of the tile (vl's first tile position) and its tile rank
    const uint32_t lastmax = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_max(last_pk), 63);
    const uint32_t ib_u = lastmax >> 16, rvl = lastmax & 0xFFFFu;

    const ulonglong2 zf = a.zo[vf], zl = a.zo[vl];
    // edge counts, key = 4 e + 2 b + parity (e = 0: vf, 1: vl), 16 bits each
    unsigned long long ecl = 0, ech = 0;
    uint32_t icount = 0;                 // next-level ones of interior symbols (all in tile t)
    uint32_t ps = 0, pe = 0, rs = 0, re = 0, vcur = 0, c0 = 0, c1 = 0;
    bool interior = false, open = false;
    uint32_t r = lr1;
    // ones of an interior node's children: a plain store when the node lies
    // in this lane, an atomic when it crosses lanes
    auto flush = [&]() {
        if (open && interior && counting && (!kOptNodes || ones_next) && (c0 | c1)) {
            unsigned long long *o = &ones_next[2ull * vcur];
            if (ps >= p0 && pe <= p0 + E) {
                o[0] = c0;
                o[1] = c1;
            } else {
                if (c0) atomicAdd(&o[0], (unsigned long long)c0);
                if (c1) atomicAdd(&o[1], (unsigned long long)c1);
            }
        }
    };
#pragma unroll 2
    for (int k = 0; k < E; k++) {
        if (k < nval) {
            const uint32_t x = (uint32_t)s_sym[k] & a.symmask;
            const uint32_t v = nbase + (x >> nsh);
            const uint32_t b = (uint32_t)(mb >> k) & 1u;
            const uint32_t p = p0 + k;
            const bool fl = ((uint64_t)fm >> k) & 1u;
            if (k == 0 || fl) {
                flush();
                open = true;
                c0 = c1 = 0;
                vcur = v;
                if (fl) { ps = p; rs = r; }
                else { ps = start_in >> 16; rs = start_in & 0xFFFFu; }
                const uint64_t above = (k + 1 < 64) ? ((uint64_t)fm >> (k + 1)) : 0ull;
                if (above) {
                    const int kn = k + 1 + __builtin_ctzll(above);
                    pe = p0 + kn;
                    re = lr1 + ((E == 64) ? (uint32_t)__popcll((unsigned long long)mb & ((1ull << kn) - 1ull))
                                          : (uint32_t)__popc((uint32_t)mb & ((1u << kn) - 1u)));
                } else {
                    pe = end_in >> 16;
                    re = end_in & 0xFFFFu;
                }
                interior = v != vf && v != vl && v - vf <= vl - vf;
            }
            const uint32_t nb = counting ? (x >> sh2) & 1u : 0u;
            if (interior) {
                const uint32_t dl = b ? pe - (re - r) : p - r + rs;
                if (dl < TILE) s_stage[dl] = (TO)x;
                c0 += nb & (b ^ 1u);
                c1 += nb & b;
                icount += nb;
            } else if (v == vf || v == vl) {
                const ulonglong2 zo = (v == vf) ? zf : zl;
                const unsigned long long R = prefix + r;
                const uint64_t dst = b ? zo.y + R : base + p - R + zo.x;
                if (dst < a.n_out) {
                    tout[dst] = (TO)x;
                    const uint32_t key = ((v == vf) ? 0u : 4u) + 2 * b + (uint32_t)((dst / TILE) & 1);
                    if (key < 4) ecl += (unsigned long long)nb << (16 * key);
                    else ech += (unsigned long long)nb << (16 * (key - 4));
                }
            }
            r += b;
        }
    }
    flush();
    wave_sync();
    // the interior block [ia_u, ib_u): whole aligned chunks (tile positions
    // and destinations agree), then the at most 2 (CH - 1) symbols of its
    // partial first and last chunk, one per lane
    {
        const uint32_t ca = (ia_u + CH - 1) / CH, cb = ib_u / CH;  // whole chunks [ca, cb)
        for (uint32_t c = ca + lane; c < cb; c += 64) {
            const uint32_t s0 = c * CH;
            if (base + s0 + CH <= a.n_out)
                *reinterpret_cast<uint4 *>(tout + (base + s0)) = *reinterpret_cast<const uint4 *>(&s_stage[s0]);
        }
        if (ia_u < ib_u) {
            // head [ia_u, min(ca CH, ib_u)) on lanes 0..CH-2, tail [max(cb CH, ca CH), ib_u) on lanes 32..
            const uint32_t he = (ca * CH < ib_u) ? ca * CH : ib_u;
            const uint32_t tb0 = (cb * CH > ca * CH) ? cb * CH : ((ca * CH < ib_u) ? ca * CH : ib_u);
            const uint32_t q = (lane < 32) ? ia_u + (uint32_t)lane : tb0 + (uint32_t)(lane - 32);
            const uint32_t qe = (lane < 32) ? he : ib_u;
            if (q < qe && base + q < a.n_out) tout[base + q] = s_stage[q];
        }
    }
    if (!counting) return;
    const uint32_t itot = wave_sum32(icount);
    if (lane == 0 && itot) atomicAdd(&a.tile_ones_next[t], itot);
    // edge runs: vf's part starts at tile position 0 (tile rank 0), vl's at
    // ib_u (tile rank rvl); a run of at most TILE symbols touches two
    // consecutive destination tiles, and its first destination tells which
    // one has a given parity
#pragma unroll
    for (int key = 0; key < 8; key++) {
        const uint32_t cnt = wave_sum32((uint32_t)((((key < 4) ? ecl : ech) >> (16 * (key & 3))) & 0xFFFFu));
        if (cnt && lane == 0) {
            const uint32_t e = (uint32_t)key >> 2, b = ((uint32_t)key >> 1) & 1u, par = (uint32_t)key & 1u;
            const ulonglong2 zo = e ? zl : zf;
            const uint32_t fp = e ? ib_u : 0u, fr = e ? rvl : 0u;
            const unsigned long long R = prefix + fr;
            const uint64_t d0 = b ? zo.y + R : base + fp - R + zo.x;
            const uint64_t dt0 = d0 / TILE;
            const uint64_t dt = ((dt0 & 1) == par) ? dt0 : dt0 + 1;
            if (dt < a.ntiles) atomicAdd(&a.tile_ones_next[dt], cnt);  // (always, with consistent tables)
            if (!kOptNodes || ones_next) atomicAdd(&ones_next[2ull * (e ? vl : vf) + b], (unsigned long long)cnt);
        }
    }
}

// Next-level ones of a single-node tile, per (run, destination-tile parity)
// q: destination tile dt[q] and count cnt[q] (0: none), for child node
// child + (q >> 1).  The workgroup adds them up before its atomics (its
// consecutive tiles mostly share a node, whose few counter addresses would
// otherwise take one atomic per tile).
struct SplitRec {
    uint32_t dt[4], cnt[4];
    uint32_t child;
};

// One level pass over tile t, run by one wave (each lane B bytes = E = B/W
// symbols of T_i); s_wave is the wave's own LDS slice.  Single-node tiles
// leave their next-level counts in *rec; other tiles add theirs directly.
// T_{i+1} is written with WO-byte symbols (WO = W, or W / 2 where the
// order narrows), in tiles of EO symbols per lane.  With kOptNodes (the
// batched passes) a null a.ones_next means that the next level's node counts
// are not wanted; the single-build passes always count them (the extra test
// costs their staged variants scalar registers).
template <int W, int B, int WO, bool kMulti, bool kCopy, int EO = B / W, bool kOptNodes = false>
__device__ __forceinline__ void level_tile(const LevelArgs &a, uint64_t t, uint8_t *s_wave, SplitRec *rec) {
    typedef typename ElemT<WO>::T TO;           // symbols of T_{i+1}
    constexpr int E = B / W;                    // symbols per lane
    constexpr int CH = 16 / WO;                 // output symbols per 16-byte chunk
    constexpr uint64_t TILE = tile_syms(W, B);  // 64 * E
    // tiles of T_{i+1}, which its next-level ones are counted by: the same,
    // or twice as long where a narrowing pass also doubles the symbols per
    // lane (a run of at most TILE symbols still touches at most two of them)
    constexpr uint64_t TILE_NEXT = 64ull * EO;
    static_assert(TILE < 65536, "per-tile counts travel in 16-bit fields");
    static_assert(WO == W || (2 * WO == W && !kMulti), "a narrowing pass halves the width, without the staged paths");
    static_assert(EO == E || (EO == 2 * E && WO < W && EO <= 64), "only a narrowing pass doubles the tiles");
    typedef typename MaskT<E>::T M;
    const int lane = threadIdx.x & 63;
    TO *s_stage = reinterpret_cast<TO *>(s_wave);
    uint32_t *s_cnt = reinterpret_cast<uint32_t *>(s_wave);
    uint32_t *s_tix = s_cnt + 4 * kNodeCap;

    const uint32_t sh = a.levels - 1 - a.level;  // bit of this level
    const uint32_t nsh = a.levels - a.level;     // node shift (Proposition 1)
    const uint64_t base = t * TILE;
    const uint64_t pos0 = base + (uint64_t)lane * E;
    const uint64_t nvalid = (a.n - base < TILE) ? a.n - base : TILE;  // base < n

    uint4 raw[B / 16];
    const int nval = load_lane<W, B>(a.tin, pos0, a.n, raw);
    // ones before the tile: superchunk prefix + earlier tiles of the superchunk
    uint32_t pv = 0;
    {
        // four consecutive counts per lane (16-byte aligned: kSup and the
        // level's base are multiples of 4 entries)
        const uint64_t q = t - t % kSup + 4 * (uint64_t)lane;
        if (q < t) {
            const uint4 c = *reinterpret_cast<const uint4 *>(a.tile_ones + q);
            pv = c.x + (q + 1 < t ? c.y : 0u) + (q + 2 < t ? c.z : 0u) + (q + 3 < t ? c.w : 0u);
        }
    }
    unsigned long long prefix = a.sup[t / kSup];

    // u8: the split reads the spread order, everything else the symbol order
    const M ms = level_bits_split<W, B>(raw, sh);
    M mb = ms;
    if constexpr (W == 1) mb = spread_order(ms);
    const uint32_t pc = (E == 64) ? (uint32_t)__popcll((uint64_t)ms) : (uint32_t)__popc((uint32_t)ms);
    const uint32_t incl = wave_incl_scan(pc);
    const uint32_t agg = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    prefix += wave_sum32(pv);
    const uint32_t lr1 = incl - pc;  // ones in the tile before this lane
    const unsigned long long r_lane = prefix + lr1;

    if (a.bits) {
        // bitmap words: 64 / E consecutive lanes form one word
        uint64_t wd = (uint64_t)mb;
#pragma unroll
        for (int d = 1; d < 64 / E; d++) wd |= (uint64_t)__shfl_down((uint32_t)mb, d, 64) << (d * E);
        if ((lane % (64 / E)) == 0) {
            const uint64_t widx = pos0 / 64;
            if (widx < a.words) {
                a.bits[widx] = wd;
                note_write(&a.bits[widx], 8);
            }
        }
        // rank directory: entry k = ones before position 512k
        if ((pos0 & 511) == 0) {
            const uint64_t k = pos0 >> 9;
            if (k < a.rank_stride) a.ranks[k] = (k < a.rank_entries) ? r_lane : 0ull;
        }
        if (t == a.ntiles - 1 && lane < 8) {  // entries past the last tile
            const uint64_t k = (base + TILE) / 512 + lane;
            if (k < a.rank_stride) a.ranks[k] = (k < a.rank_entries) ? prefix + agg : 0ull;
        }
    }
    if (a.zeros && t == a.ntiles - 1 && lane == 0) a.zeros[a.level] = a.n - (prefix + agg);
    if (a.digits) {
        // 4-ary tree: T_i is also the order of a digit level; its digits,
        // 32 per word (positions >= n read as 0, so padding digits are 0)
        constexpr int DPW = 32;
        if (E >= DPW) {
#pragma unroll
            for (int w = 0; w < E / DPW; w++) {
                uint64_t wd = 0;
#pragma unroll
                for (int k = 0; k < DPW; k++)
                    wd |= (uint64_t)((raw_elem<W, B>(raw, w * DPW + k) >> a.dsh) & 3u) << (2 * k);
                const uint64_t widx = pos0 / DPW + w;
                if (widx < a.dwords) {
                    a.digits[widx] = wd;
                    note_write(&a.digits[widx], 8);
                }
            }
        } else {
            uint32_t part = 0;  // 2E <= 32 bits
#pragma unroll
            for (int k = 0; k < E; k++) part |= ((raw_elem<W, B>(raw, k) >> a.dsh) & 3u) << (2 * k);
            uint64_t wd = part;
#pragma unroll
            for (int d = 1; d < DPW / E; d++) wd |= (uint64_t)__shfl_down(part, d, 64) << (d * 2 * E);
            if ((lane % (DPW / E)) == 0) {
                const uint64_t widx = pos0 / DPW;
                if (widx < a.dwords) {
                    a.digits[widx] = wd;
                    note_write(&a.digits[widx], 8);
                }
            }
        }
    }

    // folded last level (u8, single-node and direct paths only): bits of
    // T_{i+1} instead of its symbols, in 16-bit granules
    uint16_t *bnext = reinterpret_cast<uint16_t *>(a.bits_next);
    const bool fold = (W == 1) && !kMulti && bnext != nullptr;
    if (a.tout == nullptr && !fold) return;  // last level: no next order, no counts

    TO *tout = reinterpret_cast<TO *>(a.tout);
    const bool counting = a.tile_ones_next != nullptr;
    const uint32_t sh2 = sh - 1;  // bit of the next level (when counting)
    // (slot counts are powers of two; with kOptNodes a null a.ones_next means
    // no node counts: the next level is a last level whose node tables
    // nobody reads)
    unsigned long long *ones_next = (counting && (!kOptNodes || a.ones_next))
                                        ? a.ones_next + (t & (a.slots_next - 1)) * a.nodes_next
                                        : nullptr;

    // narrowed T_i: a node's high bits come from the anchor holding the
    // position (every symbol of the tile has the first one unless the tile
    // holds two or more anchors: then it takes the direct split, which
    // follows the anchors symbol by symbol)
    uint2 anc = make_uint2(0u, 0u);
    uint32_t asw = 0;  // node bits below the anchor, carried by the symbol
    if (a.tile_anc) {
        anc = a.tile_anc[t];
        asw = 8u * W - nsh;
    }
    const bool straddle = anc.x != anc.y;
    const uint32_t nbase = anc.x << asw;

    // node span of the tile (T_i is sorted by node)
    const bool full = (nvalid == TILE);  // every tile but a ragged last one
    // (a wavelet matrix has one node per level: every tile is single-node)
    const uint32_t vf = a.matrix ? 0u :
        nbase + (uint32_t)__builtin_amdgcn_readlane((int)((raw_elem<W, B>(raw, 0) & a.symmask) >> nsh), 0);
    uint32_t vl;
    if (full) {
        vl = (uint32_t)__builtin_amdgcn_readlane((int)((raw_elem<W, B>(raw, E - 1) & a.symmask) >> nsh), 63);
    } else {
        const uint64_t last = nvalid - 1;
        const int kl = (int)(last % E);
        uint32_t xv = 0;
#pragma unroll
        for (int k = 0; k < E; k++) xv = (k == kl) ? raw_elem<W, B>(raw, k) : xv;
        vl = (uint32_t)__builtin_amdgcn_readlane((int)((xv & a.symmask) >> nsh), (int)(last / E));
    }
    vl = a.matrix ? 0u : (anc.y << asw) + __builtin_amdgcn_readfirstlane(vl);
    if (vf == vl) {  // (never for a tile over two anchors)
        // Single node: zeros keep their order at g0.., ones at g1...
        const ulonglong2 zo = a.zo[vf];
        const uint64_t Z = nvalid - agg, O = agg;
        const uint64_t g0 = base - prefix + zo.x;
        const uint64_t g1 = zo.y + prefix;
        const uint32_t a0 = (uint32_t)(g0 % CH);
        const uint32_t r1 = (uint32_t)round_up(a0 + Z, CH);
        const uint32_t a1 = r1 + (uint32_t)(g1 % CH);
        const uint32_t zc = a0 + (uint32_t)lane * E - lr1;  // first zero slot of this lane
        const uint32_t oc = a1 + lr1;                       // first one slot of this lane
        if (full) stage_split<W, B, WO, true>(s_stage, raw, ms, zc, oc, nval);
        else stage_split<W, B, WO, false>(s_stage, raw, ms, zc, oc, nval);
        wave_sync();
        // Write the two runs out (zeros at slots [a0, a0+Z) -> g0.., ones at
        // [a1, a1+O) -> g1..); the slot and destination phases agree, so
        // chunks are aligned in both.  Chunks wholly inside a run leave as
        // one 16-byte store per lane and step; the at most two partial
        // chunks of each run (its first and last) are written afterwards,
        // one symbol per lane (4 x CH <= 64 lanes), so no lane runs a
        // per-symbol loop while the others wait.  A run holds at most TILE
        // symbols, so it touches at most two consecutive destination tiles:
        // next-level ones are counted per (run, tile).
        const uint32_t lowbits = (WO == 1) ? 0x01010101u : (WO == 2) ? 0x00010001u : 1u;
        const uint32_t mk = counting ? lowbits << sh2 : 0u;  // next-level bit of every symbol
        uint32_t cnt[4] = {0u, 0u, 0u, 0u};                   // (run, destination-tile parity)
        uint32_t lo_r[2], len_r[2], edge_r[2][2];
        uint64_t gb_r[2], dt0_r[2], cs_r[2];
#pragma unroll
        for (int r = 0; r < 2; r++) {
            const uint32_t lo = r ? a1 : a0;
            const uint64_t gb = (r ? g1 : g0) - lo;  // destination = gb + slot
            // a run whose destinations lie below 0 is dropped whole (a
            // child that the next level does not list; runs never straddle 0)
            const uint32_t len = ((int64_t)(gb + lo) < 0) ? 0u : (uint32_t)(r ? O : Z);
            const uint32_t cb = lo / CH, ce = len ? (lo + len + CH - 1) / CH : cb;
            const uint32_t fb = (lo + CH - 1) / CH, fe = (lo + len) / CH;  // chunks inside the run
            const uint64_t dt0 = (gb + (uint64_t)cb * CH) / TILE_NEXT;
            const uint64_t cs = ((dt0 + 1) * TILE_NEXT - gb) / CH;  // first chunk in tile dt0 + 1
            lo_r[r] = lo;
            len_r[r] = len;
            gb_r[r] = gb;
            dt0_r[r] = dt0;
            cs_r[r] = cs;
            // partial chunks (0xffffffff: none): the first when the run starts
            // inside it, the last when the run ends inside it (once, if the two
            // are the same chunk)
            edge_r[r][0] = (cb < ce && cb < fb) ? cb : 0xffffffffu;
            edge_r[r][1] = (cb < ce && fe < ce && ce - 1 != edge_r[r][0]) ? ce - 1 : 0xffffffffu;
            // (destinations beyond n only arise from inconsistent tables;
            // they are dropped rather than written; checked per chunk only
            // when the run's last whole chunk would pass n)
            const bool inside = gb + (uint64_t)fe * CH <= a.n_out;
            for (uint32_t c = fb + lane; c < fe; c += 64) {  // whole chunks [fb, fe)
                const uint32_t s = c * CH;
                const uint4 v = *reinterpret_cast<const uint4 *>(&s_stage[s]);
                if (inside || gb + s + CH <= a.n_out) {
                    if (fold) {  // the granule's 16 bits (gb + s is a multiple of 16)
                        bnext[(gb + s) >> 4] = (uint16_t)chunk_bits16(v, sh2);
                        note_write(&bnext[(gb + s) >> 4], 2);
                    } else
                        *reinterpret_cast<uint4 *>(tout + (gb + s)) = v;
                    const uint32_t ones = __popc(v.x & mk) + __popc(v.y & mk) + __popc(v.z & mk) + __popc(v.w & mk);
                    const bool second = c >= cs;
                    cnt[2 * r] += second ? 0u : ones;
                    cnt[2 * r + 1] += second ? ones : 0u;
                }
            }
        }
        {
            // lane -> (run, which partial chunk, symbol): 16 lanes per chunk.
            // Plain selects between the two runs' values (a lane-indexed
            // private array would live in scratch memory).
            const bool r1 = lane >= 32, which = (lane >> 4) & 1;
            const int e = lane & 15;
            const uint32_t c = r1 ? (which ? edge_r[1][1] : edge_r[1][0]) : (which ? edge_r[0][1] : edge_r[0][0]);
            const uint32_t lo = r1 ? lo_r[1] : lo_r[0], len = r1 ? len_r[1] : len_r[0];
            const uint64_t gb = r1 ? gb_r[1] : gb_r[0], cs = r1 ? cs_r[1] : cs_r[0];
            uint32_t one = 0;
            bool second = false;
            uint64_t own = ~0ull;  // folded: the granule whose first position this lane's symbol lands on
            if (e < CH && c != 0xffffffffu) {
                const uint32_t s = c * CH + (uint32_t)e;
                const uint64_t d = gb + s;
                if (s >= lo && s < lo + len && d < a.n_out) {
                    const uint32_t x = (uint32_t)s_stage[s];
                    tout[d] = (TO)x;  // (folded: read back by the stitch)
                    one = (x >> sh2) & 1u;
                    second = c >= cs;
                    if (fold && e == 0) own = d >> 4;
                }
            }
            if (fold) {
                // a run owns at most one shared granule: the one of its last
                // partial chunk when that chunk starts inside the run (lanes
                // 0 / 16 hold run 0's two edge chunks, 32 / 48 run 1's)
                const uint64_t o2 = __shfl_down(own, 16, 64);
                if ((lane & 31) == 0) a.fold_own[2 * t + (uint64_t)(lane >> 5)] = own < o2 ? own : o2;
            }
            if (counting) {
                cnt[0] += (!r1 && !second) ? one : 0u;
                cnt[1] += (!r1 && second) ? one : 0u;
                cnt[2] += (r1 && !second) ? one : 0u;
                cnt[3] += (r1 && second) ? one : 0u;
            }
        }
        if (counting) {
            // two counts per 32-bit sum (each at most TILE < 2^16)
            const uint32_t t01 = wave_sum32(cnt[0] | (cnt[1] << 16)), t23 = wave_sum32(cnt[2] | (cnt[3] << 16));
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const uint32_t tq = ((q < 2 ? t01 : t23) >> (16 * (q & 1))) & 0xFFFFu;
                if (lane == 0) {
                    rec->dt[q] = (uint32_t)dt0_r[q >> 1] + (uint32_t)(q & 1);
                    rec->cnt[q] = tq;
                }
            }
        }
        if (!counting) return;
        if (lane == 0) rec->child = 2 * vf;
        return;
    }

    if constexpr (kMulti) {
        if (straddle) {
            // (the direct split below)
        } else if (vl - vf < kRunNodes)
            stage_multi<W, B, WO, kOptNodes>(a, raw, mb, nval, lr1, agg, prefix, base, nvalid, vf, vl, nsh, nbase,
                                             s_wave, tout, counting, sh2, ones_next);
        else
            split_dense<W, B, WO, kCopy, kOptNodes>(a, raw, mb, nval, lr1, agg, prefix, base, nvalid, t, vf, vl, nsh,
                                                    nbase, s_wave, tout, counting, sh2, ones_next);
        if (!straddle) return;
    }

    // Many nodes: every symbol goes straight to its destination.
    const bool lds_counts = counting && (vl - vf < kNodeCap);
    if (lds_counts) {
        for (uint32_t q = lane; q < 4 * (vl - vf + 1); q += 64) s_cnt[q] = 0;
        wave_sync();
    }
    unsigned long long r1 = r_lane;
    // folded: every symbol is stored at its T_{i+1} position, and the
    // granules whose first position a symbol lands on are recorded for the
    // stitch (counted here, appended below)
    uint32_t nown = 0;
    if (fold && lane == 0) {
        a.fold_own[2 * t] = ~0ull;
        a.fold_own[2 * t + 1] = ~0ull;
    }
    // narrowed, over two anchors: the anchor of the lane's first symbol (the
    // last one in [anc.x, anc.y] whose node starts at or before it), then
    // the next anchor's start; a symbol at or past it searches again
    auto find_anchor = [&](uint32_t lo, uint32_t hi, uint64_t p) {
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo + 1) / 2;
            if (a.anc_start[mid] <= p) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    };
    uint32_t cur = anc.x;
    uint64_t next = ~0ull;
    if (straddle) {
        cur = find_anchor(anc.x, anc.y, pos0);
        next = (cur < anc.y) ? a.anc_start[cur + 1] : ~0ull;
    }
    // a lane's nodes never decrease (T_i is sorted by node): its node table
    // entry is loaded again only where the node changes, not per symbol
    uint32_t cv = (cur << asw) + ((raw_elem<W, B>(raw, 0) & a.symmask) >> nsh);
    ulonglong2 zo = a.zo[nval > 0 ? cv : vf];
#pragma unroll
    for (int k = 0; k < E; k++) {
        if (k < nval) {
            const uint64_t p = pos0 + k;
            if (p >= next) {
                cur = find_anchor(cur + 1, anc.y, p);
                next = (cur < anc.y) ? a.anc_start[cur + 1] : ~0ull;
            }
            const uint32_t x = raw_elem<W, B>(raw, k) & a.symmask;
            const uint32_t v = (cur << asw) + (x >> nsh);
            if (v != cv) {
                cv = v;
                zo = a.zo[v];
            }
            const uint32_t b = (uint32_t)(mb >> k) & 1u;
            const uint64_t dst = b ? zo.y + r1 : p - r1 + zo.x;
            r1 += b;
            if (dst < a.n_out) {
                tout[dst] = (TO)x;
                nown += (fold && (dst & 15) == 0) ? 1u : 0u;
                if (counting && ((x >> sh2) & 1u)) {
                    const uint64_t dt = dst / TILE_NEXT;
                    if (lds_counts && v - vf <= vl - vf) {
                        const uint32_t key = 4 * (v - vf) + 2 * b + (uint32_t)(dt & 1);
                        atomicAdd(&s_cnt[key], 1u);
                        s_tix[key] = (uint32_t)dt;
                    } else {
                        atomicAdd(&a.tile_ones_next[dt], 1u);
                        if (!kOptNodes || ones_next) atomicAdd(&ones_next[2ull * v + b], 1ull);
                    }
                }
            }
        }
    }
    if (fold) {
        // append this wave's records: one counter add per wave, then the
        // destinations walked again (a rare path: tiles on node boundaries)
        const uint32_t incl = wave_incl_scan(nown);
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        uint32_t at = 0;
        if (lane == 0 && tot) at = atomicAdd(a.fold_ovf_n, tot);
        at = (uint32_t)__builtin_amdgcn_readlane((int)at, 0) + incl - nown;
        if (lane == 0 && (uint64_t)at + tot > a.fold_ovf_cap && tot) atomicOr(a.fold_status, 2u);
        r1 = r_lane;
        // (a folded pass reads 1-byte input symbols, never a narrowed order:
        // nbase is 0 and no tile holds two anchors)
        cv = nbase + ((raw_elem<W, B>(raw, 0) & a.symmask) >> nsh);
        zo = a.zo[nval > 0 ? cv : vf];
#pragma unroll
        for (int k = 0; k < E; k++) {
            if (k < nval && nown) {
                const uint32_t v = nbase + ((raw_elem<W, B>(raw, k) & a.symmask) >> nsh);
                if (v != cv) {
                    cv = v;
                    zo = a.zo[v];
                }
                const uint32_t b = (uint32_t)(mb >> k) & 1u;
                const uint64_t dst = b ? zo.y + r1 : pos0 + k - r1 + zo.x;
                r1 += b;
                if (dst < a.n_out && (dst & 15) == 0) {
                    if (at < a.fold_ovf_cap) a.fold_ovf[at] = dst >> 4;
                    at++;
                    nown--;
                }
            }
        }
    }
    if (lds_counts) {
        wave_sync();
        for (uint32_t q = lane; q < 4 * (vl - vf + 1); q += 64) {
            const uint32_t c = s_cnt[q];
            if (c) {
                const uint32_t dt = s_tix[q];
                atomicAdd(&a.tile_ones_next[dt], c);
                if (!kOptNodes || ones_next)
                    atomicAdd(&ones_next[2ull * (vf + q / 4) + ((q >> 1) & 1u)], (unsigned long long)c);
            }
        }
    }
}


// After the workgroup's tiles: add up the single-node tiles' records by
// destination tile and by child node, one atomic per distinct key (the
// record with the lowest index adds the key's total).  Wave 0 does it with
// all its lanes: lane r + 16 g compares record r with the four records of
// wave g, and the four partial results of record r meet by two lane
// exchanges.  A partial result travels packed: the counts of the matching
// records (each below 2^16, so 16 of them stay below 2^24) plus, from bit
// 24, how many of them come before record r.
template <bool kOptNodes = false>
__device__ __forceinline__ void flush_split_recs(const LevelArgs &a, const SplitRec *recs, uint64_t t0) {
    static_assert(kWaves == 4, "16 records, four per wave, over the 64 lanes of wave 0");
    __syncthreads();
    if (threadIdx.x >= 64 || a.tile_ones_next == nullptr) return;
    const uint32_t lane = threadIdx.x, r = lane & 15, g = lane >> 4;
    const uint32_t w = r / 4, q = r % 4;
    const uint32_t c = recs[w].cnt[q];
    const uint32_t dt = recs[w].dt[q], child = a.matrix ? 0u : recs[w].child + (q >> 1);
    uint32_t pdt = 0, pch = 0;
#pragma unroll
    for (uint32_t j = 0; j < 4; j++) {
        const uint32_t c2 = recs[g].cnt[j];  // records with no count carry no key
        const uint32_t before = (4 * g + j < r) ? (1u << 24) : 0u;
        if (c2 != 0 && recs[g].dt[j] == dt) pdt += c2 + before;
        if (c2 != 0 && (a.matrix ? 0u : recs[g].child + (j >> 1)) == child) pch += c2 + before;
    }
    pdt += __shfl_xor(pdt, 16, 64);
    pch += __shfl_xor(pch, 16, 64);
    pdt += __shfl_xor(pdt, 32, 64);
    pch += __shfl_xor(pch, 32, 64);
    if (g != 0 || c == 0) return;
    if ((pdt >> 24) == 0) atomicAdd(&a.tile_ones_next[dt], pdt & 0xFFFFFFu);
    if ((pch >> 24) == 0 && (!kOptNodes || a.ones_next)) {
        unsigned long long *ones_next = a.ones_next + (t0 & (a.slots_next - 1)) * a.nodes_next;
        atomicAdd(&ones_next[child], (unsigned long long)(pch & 0xFFFFFFu));
    }
}

template <int W, int B, int WO, bool M, int EO = B / W>
__device__ __forceinline__ void level_kernel_body(const LevelArgs &a) {
    constexpr bool kCopy = dense_lds_copy<W, B>();
    __shared__ __align__(16) uint8_t s_all[kWaves * level_wave_bytes<W, B, M, kCopy>()];
    __shared__ SplitRec s_rec[kWaves];
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t t0 = (uint64_t)blockIdx.x * kWaves;
    const uint64_t t = t0 + wv;
    if ((threadIdx.x & 63) < 4) s_rec[wv].cnt[threadIdx.x & 63] = 0;
    if (t < a.ntiles)
        level_tile<W, B, WO, M, kCopy, EO>(a, t, s_all + wv * level_wave_bytes<W, B, M, kCopy>(), &s_rec[wv]);
    flush_split_recs(a, s_rec, t0);
}

template <int W, int B, bool M>
__global__ __launch_bounds__(kThreads) void k_level(LevelArgs a) {
    level_kernel_body<W, B, W, M>(a);
}

// A narrowing level pass: T_{i+1} keeps the low W / 2 bytes of each symbol,
// in tiles of BO bytes per lane (B / 2: the same symbols per lane; B: twice
// as many).
template <int W, int B, int BO>
__global__ __launch_bounds__(kThreads) void k_level_narrow(LevelArgs a) {
    level_kernel_body<W, B, W / 2, false, BO / (W / 2)>(a);
}

// Anchors of every tile: one thread per tile, binary search over the anchor
// level's node starts (the node holding p is the last one starting at or
// before p: empty nodes start where the next one does).
__global__ __launch_bounds__(kThreads) void k_tile_anchor(AnchorArgs a) {
    const uint64_t t = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (t >= a.ntiles) return;
    auto find = [&](uint64_t p) {
        uint64_t lo = 0, hi = a.nodes - 1;
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo + 1) / 2;
            if (a.start[mid] <= p) lo = mid;
            else hi = mid - 1;
        }
        return (uint32_t)lo;
    };
    const uint64_t p0 = t * a.tile;
    const uint64_t p1 = (p0 + a.tile < a.n ? p0 + a.tile : a.n) - 1;
    a.out[t] = make_uint2(find(p0), find(p1));
}

// ------------------------------------------------------------ batched ---
// A batched build runs the same per-tile work for many sequences, one launch
// per phase and width class: workgroup b of a tile kernel serves sequence
// blk_map[b], tiles (b - blk_base) * kWaves + wave.

__device__ __forceinline__ LevelArgs job_level(const BatchJob &j, uint32_t i) {
    LevelArgs a;
    const uint32_t l = j.levels;
    uint8_t *w = j.work;
    a.tin = (i == 0) ? j.S : (const void *)(w + (((i - 1) & 1) ? j.ws_tb : j.ws_ta));
    a.tout = (i + 1 < l) ? (void *)(w + ((i & 1) ? j.ws_tb : j.ws_ta)) : nullptr;
    a.bits = reinterpret_cast<uint64_t *>(j.tree + j.tree_bits_off) + (uint64_t)i * j.words;
    a.ranks = reinterpret_cast<uint64_t *>(j.tree + j.tree_ranks_off) + (uint64_t)i * j.rank_stride;
    a.zo = reinterpret_cast<const ulonglong2 *>(w + j.ws_zo) + zo_offset(i);
    uint32_t *tile_ones = reinterpret_cast<uint32_t *>(w + j.ws_tile_ones);
    a.tile_ones = tile_ones + (uint64_t)i * tile_stride(j.ntiles);
    a.sup = reinterpret_cast<const unsigned long long *>(w + j.ws_sup) + (uint64_t)i * j.nsup;
    a.tile_ones_next = (i + 1 < l) ? tile_ones + (uint64_t)(i + 1) * tile_stride(j.ntiles) : nullptr;
    // (no node counts for a last level of more than kScanChunk nodes: its
    // node tables would take the plan kernels, and its pass reads none)
    a.ones_next = (i + 1 < l && !(i + 2 == l && (2ull << i) > kScanChunk))
                      ? reinterpret_cast<unsigned long long *>(w + j.ws_ones) + ones_offset(i + 1)
                      : nullptr;
    a.nodes_next = 2ull << i;
    a.slots_next = level_slots(i + 1);
    a.n = j.n;
    a.words = j.words;
    a.rank_entries = j.rank_entries;
    a.rank_stride = j.rank_stride;
    a.ntiles = j.ntiles;
    a.levels = l;
    a.level = i;
    a.symmask = (uint32_t)((1ull << l) - 1);
    a.matrix = 0;
    a.zeros = nullptr;
    a.digits = nullptr;
    a.dwords = 0;
    a.dsh = 0;
    a.bits_next = nullptr;
    a.n_out = j.n;
    a.fold_own = a.fold_ovf = nullptr;
    a.fold_ovf_n = nullptr;
    a.fold_ovf_cap = 0;
    a.fold_status = nullptr;
    a.anc_start = nullptr;
    a.tile_anc = nullptr;
    return a;
}

__device__ __forceinline__ PrepArgs job_prep(const BatchJob &j, uint32_t i) {
    PrepArgs p;
    uint8_t *w = j.work;
    p.tile_ones = reinterpret_cast<const uint32_t *>(w + j.ws_tile_ones) + (uint64_t)i * tile_stride(j.ntiles);
    p.supsum = reinterpret_cast<unsigned long long *>(w + j.ws_supsum);
    p.sup = reinterpret_cast<unsigned long long *>(w + j.ws_sup) + (uint64_t)i * j.nsup;
    p.ntiles = j.ntiles;
    p.nsup = j.nsup;
    uint64_t *start = reinterpret_cast<uint64_t *>(w + j.ws_start);
    p.plan.start = start + start_offset(i);
    p.plan.ones = reinterpret_cast<const unsigned long long *>(w + j.ws_ones) + ones_offset(i);
    p.plan.zo = reinterpret_cast<ulonglong2 *>(w + j.ws_zo) + zo_offset(i);
    p.plan.start_next = (i + 1 < j.levels) ? start + start_offset(i + 1) : nullptr;
    p.plan.partials = reinterpret_cast<uint64_t *>(w + j.ws_partials);
    p.plan.nodes = 1ull << i;
    p.plan.slots = level_slots(i);
    p.plan.n = j.n;
    p.plan.matrix = 0;
    p.plan.shift = 0;
    p.plan_here = (p.plan.nodes > kScanChunk) ? 0u : 1u;  // larger levels: the k_batch_plan_* kernels
    p.sums_here = 0;                                       // (k_batch_supsum runs for every level)
    return p;
}

__device__ __forceinline__ IngestArgs job_ingest(const BatchJob &j) {
    IngestArgs a;
    uint8_t *w = j.work;
    a.S = j.S;
    a.tile_ones0 = j.levels ? reinterpret_cast<uint32_t *>(w + j.ws_tile_ones) : nullptr;
    a.ones0 = reinterpret_cast<unsigned long long *>(w + j.ws_ones);
    a.start0 = j.levels ? reinterpret_cast<uint64_t *>(w + j.ws_start) : nullptr;
    a.tree_status = reinterpret_cast<uint32_t *>(j.tree);
    a.n = j.n;
    a.ntiles = j.ntiles;
    a.tiles_per_block = kWaves;
    a.slots0 = level_slots(0);
    a.sigma = j.sigma;
    a.check = j.check;
    a.msb = j.levels ? j.levels - 1 : 0;
    a.zero_g = nullptr;
    a.zero_granules = 0;
    return a;
}

// Workgroup j: fill the maps of sequence j, then clear its control area and
// tree status (and, for an empty sequence, its rank directories).
// Workgroups [g * parts, (g + 1) * parts) set up sequence g: its block
// maps, zeroed counters and status word.
__global__ __launch_bounds__(kThreads) void k_batch_setup(BatchClass c, uint32_t parts) {
    const uint32_t q = blockIdx.x / parts, part = blockIdx.x % parts;
    const BatchJob &j = c.jobs[q];
    const uint64_t first = (uint64_t)part * kThreads + threadIdx.x, stride = (uint64_t)parts * kThreads;
    const uint64_t nb = ceil_div(j.ntiles, kWaves);
    for (uint64_t b = first; b < nb; b += stride) c.blk_map[j.blk_base + b] = q;
    for (uint64_t b = first; b < j.nsup; b += stride) c.sup_map[j.sup_base + b] = q;
    uint4 *ctrl = reinterpret_cast<uint4 *>(j.work + j.ws_ctrl);  // 256-byte aligned and sized
    for (uint64_t k = first; k < j.ws_ctrl_bytes / 16; k += stride) ctrl[k] = make_uint4(0, 0, 0, 0);
    if (j.n == 0) {
        uint64_t *r = reinterpret_cast<uint64_t *>(j.tree + j.tree_ranks_off);
        for (uint64_t k = first; k < (uint64_t)j.levels * j.rank_stride; k += stride) r[k] = 0;
    }
    if (part == 0 && threadIdx.x == 0) *reinterpret_cast<uint32_t *>(j.tree) = 0;
}

template <int W, int B>
__global__ __launch_bounds__(kThreads) void k_batch_ingest(BatchClass c) {
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const BatchJob &j = c.jobs[c.blk_map[blockIdx.x]];
    const uint64_t blk = blockIdx.x - j.blk_base;
    const IngestArgs a = job_ingest(j);
    if (blk == 0 && threadIdx.x == 0 && a.start0) {
        a.start0[0] = 0;
        a.start0[1] = a.n;
    }
    const uint64_t t = blk * kWaves + wv;
    if (t >= j.ntiles) return;  // whole wave
    bool bad = false;
    uint4 raw[B / 16];
    const int nval = load_lane<W, B>(a.S, t * tile_syms(W, B) + (uint64_t)(threadIdx.x & 63) * (B / W), a.n, raw);
    const uint32_t ones = ingest_tile<W, B>(a, t, raw, nval, bad);
    ingest_finish(a, bad, ones, t);
}

__global__ __launch_bounds__(kThreads) void k_batch_supsum(BatchClass c, uint32_t level) {
    const BatchJob &j = c.jobs[c.sup_map[blockIdx.x]];
    const uint32_t *tile_ones =
        reinterpret_cast<const uint32_t *>(j.work + j.ws_tile_ones) + (uint64_t)level * tile_stride(j.ntiles);
    supsum_one(tile_ones, j.ntiles, blockIdx.x - j.sup_base, reinterpret_cast<unsigned long long *>(j.work + j.ws_supsum));
}

__global__ __launch_bounds__(kThreads) void k_batch_prep(BatchClass c, uint32_t level) {
    prep_level(job_prep(c.jobs[blockIdx.x], level));
}

// Node tables of levels above kScanChunk nodes, chunks of every active
// sequence side by side: workgroup b serves sequence b / cpj, chunk b % cpj
// (every sequence has 2^level nodes, so cpj chunks, at this level).
// (a sequence's last level needs no node tables: its pass writes only its
// bitmap and directory)
__global__ __launch_bounds__(kThreads) void k_batch_plan_reduce(BatchClass c, uint32_t level, uint32_t cpj) {
    const BatchJob &j = c.jobs[blockIdx.x / cpj];
    if (level + 1 == j.levels) return;
    const PrepArgs p = job_prep(j, level);
    plan_reduce_chunk(p.plan, blockIdx.x % cpj);
}

__global__ __launch_bounds__(kThreads) void k_batch_plan_partials(BatchClass c, uint32_t level, uint32_t cpj) {
    const BatchJob &j = c.jobs[blockIdx.x];
    if (level + 1 == j.levels) return;
    const PrepArgs p = job_prep(j, level);
    plan_scan_partials(p.plan, cpj);
}

__global__ __launch_bounds__(kThreads) void k_batch_plan_apply(BatchClass c, uint32_t level, uint32_t cpj) {
    const BatchJob &j = c.jobs[blockIdx.x / cpj];
    if (level + 1 == j.levels) return;
    const PrepArgs p = job_prep(j, level);
    const uint64_t b = blockIdx.x % cpj;
    plan_chunk(p.plan, p.plan.ones + b * kScanChunk, b * kScanChunk, p.plan.partials[b]);
}

template <int W, int B, bool M>
__global__ __launch_bounds__(kThreads) void k_batch_level(BatchClass c, uint32_t level) {
    __shared__ __align__(16) uint8_t s_all[kWaves * level_wave_bytes<W, B, M, true>()];
    __shared__ SplitRec s_rec[kWaves];
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const BatchJob &j = c.jobs[c.blk_map[blockIdx.x]];
    const uint64_t t0 = (blockIdx.x - j.blk_base) * kWaves;
    const LevelArgs a = job_level(j, level);
    if ((threadIdx.x & 63) < 4) s_rec[wv].cnt[threadIdx.x & 63] = 0;
    if (t0 + wv < j.ntiles)
        level_tile<W, B, W, M, true, B / W, true>(a, t0 + wv, s_all + wv * level_wave_bytes<W, B, M, true>(),
                                                  &s_rec[wv]);
    flush_split_recs<true>(a, s_rec, t0);
}

}  // namespace

// ------------------------------------------------------------- launchers --

static inline uint32_t grid_for(uint64_t items, uint64_t per_block, uint32_t cap) {
    uint64_t g = ceil_div(items, per_block);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

hipError_t launch_zero(void *p, uint64_t bytes, uint32_t *tree_status, uint64_t *p2, uint64_t count2, hipStream_t s) {
    const uint64_t words = bytes / 8;
    const uint64_t items = (words > count2 ? words : count2) / 2 + 1;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(items, 256, 4096)), dim3(256), 0, s, (uint64_t *)p, words,
                       tree_status, p2, count2);
    return hipGetLastError();
}

// ------------------------------------------------ folded last level -----
// One thread per granule record of the folded pass (two per tile, then the
// direct path's): the granule's 16 symbols are in T_{l-1} at its positions
// (stored there by the runs that share it), and its 16 bits are written
// once.  Every granule below n is written either by the pass (a whole chunk)
// or here (exactly one record names it: the run holding its first position).
__global__ __launch_bounds__(kThreads) void k_fold_stitch(StitchArgs a) {
    const uint64_t k = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    uint64_t g = ~0ull;
    if (k < a.nown) {
        g = a.own[k];
    } else {
        const uint64_t o = k - a.nown, m = *a.ovf_n;
        if (o < m && o < a.ovf_cap) g = a.ovf[o];
    }
    if (g == ~0ull) return;
    const uint64_t p = g * 16;
    const uint4 v = *reinterpret_cast<const uint4 *>(a.t + p);  // inside the n-byte (256-rounded) buffer
    uint32_t bits = chunk_bits16(v, a.sh);
    if (p + 16 > a.n) bits &= (1u << (uint32_t)(a.n - p)) - 1u;
    a.bits16[g] = (uint16_t)bits;
    note_write(&a.bits16[g], 2);
}

// ------------------------------------------------ directory of a bitmap ---
// Used for the last level when its bitmap comes out of the pass before it:
// k_bitdir_blocks scans the popcounts of kBitDirBlocks 512-bit blocks per
// workgroup, k_bitdir_fix scans the workgroup sums (one workgroup) and writes
// the total and the padding, k_bitdir_apply adds each workgroup's base.

__global__ __launch_bounds__(kThreads) void k_bitdir_blocks(BitDirArgs a) {
    __shared__ unsigned long long s_w[kWaves];
    static_assert(kBitDirBlocks == kThreads, "one block per thread");
    const uint64_t blk = (uint64_t)blockIdx.x * kBitDirBlocks + threadIdx.x;
    unsigned long long c = 0;
    if (blk < a.nblk) {
        const uint4 *p = reinterpret_cast<const uint4 *>(a.bits + blk * 8);
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const uint4 v = p[q];
            c += (unsigned long long)(__popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w));
        }
    }
    unsigned long long tot;
    const unsigned long long ex = block_excl_scan64(c, s_w, &tot);
    if (blk < a.nblk) a.ranks[blk] = ex;
    if (threadIdx.x == 0) a.wsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kThreads) void k_bitdir_fix(BitDirArgs a) {
    __shared__ unsigned long long s_w[kWaves];
    const uint64_t per = (a.nwg + kThreads - 1) / kThreads;
    const uint64_t k0 = (uint64_t)threadIdx.x * per;
    unsigned long long sum = 0;
    for (uint64_t k = k0; k < k0 + per && k < a.nwg; k++) sum += a.wsum[k];
    unsigned long long tot;
    unsigned long long off = block_excl_scan64(sum, s_w, &tot);
    for (uint64_t k = k0; k < k0 + per && k < a.nwg; k++) {
        const unsigned long long v = a.wsum[k];
        a.wsum[k] = off;
        off += v;
    }
    for (uint64_t k = a.nblk + threadIdx.x; k < a.rank_stride; k += kThreads) a.ranks[k] = (k == a.nblk) ? tot : 0ull;
}

__global__ __launch_bounds__(kThreads) void k_bitdir_apply(BitDirArgs a) {
    const uint64_t blk = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (blk < a.nblk) a.ranks[blk] += a.wsum[blk / kBitDirBlocks];
}

// Short bitmaps (at most 8 * kBitDirBlocks blocks): the whole directory in
// one workgroup, each thread a run of consecutive blocks.
constexpr uint64_t kBitDirSmallPer = 8;
__global__ __launch_bounds__(kThreads) void k_bitdir_small(BitDirArgs a) {
    __shared__ unsigned long long s_w[kWaves];
    const uint64_t per = (a.nblk + kThreads - 1) / kThreads;  // <= kBitDirSmallPer
    const uint64_t b0 = (uint64_t)threadIdx.x * per;
    uint32_t c[kBitDirSmallPer];
    unsigned long long sum = 0;
#pragma unroll
    for (uint64_t q = 0; q < kBitDirSmallPer; q++) {
        c[q] = 0;
        if (q < per && b0 + q < a.nblk) {
            const uint4 *p = reinterpret_cast<const uint4 *>(a.bits + (b0 + q) * 8);
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint4 v = p[j];
                c[q] += (uint32_t)(__popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w));
            }
        }
        sum += c[q];
    }
    unsigned long long tot;
    unsigned long long off = block_excl_scan64(sum, s_w, &tot);
#pragma unroll
    for (uint64_t q = 0; q < kBitDirSmallPer; q++) {
        if (q < per && b0 + q < a.nblk) a.ranks[b0 + q] = off;
        off += c[q];
    }
    for (uint64_t k = a.nblk + threadIdx.x; k < a.rank_stride; k += kThreads) a.ranks[k] = (k == a.nblk) ? tot : 0ull;
}

hipError_t launch_fold_stitch(const StitchArgs &a, hipStream_t s) {
    const uint64_t items = a.nown + a.ovf_cap;
    if (items == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fold_stitch, dim3((uint32_t)ceil_div(items, kThreads)), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bitdir(const BitDirArgs &a, hipStream_t s) {
    hipError_t err;
    if (a.nblk <= kBitDirSmallPer * kThreads) {
        hipLaunchKernelGGL(k_bitdir_small, dim3(1), dim3(kThreads), 0, s, a);
        return hipGetLastError();
    }
    if (a.nblk) {
        hipLaunchKernelGGL(k_bitdir_blocks, dim3((uint32_t)a.nwg), dim3(kThreads), 0, s, a);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    hipLaunchKernelGGL(k_bitdir_fix, dim3(1), dim3(kThreads), 0, s, a);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (a.nblk) {
        hipLaunchKernelGGL(k_bitdir_apply, dim3((uint32_t)ceil_div(a.nblk, kThreads)), dim3(kThreads), 0, s, a);
        err = hipGetLastError();
    }
    return err;
}

// Launch KERNEL<width, lane_bytes> (every valid pair is instantiated).
#define WT_LAUNCH_WB(KERNEL, W_, LB_, GRID, ...)                                                         \
    do {                                                                                               \
        switch ((W_) * 1000 + (LB_)) {                                                                 \
            case 1032: hipLaunchKernelGGL((KERNEL<1, 32>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;  \
            case 1064: hipLaunchKernelGGL((KERNEL<1, 64>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;  \
            case 2032: hipLaunchKernelGGL((KERNEL<2, 32>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;  \
            case 2064: hipLaunchKernelGGL((KERNEL<2, 64>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;  \
            case 2128: hipLaunchKernelGGL((KERNEL<2, 128>), GRID, dim3(kThreads), 0, __VA_ARGS__); break; \
            case 4032: hipLaunchKernelGGL((KERNEL<4, 32>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;  \
            case 4064: hipLaunchKernelGGL((KERNEL<4, 64>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;  \
            case 4128: hipLaunchKernelGGL((KERNEL<4, 128>), GRID, dim3(kThreads), 0, __VA_ARGS__); break; \
            default: return hipErrorInvalidValue;                                                      \
        }                                                                                              \
    } while (0)

// Launch KERNEL<width, lane_bytes, multi> (level passes: with or without
// the staged split of tiles spanning a few nodes).
#define WT_LAUNCH_WBM(KERNEL, W_, LB_, M_, GRID, ...)                                                    \
    do {                                                                                                \
        switch ((W_) * 10000 + (LB_) * 10 + ((M_) ? 1 : 0)) {                                          \
            case 10320: hipLaunchKernelGGL((KERNEL<1, 32, false>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;  \
            case 10321: hipLaunchKernelGGL((KERNEL<1, 32, true>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;   \
            case 10640: hipLaunchKernelGGL((KERNEL<1, 64, false>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;  \
            case 10641: hipLaunchKernelGGL((KERNEL<1, 64, true>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;   \
            case 20320: hipLaunchKernelGGL((KERNEL<2, 32, false>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;  \
            case 20321: hipLaunchKernelGGL((KERNEL<2, 32, true>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;   \
            case 20640: hipLaunchKernelGGL((KERNEL<2, 64, false>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;  \
            case 20641: hipLaunchKernelGGL((KERNEL<2, 64, true>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;   \
            case 21280: hipLaunchKernelGGL((KERNEL<2, 128, false>), GRID, dim3(kThreads), 0, __VA_ARGS__); break; \
            case 21281: hipLaunchKernelGGL((KERNEL<2, 128, true>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;  \
            case 40320: hipLaunchKernelGGL((KERNEL<4, 32, false>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;  \
            case 40321: hipLaunchKernelGGL((KERNEL<4, 32, true>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;   \
            case 40640: hipLaunchKernelGGL((KERNEL<4, 64, false>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;  \
            case 40641: hipLaunchKernelGGL((KERNEL<4, 64, true>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;   \
            case 41280: hipLaunchKernelGGL((KERNEL<4, 128, false>), GRID, dim3(kThreads), 0, __VA_ARGS__); break; \
            case 41281: hipLaunchKernelGGL((KERNEL<4, 128, true>), GRID, dim3(kThreads), 0, __VA_ARGS__); break;  \
            default: return hipErrorInvalidValue;                                                       \
        }                                                                                               \
    } while (0)

hipError_t launch_ingest(const IngestArgs &a, uint32_t width, uint32_t lane_bytes, hipStream_t s) {
    const dim3 g((uint32_t)ceil_div(a.ntiles, a.tiles_per_block));
    WT_LAUNCH_WB(k_ingest, width, lane_bytes, g, s, a);
    return hipGetLastError();
}

hipError_t launch_prep(const PrepArgs &a, hipStream_t s) {
    if (!a.sums_here) hipLaunchKernelGGL(k_supsum, dim3((uint32_t)a.nsup), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_prep, dim3(1), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_plan(const PlanArgs &a, hipStream_t s) {
    const uint64_t nb = ceil_div(a.nodes, kScanChunk);
    hipLaunchKernelGGL(k_plan_reduce, dim3((uint32_t)nb), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_plan_partials, dim3(1), dim3(kThreads), 0, s, a, nb);
    hipLaunchKernelGGL(k_plan_apply, dim3((uint32_t)nb), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_level(const LevelArgs &a, uint32_t width, uint32_t lane_bytes, bool multi, uint32_t out_width,
                        uint32_t out_lane_bytes, hipStream_t s) {
    const dim3 g((uint32_t)ceil_div(a.ntiles, kWaves));
    if (out_width == width) {
        if (out_lane_bytes != lane_bytes) return hipErrorInvalidValue;
        WT_LAUNCH_WBM(k_level, width, lane_bytes, multi, g, s, a);
        return hipGetLastError();
    }
    if (multi || 2 * out_width != width) return hipErrorInvalidValue;
    const dim3 b(kThreads);
    switch ((width << 16) | (lane_bytes << 8) | out_lane_bytes) {
        case (4 << 16) | (64 << 8) | 32: hipLaunchKernelGGL((k_level_narrow<4, 64, 32>), g, b, 0, s, a); break;
        case (4 << 16) | (64 << 8) | 64: hipLaunchKernelGGL((k_level_narrow<4, 64, 64>), g, b, 0, s, a); break;
        case (4 << 16) | (128 << 8) | 64: hipLaunchKernelGGL((k_level_narrow<4, 128, 64>), g, b, 0, s, a); break;
        case (2 << 16) | (64 << 8) | 32: hipLaunchKernelGGL((k_level_narrow<2, 64, 32>), g, b, 0, s, a); break;
        case (2 << 16) | (64 << 8) | 64: hipLaunchKernelGGL((k_level_narrow<2, 64, 64>), g, b, 0, s, a); break;
        case (2 << 16) | (128 << 8) | 64: hipLaunchKernelGGL((k_level_narrow<2, 128, 64>), g, b, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tile_anchor(const AnchorArgs &a, hipStream_t s) {
    if (a.ntiles == 0 || a.nodes == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_anchor, dim3((uint32_t)ceil_div(a.ntiles, kThreads)), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_batch_setup(const BatchClass &c, uint64_t max_ctrl_bytes, hipStream_t s) {
    // about 256 KB of counters per workgroup for the largest sequence
    uint64_t parts = max_ctrl_bytes >> 18;
    parts = parts < 1 ? 1 : (parts > 64 ? 64 : parts);
    hipLaunchKernelGGL(k_batch_setup, dim3(c.njobs * (uint32_t)parts), dim3(kThreads), 0, s, c, (uint32_t)parts);
    return hipGetLastError();
}

hipError_t launch_batch_ingest(const BatchClass &c, uint32_t width, uint32_t lane_bytes, uint64_t blocks,
                               hipStream_t s) {
    if (blocks == 0) return hipSuccess;
    WT_LAUNCH_WB(k_batch_ingest, width, lane_bytes, dim3((uint32_t)blocks), s, c);
    return hipGetLastError();
}

// Level `level` of the first `active` sequences of the class: superchunk
// sums, prefixes and node tables, then the level pass.
hipError_t launch_batch_level(const BatchClass &c, uint32_t width, uint32_t lane_bytes, bool multi, uint32_t level,
                              uint32_t active, uint64_t blocks, uint64_t sups, hipStream_t s) {
    if (active == 0) return hipSuccess;
    if ((1ull << level) > kScanChunk) {
        const uint32_t cpj = (uint32_t)((1ull << level) / kScanChunk);
        hipLaunchKernelGGL(k_batch_plan_reduce, dim3(active * cpj), dim3(kThreads), 0, s, c, level, cpj);
        hipLaunchKernelGGL(k_batch_plan_partials, dim3(active), dim3(kThreads), 0, s, c, level, cpj);
        hipLaunchKernelGGL(k_batch_plan_apply, dim3(active * cpj), dim3(kThreads), 0, s, c, level, cpj);
    }
    if (sups) hipLaunchKernelGGL(k_batch_supsum, dim3((uint32_t)sups), dim3(kThreads), 0, s, c, level);
    hipLaunchKernelGGL(k_batch_prep, dim3(active), dim3(kThreads), 0, s, c, level);
    if (blocks) WT_LAUNCH_WBM(k_batch_level, width, lane_bytes, multi, dim3((uint32_t)blocks), s, c, level);
    return hipGetLastError();
}

#ifdef WT_WRITE_CHECK
hipError_t write_check_build(uint32_t *cnt, uint64_t base, uint64_t bytes) {
    return set_write_check_here(cnt, base, bytes);
}
#endif

}  // namespace wt
