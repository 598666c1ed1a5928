// Batched access / rank / select on a built pointerless wavelet tree (and
// on the wavelet-matrix and 4-ary variants).
//
// Section 2.2: queries walk the tree top-down; with one bitmap per level the
// current node is a range [b, e) of the level, its left child is the first
// zeros(b, e) positions of the same range at the next level and its right
// child the rest, so every step needs rank on the level bitmap.  rank uses
// the level's directory of absolute counts at multiples of 512 positions
// plus popcounts of at most eight words; select binary-searches the
// directory, then scans words.  One thread answers one query.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wt_internal.h"

namespace wt {

namespace {

struct Level {
    const uint64_t *B, *R;
};

__device__ __forceinline__ Level level_of(const TreeView &t, uint32_t k) {
    return Level{t.bits + (uint64_t)k * t.words, t.ranks + (uint64_t)k * t.rank_stride};
}

// ones in positions [0, p), 0 <= p <= n
__device__ __forceinline__ uint64_t rank1(const Level &L, uint64_t p) {
    const uint64_t k = p >> 9;
    uint64_t r = L.R[k];
    const uint64_t w1 = p >> 6;
    for (uint64_t w = k * 8; w < w1; w++) r += __popcll(L.B[w]);
    if (p & 63) r += __popcll(L.B[w1] & ((1ull << (p & 63)) - 1ull));
    return r;
}

__device__ __forceinline__ uint32_t select_in_word(uint64_t x, uint32_t r) {
    for (uint32_t q = 0; q < r; q++) x &= x - 1;  // drop the r lowest set bits
    return (uint32_t)__builtin_ctzll(x);
}

// position of the m-th (1-based) one; requires 1 <= m <= ones of the level
__device__ uint64_t select1(const Level &L, uint64_t K, uint64_t nw, uint64_t m) {
    uint64_t lo = 0, hi = K - 1;
    while (lo < hi) {  // largest k with R[k] < m (R[0] = 0 < m)
        const uint64_t mid = (lo + hi + 1) / 2;
        if (L.R[mid] < m) lo = mid; else hi = mid - 1;
    }
    uint64_t r = L.R[lo], w = lo * 8;
    while (w < nw) {  // nw = words holding positions < n
        const uint64_t pc = __popcll(L.B[w]);
        if (r + pc >= m) break;
        r += pc;
        w++;
    }
    if (w >= nw) return ~0ull;  // only for a corrupted directory
    return w * 64 + select_in_word(L.B[w], (uint32_t)(m - r - 1));
}

// position of the m-th (1-based) zero; requires 1 <= m <= zeros in [0, n)
__device__ uint64_t select0(const Level &L, uint64_t K, uint64_t n, uint64_t m) {
    const uint64_t nw = (n + 63) / 64;
    uint64_t lo = 0, hi = K - 1;
    while (lo < hi) {  // largest k with zeros before min(512k, n) < m
        const uint64_t mid = (lo + hi + 1) / 2;
        const uint64_t p = mid * 512 < n ? mid * 512 : n;
        if (p - L.R[mid] < m) lo = mid; else hi = mid - 1;
    }
    uint64_t r = lo * 512 - L.R[lo], w = lo * 8;
    while (w < nw) {
        const uint64_t pc = __popcll(~L.B[w]);
        if (r + pc >= m) break;
        r += pc;
        w++;
    }
    if (w >= nw) return ~0ull;
    return w * 64 + select_in_word(~L.B[w], (uint32_t)(m - r - 1));
}

// Wavelet matrix (one node per level, z_k zeros at level k): reading bit b
// at position p of level k, the walk continues at rank0(p) for b = 0 and at
// z_k + rank1(p) for b = 1.
__device__ uint32_t matrix_access(const TreeView &t, uint64_t i) {
    uint64_t p = i;
    uint32_t s = 0;
    for (uint32_t k = 0; k < t.levels; k++) {
        const Level L = level_of(t, k);
        const uint32_t bit = (uint32_t)((L.B[p >> 6] >> (p & 63)) & 1ull);
        const uint64_t r1 = rank1(L, p);
        p = bit ? t.zeros[k] + r1 : p - r1;
        s = (s << 1) | bit;
        if (p >= t.n) return 0xFFFFFFFEu;  // corrupted matrix only
    }
    return s;
}

// The range [b, e) of the symbols c among positions [0, i), at the bottom.
__device__ void matrix_range(const TreeView &t, uint32_t c, uint64_t i, uint64_t &b, uint64_t &e) {
    b = 0;
    e = i;
    for (uint32_t k = 0; k < t.levels; k++) {
        const Level L = level_of(t, k);
        const uint64_t rb = rank1(L, b), re = rank1(L, e);
        if ((c >> (t.levels - 1 - k)) & 1u) { b = t.zeros[k] + rb; e = t.zeros[k] + re; }
        else                                 { b = b - rb; e = e - re; }
    }
}

__device__ uint64_t matrix_select(const TreeView &t, uint32_t c, uint64_t j) {
    uint64_t b, e;
    matrix_range(t, c, t.n, b, e);
    if (j == 0 || j > e - b) return ~0ull;
    uint64_t p = b + j - 1;
    for (uint32_t k = t.levels; k-- > 0;) {  // back up: the (t+1)-th zero / one of level k
        const Level L = level_of(t, k);
        if ((c >> (t.levels - 1 - k)) & 1u) p = select1(L, t.rank_entries, (t.n + 63) / 64, p - t.zeros[k] + 1);
        else p = select0(L, t.rank_entries, t.n, p + 1);
        if (p >= t.n) return ~0ull;
    }
    return p;
}

// 4-ary tree: level k lists 2-bit digits (32 per word); the child of digit
// d of node [b, e) occupies, at the next level, the part of [b, e) after the
// digits smaller than d, as long as the digits equal to d.  Counts come from
// the per-digit directory plus popcounts over the two bit planes of at most
// fifteen words.
constexpr uint64_t kEvenBits = 0x5555555555555555ull;

struct DLevel {
    const uint64_t *D, *R;  // digit words; directory entries of four counts
};

struct DCounts {
    uint64_t c[4];
};

__device__ __forceinline__ DLevel dlevel_of(const TreeView &t, uint32_t k) {
    return DLevel{t.digits + (uint64_t)k * t.dwords, t.dir + (uint64_t)k * t.rank_stride * 4};
}

__device__ __forceinline__ uint64_t pick(const DCounts &x, uint32_t d) {
    return d == 0 ? x.c[0] : (d == 1 ? x.c[1] : (d == 2 ? x.c[2] : x.c[3]));
}

__device__ __forceinline__ uint32_t digit_at(const DLevel &L, uint64_t p) {
    return (uint32_t)((L.D[p >> 5] >> (2 * (p & 31))) & 3ull);
}

// even-bit mask of the digits equal to d in word w
__device__ __forceinline__ uint64_t digit_mask(uint64_t w, uint32_t d) {
    const uint64_t lo = w & kEvenBits, hi = (w >> 1) & kEvenBits;
    return ((d & 1) ? lo : (~lo & kEvenBits)) & ((d & 2) ? hi : (~hi & kEvenBits));
}

// counts of every digit in positions [0, p), 0 <= p <= n
__device__ DCounts rank_digits(const DLevel &L, uint64_t p) {
    const uint64_t k = p >> 9, w1 = p >> 5;
    uint64_t c1 = 0, c2 = 0, c3 = 0;
    for (uint64_t w = k * 16; w <= w1; w++) {
        if (w == w1 && (p & 31) == 0) break;
        uint64_t x = L.D[w];
        if (w == w1) x &= (1ull << (2 * (p & 31))) - 1ull;
        const uint64_t lo = x & kEvenBits, hi = (x >> 1) & kEvenBits;
        c1 += __popcll(lo & ~hi);
        c2 += __popcll(hi & ~lo);
        c3 += __popcll(lo & hi);
    }
    const uint64_t *E = L.R + k * 4;
    DCounts r;
    r.c[0] = E[0] + (p - k * 512) - c1 - c2 - c3;
    r.c[1] = E[1] + c1;
    r.c[2] = E[2] + c2;
    r.c[3] = E[3] + c3;
    return r;
}

// position of the m-th (1-based) digit d of the level; requires 1 <= m <=
// the digits d in [0, n)
__device__ uint64_t select_digit(const DLevel &L, uint64_t K, uint64_t n, uint32_t d, uint64_t m) {
    uint64_t lo = 0, hi = K - 1;
    while (lo < hi) {  // largest k with R[k][d] < m (R[0][d] = 0 < m)
        const uint64_t mid = (lo + hi + 1) / 2;
        if (L.R[mid * 4 + d] < m) lo = mid; else hi = mid - 1;
    }
    uint64_t r = L.R[lo * 4 + d], w = lo * 16;
    const uint64_t nw = (n + 31) / 32;
    while (w < nw) {
        uint64_t mk = digit_mask(L.D[w], d);
        if (w * 32 + 32 > n) mk &= (1ull << (2 * (n - w * 32))) - 1ull;  // digits past n are padding
        const uint64_t pc = __popcll(mk);
        if (r + pc >= m) return w * 32 + select_in_word(mk, (uint32_t)(m - r - 1)) / 2;
        r += pc;
        w++;
    }
    return ~0ull;  // only for a corrupted directory
}

__device__ uint32_t access4(const TreeView &t, uint64_t i) {
    uint64_t b = 0, e = t.n, p = i;
    uint32_t s = 0;
    for (uint32_t k = 0; k < t.levels4; k++) {
        const DLevel L = dlevel_of(t, k);
        const uint32_t d = digit_at(L, p);
        const DCounts rb = rank_digits(L, b), re = rank_digits(L, e), rp = rank_digits(L, p);
        uint64_t below = 0;
        for (uint32_t x = 0; x < d; x++) below += pick(re, x) - pick(rb, x);
        const uint64_t nb = b + below;
        e = nb + (pick(re, d) - pick(rb, d));
        p = nb + (pick(rp, d) - pick(rb, d));
        b = nb;
        s = (s << 2) | d;
        if (p >= e || e > t.n) return 0xFFFFFFFEu;  // corrupted tree only
    }
    return s;
}

__device__ uint64_t rank4(const TreeView &t, uint32_t c, uint64_t i) {
    uint64_t b = 0, e = t.n, p = i;
    for (uint32_t k = 0; k < t.levels4; k++) {
        const DLevel L = dlevel_of(t, k);
        const uint32_t d = (c >> (2 * (t.levels4 - 1 - k))) & 3u;
        const DCounts rb = rank_digits(L, b), re = rank_digits(L, e), rp = rank_digits(L, p);
        uint64_t below = 0;
        for (uint32_t x = 0; x < d; x++) below += pick(re, x) - pick(rb, x);
        const uint64_t nb = b + below;
        e = nb + (pick(re, d) - pick(rb, d));
        p = nb + (pick(rp, d) - pick(rb, d));
        b = nb;
        if (p > e || e > t.n) return ~1ull;  // corrupted tree only
    }
    return p - b;
}

__device__ uint64_t select4(const TreeView &t, uint32_t c, uint64_t j) {
    uint64_t bs[16];
    uint64_t b = 0, e = t.n;
    for (uint32_t k = 0; k < t.levels4; k++) {  // node ranges of c, top-down
        const DLevel L = dlevel_of(t, k);
        const uint32_t d = (c >> (2 * (t.levels4 - 1 - k))) & 3u;
        bs[k] = b;
        const DCounts rb = rank_digits(L, b), re = rank_digits(L, e);
        uint64_t below = 0;
        for (uint32_t x = 0; x < d; x++) below += pick(re, x) - pick(rb, x);
        b = b + below;
        e = b + (pick(re, d) - pick(rb, d));
        if (e > t.n) return ~1ull;  // corrupted tree only
    }
    if (j == 0 || j > e - b) return ~0ull;
    uint64_t idx = j - 1;
    for (uint32_t k = t.levels4; k-- > 0;) {  // bottom-up back to S
        const DLevel L = dlevel_of(t, k);
        const uint32_t d = (c >> (2 * (t.levels4 - 1 - k))) & 3u;
        const uint64_t bb = bs[k];
        const uint64_t pos = select_digit(L, t.rank_entries, t.n, d, pick(rank_digits(L, bb), d) + idx + 1);
        if (pos >= t.n) return ~0ull;
        idx = pos - bb;
    }
    return idx;
}

// Huffman-shaped tree: depth d holds the n_d symbols whose code is longer
// than d.  The walk keeps the plain coordinates of the level split over the
// left-aligned codes (a node's children occupy its range at the next
// depth, zeros first), where depth d starts at m_d = n - n_d: position P of
// an internal node is position P - m_d of depth d's bitmap.  A child whose
// first d + 1 code bits form a code of that length is a leaf (canonical
// codes of length l are first[l] .. first[l] + count[l] - 1).
__device__ __forceinline__ Level hlevel(const TreeView &t, uint32_t d) {
    return Level{reinterpret_cast<const uint64_t *>(t.hbase + t.huff->bits_off[d]),
                 reinterpret_cast<const uint64_t *>(t.hbase + t.huff->dir_off[d])};
}

__device__ uint32_t huff_access(const TreeView &t, uint64_t i) {
    const HuffMeta &m = *t.huff;
    if (m.levels == 0) return m.only;
    const uint32_t *syms = reinterpret_cast<const uint32_t *>(t.hbase + m.syms_off);
    uint64_t b = 0, e = m.n, p = i;
    uint32_t pre = 0;
    for (uint32_t d = 0; d < m.levels; d++) {
        const Level L = hlevel(t, d);
        const uint64_t md = m.n - m.size[d];
        const uint64_t rb = rank1(L, b - md), re = rank1(L, e - md), rp = rank1(L, p - md);
        const uint64_t zeros = (e - b) - (re - rb);
        const uint64_t q = p - md;
        const uint32_t bit = (uint32_t)((L.B[q >> 6] >> (q & 63)) & 1ull);
        uint64_t before;
        if (bit) { before = rp - rb; b = b + zeros; }
        else     { before = (p - b) - (rp - rb); e = b + zeros; }
        p = b + before;
        pre = 2 * pre + bit;
        const uint32_t len = d + 1;
        if (pre - m.first[len] < m.count[len]) return syms[m.start[len] + (pre - m.first[len])];
        if (p >= e) return 0xFFFFFFFEu;  // corrupted tree only
    }
    return 0xFFFFFFFEu;
}

__device__ uint64_t huff_rank(const TreeView &t, uint32_t c, uint64_t i) {
    const HuffMeta &m = *t.huff;
    if (m.levels == 0) return (c == m.only) ? i : 0;
    const uint32_t ent = reinterpret_cast<const uint32_t *>(t.hbase + m.code_off)[c];
    const uint32_t len = ent & 31u, code = ent >> 8;
    if (len == 0) return 0;
    uint64_t b = 0, e = m.n, p = i;
    for (uint32_t d = 0; d < len; d++) {
        const Level L = hlevel(t, d);
        const uint64_t md = m.n - m.size[d];
        const uint64_t rb = rank1(L, b - md), re = rank1(L, e - md), rp = rank1(L, p - md);
        const uint64_t zeros = (e - b) - (re - rb);
        if ((code >> (len - 1 - d)) & 1u) { p = b + zeros + (rp - rb); b = b + zeros; }
        else                              { p = p - (rp - rb); e = b + zeros; }
        if (p > e) return ~1ull;  // corrupted tree only
    }
    return p - b;
}

__device__ uint64_t huff_select(const TreeView &t, uint32_t c, uint64_t j) {
    const HuffMeta &m = *t.huff;
    if (m.levels == 0) return (c == m.only && j >= 1 && j <= m.n) ? j - 1 : ~0ull;
    const uint32_t ent = reinterpret_cast<const uint32_t *>(t.hbase + m.code_off)[c];
    const uint32_t len = ent & 31u, code = ent >> 8;
    if (len == 0) return ~0ull;
    uint64_t bs[kHuffMaxLevels + 1];
    uint64_t b = 0, e = m.n;
    for (uint32_t d = 0; d < len; d++) {  // node ranges of c, top-down
        const Level L = hlevel(t, d);
        const uint64_t md = m.n - m.size[d];
        bs[d] = b;
        const uint64_t rb = rank1(L, b - md), re = rank1(L, e - md);
        const uint64_t zeros = (e - b) - (re - rb);
        if ((code >> (len - 1 - d)) & 1u) b = b + zeros; else e = b + zeros;
        if (b > e) return ~1ull;  // corrupted tree only
    }
    if (j == 0 || j > e - b) return ~0ull;
    uint64_t idx = j - 1;  // index among the leaf's symbols
    for (uint32_t d = len; d-- > 0;) {  // bottom-up back to S
        const Level L = hlevel(t, d);
        const uint64_t md = m.n - m.size[d], nd = m.size[d];
        const uint64_t bb = bs[d];
        const uint64_t rb = rank1(L, bb - md);
        uint64_t q;
        if ((code >> (len - 1 - d)) & 1u) q = select1(L, m.dir_entries[d], (nd + 63) / 64, rb + idx + 1);
        else q = select0(L, m.dir_entries[d], nd, (bb - md - rb) + idx + 1);
        if (q >= nd) return ~0ull;
        idx = q + md - bb;
    }
    return idx;
}

// access(i): the symbol at position i (0xFFFFFFFF if i >= n).
__device__ uint32_t access_one(const TreeView &t, uint64_t i) {
    if (i >= t.n) return 0xFFFFFFFFu;
    if (t.huff) return huff_access(t, i);
    if (t.zeros) return matrix_access(t, i);
    if (t.digits) return access4(t, i);
    uint64_t b = 0, e = t.n, p = i;
    uint32_t s = 0;
    for (uint32_t k = 0; k < t.levels; k++) {
        const Level L = level_of(t, k);
        const uint64_t rb = rank1(L, b), re = rank1(L, e), rp = rank1(L, p);
        const uint64_t zeros = (e - b) - (re - rb);
        const uint32_t bit = (uint32_t)((L.B[p >> 6] >> (p & 63)) & 1ull);
        uint64_t before;
        if (bit) { before = rp - rb; b = b + zeros; }
        else     { before = (p - b) - (rp - rb); e = b + zeros; }
        p = b + before;
        s = (s << 1) | bit;
        if (p >= e || e > t.n) return 0xFFFFFFFEu;  // corrupted tree only
    }
    return s;
}

// rank(c, i): occurrences of c in S[0, i) (UINT64_MAX if c >= sigma or i > n).
__device__ uint64_t rank_one(const TreeView &t, uint32_t c, uint64_t i) {
    if (c >= t.sigma || i > t.n) return ~0ull;
    if (t.huff) return huff_rank(t, c, i);
    if (t.zeros) {
        uint64_t b, e;
        matrix_range(t, c, i, b, e);
        return e - b;
    }
    if (t.digits) return rank4(t, c, i);
    uint64_t b = 0, e = t.n, cnt = i;
    for (uint32_t k = 0; k < t.levels; k++) {
        const Level L = level_of(t, k);
        const uint64_t rb = rank1(L, b), re = rank1(L, e);
        const uint64_t zeros = (e - b) - (re - rb);
        const uint64_t ones_before = rank1(L, b + cnt) - rb;
        if ((c >> (t.levels - 1 - k)) & 1u) { cnt = ones_before; b = b + zeros; }
        else                                 { cnt = cnt - ones_before; e = b + zeros; }
        if (b + cnt > e || e > t.n) return ~1ull;  // corrupted tree only
    }
    return cnt;
}

// select(c, j): 0-based position of the j-th (1-based) c (UINT64_MAX if none).
__device__ uint64_t select_one(const TreeView &t, uint32_t c, uint64_t j) {
    if (c >= t.sigma) return ~0ull;
    if (t.huff) return huff_select(t, c, j);
    if (t.zeros) return matrix_select(t, c, j);
    if (t.digits) return select4(t, c, j);
    uint64_t bs[32];
    uint64_t b = 0, e = t.n;
    for (uint32_t k = 0; k < t.levels; k++) {  // node ranges of c, top-down
        const Level L = level_of(t, k);
        bs[k] = b;
        const uint64_t rb = rank1(L, b), re = rank1(L, e);
        const uint64_t zeros = (e - b) - (re - rb);
        if ((c >> (t.levels - 1 - k)) & 1u) b = b + zeros; else e = b + zeros;
        if (b > e || e > t.n) return ~1ull;  // corrupted tree only
    }
    if (j == 0 || j > e - b) return ~0ull;
    uint64_t idx = j - 1;
    for (uint32_t k = t.levels; k-- > 0;) {  // bottom-up back to S
        const Level L = level_of(t, k);
        const uint64_t bb = bs[k];
        const uint64_t rb = rank1(L, bb);
        uint64_t pos;
        if ((c >> (t.levels - 1 - k)) & 1u) pos = select1(L, t.rank_entries, (t.n + 63) / 64, rb + idx + 1);
        else pos = select0(L, t.rank_entries, t.n, (bb - rb) + idx + 1);
        if (pos >= t.n) return ~0ull;
        idx = pos - bb;
    }
    return idx;
}

__global__ void k_access(TreeView t, const uint64_t *qi, uint32_t *out, uint64_t m) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < m) out[q] = access_one(t, qi[q]);
}

__global__ void k_rank(TreeView t, const uint32_t *qc, const uint64_t *qi, uint64_t *out, uint64_t m) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < m) out[q] = rank_one(t, qc[q], qi[q]);
}

__global__ void k_select(TreeView t, const uint32_t *qc, const uint64_t *qj, uint64_t *out, uint64_t m) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < m) out[q] = select_one(t, qc[q], qj[q]);
}

// Mixed queries over many trees: query q asks tree views[tree[q]].
__global__ void k_query_multi(const TreeView *views, uint32_t ntrees, const uint32_t *tree, const uint8_t *kind,
                              const uint32_t *qc, const uint64_t *qx, uint64_t *out, uint64_t m) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const uint32_t ti = tree[q];
    if (ti >= ntrees) { out[q] = ~0ull; return; }
    const TreeView t = views[ti];
    switch (kind[q]) {
        case 0: {
            const uint32_t s = access_one(t, qx[q]);
            out[q] = (s == 0xFFFFFFFFu) ? ~0ull : (s == 0xFFFFFFFEu ? ~1ull : (uint64_t)s);
            break;
        }
        case 1: out[q] = rank_one(t, qc[q], qx[q]); break;
        case 2: out[q] = select_one(t, qc[q], qx[q]); break;
        default: out[q] = ~0ull;
    }
}

inline uint32_t blocks_for(uint64_t m) { return (uint32_t)((m + 255) / 256); }

}  // namespace

hipError_t launch_access(const TreeView &t, const uint64_t *i, uint32_t *sym, uint64_t m, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_access, dim3(blocks_for(m)), dim3(256), 0, s, t, i, sym, m);
    return hipGetLastError();
}

hipError_t launch_rank(const TreeView &t, const uint32_t *c, const uint64_t *i, uint64_t *r, uint64_t m,
                       hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rank, dim3(blocks_for(m)), dim3(256), 0, s, t, c, i, r, m);
    return hipGetLastError();
}

hipError_t launch_query_multi(const TreeView *d_views, uint32_t ntrees, const uint32_t *tree, const uint8_t *kind,
                              const uint32_t *c, const uint64_t *x, uint64_t *out, uint64_t m, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_query_multi, dim3(blocks_for(m)), dim3(256), 0, s, d_views, ntrees, tree, kind, c, x, out, m);
    return hipGetLastError();
}

hipError_t launch_select(const TreeView &t, const uint32_t *c, const uint64_t *j, uint64_t *pos, uint64_t m,
                         hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_select, dim3(blocks_for(m)), dim3(256), 0, s, t, c, j, pos, m);
    return hipGetLastError();
}

}  // namespace wt
