// Buffered construction of a sequence that is read in pieces (the extension
// of Algorithm dd to inputs that do not fit, Section 5): every buffer of S is
// built as a partial wavelet tree of its own, the node offsets of all
// partial trees are combined by prefix sums, and the partial bitmaps are
// concatenated into the final levels (Function mergeBA).
//
// Node offsets are kept per leaf.  Row q of the table C first receives the
// exclusive prefix, over leaf codes c in [0, 2^l], of buffer q's symbol
// counts (Hp_q; read off the partial build's last-level node tables), and is
// then turned into C_q[c] = sum over earlier buffers q' < q of Hp_q'[c], with
// row nbuf holding the prefix over all of S.  For node v of level i (leaves
// [v 2^k, (v+1) 2^k), k = l - i) and buffer q, with a = v 2^k, b = (v+1) 2^k:
//     source start in partial q   = Hp_q[a]              = C_{q+1}[a] - C_q[a]
//     run length                  = Hp_q[b] - Hp_q[a]
//     destination in the level    = C_nbuf[a] + C_q[b] - C_q[a]
// i.e. node v starts where all earlier nodes of every buffer end, and inside
// it the buffers follow each other in input order (the global offsets G of
// Algorithm dd).  Runs ordered by (v, q) have non-decreasing destinations
// and tile the level.
//
// The merge is written word by word rather than run by run: each thread owns
// one 64-bit word of the output, finds the run holding its first bit (from
// a per-span table of first runs), and ORs
// shifted pieces of the partial bitmaps into it.  Every word has a single
// writer, so the boundary-word atomics of mergeBA are not needed, and the
// popcounts of the words feed the rank directory in the same pass.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wt_check.h"
#include "wt_internal.h"

namespace wt {

namespace {

constexpr int kMT = 256;  // threads per workgroup of the merge kernels

// Exclusive scan of one u64 per thread over the workgroup (kMT threads).
__device__ __forceinline__ unsigned long long block_excl_scan(unsigned long long x, unsigned long long *s,
                                                              unsigned long long *total) {
    const int t = threadIdx.x;
    s[t] = x;
    __syncthreads();
    for (int d = 1; d < kMT; d <<= 1) {
        const unsigned long long y = (t >= d) ? s[t - d] : 0ull;
        __syncthreads();
        s[t] += y;
        __syncthreads();
    }
    const unsigned long long inc = s[t];
    *total = s[kMT - 1];
    __syncthreads();
    return inc - x;
}

// Row q of the offset table from partial build q: the exclusive prefix of
// the buffer's leaf counts.  Leaf 2v of the last level's node v starts where
// the node starts; leaf 2v+1 starts after the node's zeros, i.e. at the one
// base of the node (zo.x + zo.y).
__global__ __launch_bounds__(kMT) void k_leaf_prefix(const uint64_t *start_last, const ulonglong2 *zo_last,
                                                     uint64_t leaves, uint64_t nq, unsigned long long *row) {
    const uint64_t c = (uint64_t)blockIdx.x * kMT + threadIdx.x;
    if (c > leaves) return;
    unsigned long long v;
    if (c == leaves) {
        v = nq;
    } else if ((c & 1) == 0) {
        v = start_last[c >> 1];
    } else {
        const ulonglong2 z = zo_last[c >> 1];
        v = z.x + z.y;
    }
    row[c] = v;
}

// Column prefix over the buffers: C_q[c] = sum of Hp_q'[c] over q' < q, in
// place, and C_nbuf[c] = the sum over every buffer.
__global__ __launch_bounds__(kMT) void k_column_prefix(unsigned long long *C, uint32_t nbuf, uint64_t row) {
    const uint64_t c = (uint64_t)blockIdx.x * kMT + threadIdx.x;
    if (c >= row) return;
    unsigned long long acc = 0;
    for (uint32_t q = 0; q < nbuf; q++) {
        const unsigned long long t = C[(uint64_t)q * row + c];
        C[(uint64_t)q * row + c] = acc;
        acc += t;
    }
    C[(uint64_t)nbuf * row + c] = acc;
}

struct Run {
    uint64_t d0, d1, src;
    uint32_t q;
};

// Run r = v * nbuf + q of level i (k = l - i).
__device__ __forceinline__ Run run_at(const MergeArgs &a, uint32_t k, uint64_t r) {
    const uint64_t v = r / a.nbuf;
    const uint32_t q = (uint32_t)(r - v * a.nbuf);
    const uint64_t lo = v << k, hi = (v + 1) << k;
    const unsigned long long *cq = a.C + (uint64_t)q * a.row, *cn = cq + a.row;
    const unsigned long long base = a.C[(uint64_t)a.nbuf * a.row + lo];
    const unsigned long long qa = cq[lo], qb = cq[hi];
    Run x;
    x.src = cn[lo] - qa;
    x.d0 = base + qb - qa;
    x.d1 = x.d0 + ((cn[hi] - qb) - x.src);
    x.q = q;
    return x;
}

__device__ __forceinline__ uint64_t run_dst(const MergeArgs &a, uint32_t k, uint64_t r) {
    const uint64_t v = r / a.nbuf;
    const uint64_t q = r - v * a.nbuf;
    const uint64_t lo = v << k, hi = (v + 1) << k;
    return a.C[(uint64_t)a.nbuf * a.row + lo] + a.C[q * a.row + hi] - a.C[q * a.row + lo];
}

// The last run r in [lo, R) whose destination is <= p, given that run lo's
// is: gallop forward, then bisect.
__device__ __forceinline__ uint64_t find_run(const MergeArgs &a, uint32_t k, uint64_t R, uint64_t lo, uint64_t p) {
    uint64_t step = 1, hi = lo + 1;
    while (hi < R && run_dst(a, k, hi) <= p) {
        lo = hi;
        step <<= 1;
        hi = lo + step;
    }
    if (hi > R) hi = R;
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (run_dst(a, k, mid) <= p) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Words per merge thread.  A workgroup covers kMW = kMT * kWPT consecutive
// words; thread t takes words t, t + kMT, ... so every load and store
// instruction of a wave touches consecutive words.
constexpr int kWPT = 4;
constexpr uint64_t kMW = (uint64_t)kMT * kWPT;
constexpr uint64_t kSpan = kMW * 64;  // positions per merge workgroup

// Exclusive scan of one u64 per thread over the workgroup with wave
// shuffles (one barrier pair).  s holds kMT / 64 entries.
__device__ __forceinline__ unsigned long long block_excl_scan_w(unsigned long long x, unsigned long long *s,
                                                                unsigned long long *total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    unsigned long long inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) s[wv] = inc;
    __syncthreads();
    unsigned long long before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kMT / 64; w++) {
        const unsigned long long v = s[w];
        before += (w < wv) ? v : 0ull;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return before + inc - x;
}

// span_run[level][b] = the run holding position min(b * kSpan, n - 1), for b
// in [0, spans]: the first run of span b, and (b + 1) an upper bound on its
// last.  One thread per (level, span).
__global__ __launch_bounds__(kMT) void k_span_runs(MergeArgs a) {
    const uint32_t i = blockIdx.y, k = a.levels - i;
    const uint64_t b = (uint64_t)blockIdx.x * kMT + threadIdx.x;
    if (b > a.wg_per_level) return;
    const uint64_t p = (b * kSpan < a.n) ? b * kSpan : a.n - 1;
    a.span_run[(uint64_t)i * (a.wg_per_level + 1) + b] = find_run(a, k, (uint64_t)a.nbuf << i, 0, p);
}

// Source words of the piece of run x at position p, for positions [p, e).
__device__ __forceinline__ const uint64_t *piece_src(const MergeArgs &a, uint32_t i, const Run &x, uint64_t p,
                                                     uint64_t e, uint64_t *s_out, bool *ok) {
    const uint64_t s = x.src + (p - x.d0);
    const uint64_t pw = (x.q + 1 == a.nbuf) ? a.pwords_last : a.pwords;
    *ok = ((s + (e - p) - 1) >> 6) < pw;
    *s_out = s;
    return reinterpret_cast<const uint64_t *>(a.ptrees + (uint64_t)x.q * a.pstride + a.pbits_off) + (uint64_t)i * pw;
}

__device__ __forceinline__ uint64_t piece_bits(uint64_t lo_w, uint64_t hi_w, uint64_t s, uint32_t m) {
    const uint32_t sh = (uint32_t)(s & 63);
    uint64_t val = lo_w >> sh;
    if (sh + m > 64) val |= hi_w << (64 - sh);
    if (m < 64) val &= (1ull << m) - 1;
    return val;
}

// The pieces of word w0 (positions [w0, wend)) after the first one, which
// ended at p, with next(p, x) -> the run holding p.
template <class Next>
__device__ __forceinline__ uint64_t gather_rest(const MergeArgs &a, uint32_t i, uint64_t w0, uint64_t wend,
                                                uint64_t p, Run x, uint64_t word, Next next) {
    while (p < wend) {
        if (x.d1 <= p) {  // the run is used up: the next non-empty one starts at p
            if (!next(p, x)) break;  // inconsistent tables: leave the rest zero
        }
        const uint64_t e = (x.d1 < wend) ? x.d1 : wend;
        uint64_t s;
        bool ok;
        const uint64_t *src = piece_src(a, i, x, p, e, &s, &ok);
        if (!ok) break;
        const uint32_t m = (uint32_t)(e - p);
        const uint64_t hi_w = ((s & 63) + m > 64) ? src[(s >> 6) + 1] : 0ull;
        word |= piece_bits(src[s >> 6], hi_w, s, m) << (p - w0);
        p = e;
    }
    return word;
}

// One merge workgroup: the kMW words of span blockIdx.x of level
// blockIdx.y (kMW / 8 rank-directory blocks).  The runs the span touches
// are [span_run[b], span_run[b + 1]]; when there are at most kMT of them
// (almost always: runs are long unless the level has millions of nodes)
// they are decoded once into LDS and every word finds its runs there, so
// the offset table is read a few times per workgroup rather than several
// times per word.  Otherwise each thread gallops over the run order from the
// span's first run.  The loads of the first piece of all kWPT words of a
// thread are issued before any is used.
__global__ __launch_bounds__(kMT) void k_merge(MergeArgs a) {
    __shared__ unsigned long long s_scan[kMT / 64];
    __shared__ uint64_t s_d0[kMT], s_d1[kMT], s_src[kMT];
    __shared__ uint32_t s_q[kMT];
    const uint32_t i = blockIdx.y, k = a.levels - i;
    const uint64_t R = (uint64_t)a.nbuf << i;
    const uint64_t wbase = (uint64_t)blockIdx.x * kMW;
    const uint64_t nw = ceil_div(a.n, 64);
    const uint64_t *sr = a.span_run + (uint64_t)i * (a.wg_per_level + 1) + blockIdx.x;
    const uint64_t lo = sr[0], hi = sr[1];
    const bool in_lds = hi - lo < (uint64_t)kMT;  // workgroup-uniform
    if (in_lds) {
        if (threadIdx.x <= hi - lo) {
            const Run x = run_at(a, k, lo + threadIdx.x);
            s_d0[threadIdx.x] = x.d0;
            s_d1[threadIdx.x] = x.d1;
            s_src[threadIdx.x] = x.src;
            s_q[threadIdx.x] = x.q;
        }
        __syncthreads();
    }
    const uint32_t nr = (uint32_t)(hi - lo + 1);
    uint64_t words[kWPT];
    uint32_t jj[kWPT];
    uint64_t rr[kWPT];
    Run xs[kWPT];
    uint64_t lo_w[kWPT], hi_w[kWPT], ss[kWPT], ee[kWPT];
    // first piece of every word: locate, then load
#pragma unroll
    for (int u = 0; u < kWPT; u++) {
        const uint64_t wi = wbase + (uint64_t)u * kMT + threadIdx.x;
        const uint64_t w0 = wi * 64;
        const uint64_t wend = (w0 + 64 < a.n) ? w0 + 64 : a.n;
        words[u] = 0;
        ee[u] = w0;  // no piece
        lo_w[u] = hi_w[u] = 0;
        ss[u] = 0;
        if (wi >= nw) continue;
        Run x;
        if (in_lds) {
            uint32_t j = 0, top = nr;  // last j with s_d0[j] <= w0 (s_d0[0] <= w0)
            while (top - j > 1) {
                const uint32_t mid = (j + top) / 2;
                if (s_d0[mid] <= w0) j = mid;
                else top = mid;
            }
            jj[u] = j;
            x.d0 = s_d0[j];
            x.d1 = s_d1[j];
            x.src = s_src[j];
            x.q = s_q[j];
        } else {
            rr[u] = find_run(a, k, R, lo, w0);
            x = run_at(a, k, rr[u]);
        }
        xs[u] = x;
        if (x.d1 <= w0 || x.d0 > w0) continue;  // inconsistent tables: leave the word zero
        const uint64_t e = (x.d1 < wend) ? x.d1 : wend;
        bool ok;
        const uint64_t *src = piece_src(a, i, x, w0, e, &ss[u], &ok);
        if (!ok) continue;
        ee[u] = e;
        lo_w[u] = src[ss[u] >> 6];
        if ((ss[u] & 63) + (e - w0) > 64) hi_w[u] = src[(ss[u] >> 6) + 1];
    }
#pragma unroll
    for (int u = 0; u < kWPT; u++) {
        const uint64_t wi = wbase + (uint64_t)u * kMT + threadIdx.x;
        const uint64_t w0 = wi * 64;
        const uint64_t wend = (w0 + 64 < a.n) ? w0 + 64 : a.n;
        uint64_t word = 0;
        if (wi < nw && ee[u] > w0) {
            word = piece_bits(lo_w[u], hi_w[u], ss[u], (uint32_t)(ee[u] - w0));
            if (ee[u] < wend) {  // more runs inside this word
                if (in_lds) {
                    uint32_t j = jj[u];
                    word = gather_rest(a, i, w0, wend, ee[u], xs[u], word, [&](uint64_t p, Run &y) {
                        while (j + 1 < nr && s_d1[j] <= p) j++;
                        if (s_d1[j] <= p || s_d0[j] > p) return false;
                        y.d0 = s_d0[j];
                        y.d1 = s_d1[j];
                        y.src = s_src[j];
                        y.q = s_q[j];
                        return true;
                    });
                } else {
                    uint64_t r = rr[u];
                    word = gather_rest(a, i, w0, wend, ee[u], xs[u], word, [&](uint64_t p, Run &y) {
                        if (r + 1 >= R) return false;
                        r = find_run(a, k, R, r + 1, p);
                        y = run_at(a, k, r);
                        return !(y.d1 <= p || y.d0 > p);
                    });
                }
            }
        }
        // words from nw up to the level's padded end are zero
        if (wi < a.words) {
            a.bits[(uint64_t)i * a.words + wi] = word;
            note_write(&a.bits[(uint64_t)i * a.words + wi], 8);
        }
        words[u] = word;
    }
    // rank directory: block blk = wi / 8 holds words of one u (kMT is a
    // multiple of 8); its local prefix is the ones of every earlier word of
    // the span
    unsigned long long carry = 0;
#pragma unroll
    for (int u = 0; u < kWPT; u++) {
        const uint64_t wi = wbase + (uint64_t)u * kMT + threadIdx.x;
        unsigned long long sub_total;
        const unsigned long long before = block_excl_scan_w((unsigned long long)__popcll(words[u]), s_scan, &sub_total);
        const uint64_t blk = wi >> 3;
        if ((wi & 7) == 0 && blk < a.nblk) a.ranks[(uint64_t)i * a.rank_stride + blk] = carry + before;
        carry += sub_total;
    }
    if (threadIdx.x == 0) a.csum[(uint64_t)i * a.wg_per_level + blockIdx.x] = carry;
}

// One workgroup per level: exclusive scan of the workgroup ones in place,
// the level total at entry nblk, zero padding; workgroup 0 also ORs the
// partial builds' status words into the tree's.
__global__ __launch_bounds__(kMT) void k_rank_fix(MergeArgs a) {
    __shared__ unsigned long long s_scan[kMT];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        uint32_t st = 0;
        for (uint32_t q = 0; q < a.nbuf; q++) st |= *reinterpret_cast<const uint32_t *>(a.ptrees + (uint64_t)q * a.pstride);
        *a.tree_status = st;
    }
    if (blockIdx.x >= a.levels) return;
    const uint32_t i = blockIdx.x;
    unsigned long long *cs = a.csum + (uint64_t)i * a.wg_per_level;
    const uint64_t per = (a.wg_per_level + kMT - 1) / kMT;
    const uint64_t k0 = (uint64_t)threadIdx.x * per;
    unsigned long long sum = 0;
    for (uint64_t t = k0; t < k0 + per && t < a.wg_per_level; t++) sum += cs[t];
    unsigned long long total;
    unsigned long long off = block_excl_scan(sum, s_scan, &total);
    for (uint64_t t = k0; t < k0 + per && t < a.wg_per_level; t++) {
        const unsigned long long v = cs[t];
        cs[t] = off;
        off += v;
    }
    uint64_t *R = a.ranks + (uint64_t)i * a.rank_stride;
    for (uint64_t t = a.nblk + threadIdx.x; t < a.rank_stride; t += kMT) R[t] = (t == a.nblk) ? total : 0ull;
}

// Adds each merge workgroup's base (kMW / 8 blocks each) to the local rank
// prefixes of its blocks.
__global__ __launch_bounds__(kMT) void k_rank_apply(MergeArgs a) {
    const uint32_t i = blockIdx.y;
    const uint64_t blk = (uint64_t)blockIdx.x * kMT + threadIdx.x;
    if (blk < a.nblk)
        a.ranks[(uint64_t)i * a.rank_stride + blk] += a.csum[(uint64_t)i * a.wg_per_level + blk / (kMW / 8)];
}

}  // namespace

hipError_t launch_leaf_prefix(const uint64_t *start_last, const ulonglong2 *zo_last, uint32_t levels, uint64_t nq,
                              unsigned long long *row, hipStream_t s) {
    const uint64_t leaves = 1ull << levels;
    hipLaunchKernelGGL(k_leaf_prefix, dim3((unsigned)ceil_div(leaves + 1, kMT)), dim3(kMT), 0, s, start_last, zo_last,
                       leaves, nq, row);
    return hipGetLastError();
}

hipError_t launch_merge(const MergeArgs &a, hipStream_t s) {
    const uint64_t row_blocks = ceil_div(a.row, kMT);
    hipLaunchKernelGGL(k_column_prefix, dim3((unsigned)row_blocks), dim3(kMT), 0, s, a.C, a.nbuf, a.row);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (a.levels) {
        hipLaunchKernelGGL(k_span_runs, dim3((unsigned)ceil_div(a.wg_per_level + 1, kMT), a.levels), dim3(kMT), 0, s,
                           a);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        hipLaunchKernelGGL(k_merge, dim3((unsigned)a.wg_per_level, a.levels), dim3(kMT), 0, s, a);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    hipLaunchKernelGGL(k_rank_fix, dim3(a.levels ? a.levels : 1u), dim3(kMT), 0, s, a);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (a.levels) {
        hipLaunchKernelGGL(k_rank_apply, dim3((unsigned)ceil_div(a.nblk, kMT), a.levels), dim3(kMT), 0, s, a);
        err = hipGetLastError();
    }
    return err;
}

#ifdef WT_WRITE_CHECK
hipError_t write_check_buffered(uint32_t *cnt, uint64_t base, uint64_t bytes) {
    return set_write_check_here(cnt, base, bytes);
}
#endif

}  // namespace wt
