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
// one 512-bit block of the output (one rank-directory entry), finds the run
// holding its first bit by a galloping search over the run order, and ORs
// shifted pieces of the partial bitmaps into its eight words.  Every word has
// a single writer, so the boundary-word atomics of mergeBA are not needed,
// and the popcounts of the block feed the rank directory in the same pass.
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// One thread per 512-bit block of level blockIdx.y: its eight words from
// the partial bitmaps, its local rank prefix, and the workgroup's ones.
__global__ __launch_bounds__(kMT) void k_merge(MergeArgs a) {
    __shared__ unsigned long long s_scan[kMT];
    const uint32_t i = blockIdx.y, k = a.levels - i;
    const uint64_t blk = (uint64_t)blockIdx.x * kMT + threadIdx.x;
    const uint64_t R = (uint64_t)a.nbuf << i;
    uint32_t ones = 0;
    if (blk < a.nblk) {
        uint64_t *out = a.bits + (uint64_t)i * a.words + blk * 8;
        const uint64_t p0 = blk * 512;
        const uint64_t pend = (p0 + 512 < a.n) ? p0 + 512 : a.n;
        uint64_t r = find_run(a, k, R, 0, p0);
        Run x = run_at(a, k, r);
        for (int wi = 0; wi < 8; wi++) {
            const uint64_t w0 = p0 + 64ull * wi;
            const uint64_t wend = (w0 + 64 < pend) ? w0 + 64 : pend;
            uint64_t word = 0, p = w0;
            while (p < wend) {
                if (x.d1 <= p) {  // the run is used up: the next non-empty one starts at p
                    if (r + 1 >= R) break;  // inconsistent tables: leave the rest zero
                    r = find_run(a, k, R, r + 1, p);
                    x = run_at(a, k, r);
                    if (x.d1 <= p || x.d0 > p) break;  // inconsistent tables: leave the rest zero
                }
                const uint64_t e = (x.d1 < wend) ? x.d1 : wend;
                const uint32_t m = (uint32_t)(e - p);
                const uint64_t s = x.src + (p - x.d0);
                const uint64_t pw = (x.q + 1 == a.nbuf) ? a.pwords_last : a.pwords;
                if (((s + m - 1) >> 6) >= pw) break;
                const uint64_t *src = reinterpret_cast<const uint64_t *>(a.ptrees + (uint64_t)x.q * a.pstride +
                                                                         a.pbits_off) + (uint64_t)i * pw;
                const uint32_t sh = (uint32_t)(s & 63);
                uint64_t val = src[s >> 6] >> sh;
                if (sh + m > 64) val |= src[(s >> 6) + 1] << (64 - sh);
                if (m < 64) val &= (1ull << m) - 1;
                word |= val << (p - w0);
                p = e;
            }
            out[wi] = word;
            ones += (uint32_t)__popcll(word);
        }
    }
    unsigned long long total;
    const unsigned long long before = block_excl_scan(ones, s_scan, &total);
    if (blk < a.nblk) a.ranks[(uint64_t)i * a.rank_stride + blk] = before;
    if (threadIdx.x == 0) a.csum[(uint64_t)i * a.wg_per_level + blockIdx.x] = total;
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

// Adds each workgroup's base to the local rank prefixes of its blocks.
__global__ __launch_bounds__(kMT) void k_rank_apply(MergeArgs a) {
    const uint32_t i = blockIdx.y;
    const uint64_t blk = (uint64_t)blockIdx.x * kMT + threadIdx.x;
    if (blk < a.nblk) a.ranks[(uint64_t)i * a.rank_stride + blk] += a.csum[(uint64_t)i * a.wg_per_level + blockIdx.x];
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
        hipLaunchKernelGGL(k_merge, dim3((unsigned)a.wg_per_level, a.levels), dim3(kMT), 0, s, a);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    hipLaunchKernelGGL(k_rank_fix, dim3(a.levels ? a.levels : 1u), dim3(kMT), 0, s, a);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (a.levels) {
        hipLaunchKernelGGL(k_rank_apply, dim3((unsigned)a.wg_per_level, a.levels), dim3(kMT), 0, s, a);
        err = hipGetLastError();
    }
    return err;
}

}  // namespace wt
