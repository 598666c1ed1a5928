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
// position by position: a 64-position word is built by one workgroup from
// 64 consecutive symbols and has exactly one writer (no atomics on bitmaps).
//
// One level pass over tiles of kTile symbols does, in a single read of T_i:
//   * the bitmap words of the tile (one writer per word),
//   * the tile's ones count, turned into the global rank of its first
//     position by a decoupled look-back over tiles taken in ticket order
//     (the device-wide exclusive scan of the segment counts),
//   * the rank directory entries at the multiples of 512 inside the tile,
//   * the stable split into T_{i+1}: with O1(v) the ones before node v and
//     rank1(p) the ones before position p,
//       bit 0 at p  ->  p - rank1(p) + O1(v)
//       bit 1 at p  ->  start_{i+1}(2v+1) - O1(v) + rank1(p)
//     staged in LDS so that the global stores are aligned 16-byte chunks,
//   * for levels beyond the first-pass histogram, the ones counts of the
//     next level's nodes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wt_internal.h"

namespace wt {

namespace {

constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagPre = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;

template <int W> struct ElemT;
template <> struct ElemT<1> { typedef uint8_t T; };
template <> struct ElemT<2> { typedef uint16_t T; };
template <> struct ElemT<4> { typedef uint32_t T; };

__device__ __forceinline__ uint64_t ld_acq(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ unsigned long long wave_incl_scan64(unsigned long long v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        unsigned long long t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Load kEPT (=16) consecutive symbols starting at position pos.  Symbols at
// positions >= n read as 0.  pos is a multiple of 16, so a full load is
// 16-byte aligned for every width (buffers are 16-byte aligned).
template <int W>
__device__ __forceinline__ int load16(const void *src, uint64_t pos, uint64_t n, uint32_t (&x)[16]) {
    typedef typename ElemT<W>::T T;
    const T *s = reinterpret_cast<const T *>(src);
    if (pos + 16 <= n) {
        const uint4 *p = reinterpret_cast<const uint4 *>(s + pos);
#pragma unroll
        for (int q = 0; q < W; q++) {
            uint4 v = p[q];
            uint32_t d4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int d = 0; d < 4; d++) {
#pragma unroll
                for (int e = 0; e < 4 / W; e++) {
                    uint32_t val = (W == 4) ? d4[d] : ((d4[d] >> (8 * W * e)) & ((1u << (8 * W)) - 1u));
                    x[q * (16 / W) + d * (4 / W) + e] = val;
                }
            }
        }
        return 16;
    }
    int nval = pos < n ? (int)(n - pos) : 0;
#pragma unroll
    for (int k = 0; k < 16; k++) x[k] = (k < nval) ? (uint32_t)s[pos + k] : 0u;
    return nval;
}

// ------------------------------------------------------------- zero fill --

__global__ void k_zero(uint64_t *p, uint64_t words, uint32_t *tree_status, uint64_t *tree_ranks,
                       uint64_t tree_ranks_count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < words; k += stride) p[k] = 0;
    if (tree_ranks)
        for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < tree_ranks_count; k += stride)
            tree_ranks[k] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *tree_status = 0;
}

// ----------------------------------------------- validation + histogram ---
// Reads S once: flags symbols >= sigma and counts the top min(l, kTopBits)
// bits of every symbol (the node counts of the first levels, Algorithm pwt's
// counting step hoisted out of the level loop).

template <int W>
__global__ __launch_bounds__(kThreads) void k_hist(HistArgs a) {
    __shared__ uint32_t s_h[1u << kTopBits];
    for (uint32_t b = threadIdx.x; b < a.nbins; b += kThreads) s_h[b] = 0;
    __syncthreads();
    bool bad = false;
    const uint64_t step = (uint64_t)gridDim.x * kThreads * kEPT;
    for (uint64_t pos = ((uint64_t)blockIdx.x * kThreads + threadIdx.x) * kEPT; pos < a.n; pos += step) {
        uint32_t x[16];
        int nval = load16<W>(a.S, pos, a.n, x);
#pragma unroll
        for (int k = 0; k < 16; k++) {
            if (k < nval) {
                bad |= x[k] >= a.sigma;
                atomicAdd(&s_h[(x[k] & a.symmask) >> a.hshift], 1u);
            }
        }
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(a.tree_status, 1u);
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < a.nbins; b += kThreads)
        if (s_h[b]) atomicAdd(&a.hist[b], (unsigned long long)s_h[b]);
}

// ----------------------------------------- node tables of the top levels --
// From the histogram H of the top h bits (P = exclusive prefix sum of H):
//   node v of level i < h starts at P[v << (h-i)],
//   its ones are the symbols of prefix 2v+1 at level i+1,
//   O1(v) = ones of the nodes before v,
//   zo(v) = (O1(v), start of node 2v+1 at level i+1 - O1(v)).

__global__ __launch_bounds__(kThreads) void k_top(TopArgs a) {
    __shared__ unsigned long long P[(1u << kTopBits) + 1];
    const uint32_t nb = 1u << a.h;
    if (threadIdx.x == 0) {
        unsigned long long acc = 0;
        for (uint32_t b = 0; b < nb; b++) {
            P[b] = acc;
            acc += a.hist[b];
        }
        P[nb] = acc;
    }
    __syncthreads();
    for (uint32_t i = 0; i < a.h; i++) {
        const uint32_t s = a.h - i - 1;  // prefix length i+1 -> shift into H's bins
        ulonglong2 *zo = a.zo + a.zo_off[i];
        for (uint32_t v = threadIdx.x; v < (1u << i); v += kThreads) {
            unsigned long long o1 = 0;
            for (uint32_t u = 0; u < v; u++) o1 += P[(2 * u + 2) << s] - P[(2 * u + 1) << s];
            zo[v] = make_ulonglong2(o1, P[(2 * v + 1) << s] - o1);
        }
    }
    if (a.start_h)
        for (uint32_t v = threadIdx.x; v <= nb; v += kThreads) a.start_h[v] = P[v];
}

// ------------------------------------------ node tables of deeper levels --
// For level i with node starts start_i and ones counts ones_i:
//   O1 = exclusive scan of ones_i,
//   zo_i(v) = (O1(v), start_i(v+1) - ones_i(v) - O1(v)),
//   start_{i+1}(2v) = start_i(v), start_{i+1}(2v+1) = start_i(v+1) - ones_i(v).

__global__ __launch_bounds__(kThreads) void k_plan_reduce(PlanArgs a) {
    __shared__ unsigned long long s_w[kThreads / 64];
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanChunk;
    unsigned long long sum = 0;
    for (uint64_t k = b0 + threadIdx.x; k < b0 + kScanChunk && k < a.nodes; k += kThreads) sum += a.ones[k];
    sum = wave_sum64(sum);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kThreads / 64; w++) t += s_w[w];
        a.partials[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kThreads) void k_plan_partials(PlanArgs a, uint64_t nblocks) {
    if (threadIdx.x == 0) {
        unsigned long long acc = 0;
        for (uint64_t b = 0; b < nblocks; b++) {
            unsigned long long v = a.partials[b];
            a.partials[b] = acc;
            acc += v;
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_plan_apply(PlanArgs a, int use_partials) {
    __shared__ unsigned long long s_w[kThreads / 64];
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanChunk;
    const uint64_t per = kScanChunk / kThreads;  // 16 consecutive entries per thread
    const uint64_t k0 = b0 + threadIdx.x * per;
    unsigned long long loc[kScanChunk / kThreads];
    unsigned long long tsum = 0;
#pragma unroll
    for (uint64_t q = 0; q < per; q++) {
        loc[q] = (k0 + q < a.nodes) ? a.ones[k0 + q] : 0ull;
        tsum += loc[q];
    }
    unsigned long long incl = wave_incl_scan64(tsum);
    if ((threadIdx.x & 63) == 63) s_w[threadIdx.x >> 6] = incl;
    __syncthreads();
    unsigned long long off = use_partials ? a.partials[blockIdx.x] : 0ull;
    for (int w = 0; w < (int)(threadIdx.x >> 6); w++) off += s_w[w];
    unsigned long long o1 = off + incl - tsum;
#pragma unroll
    for (uint64_t q = 0; q < per; q++) {
        const uint64_t v = k0 + q;
        if (v < a.nodes) {
            const unsigned long long ones = loc[q];
            const uint64_t s_next = a.start[v + 1];
            a.zo[v] = make_ulonglong2(o1, s_next - ones - o1);
            if (a.start_next) {
                a.start_next[2 * v] = a.start[v];
                a.start_next[2 * v + 1] = s_next - ones;
            }
            o1 += ones;
        }
    }
    if (a.start_next && blockIdx.x == 0 && threadIdx.x == 0) a.start_next[2 * a.nodes] = a.n;
}

// ----------------------------------------------------------- level pass ---

// Decoupled look-back over the tiles (taken in ticket order, so every
// predecessor is resident or finished): returns the number of ones in all
// tiles before tile t.  Executed by one full wave.
__device__ __forceinline__ unsigned long long lookback(uint64_t *status, uint64_t t, uint32_t agg) {
    const int lane = threadIdx.x & 63;
    if (t == 0) {
        if (lane == 0) st_rel(&status[0], kFlagPre | (uint64_t)agg);
        return 0;
    }
    if (lane == 0) st_rel(&status[t], kFlagAgg | (uint64_t)agg);
    unsigned long long excl = 0;
    int64_t j = (int64_t)t - 1;
    while (true) {
        const int64_t idx = j - lane;
        uint64_t s = kFlagPre;  // before tile 0: a prefix of zero
        if (idx >= 0) {
            do {
                s = ld_acq(&status[idx]);
            } while ((s >> 62) == 0);
        }
        const unsigned long long pm = __ballot((s >> 62) == 2);
        if (pm) {
            const int first = __builtin_ctzll(pm);
            excl += wave_sum64(lane <= first ? (s & kValMask) : 0ull);
            break;
        }
        excl += wave_sum64(s & kValMask);
        j -= 64;
    }
    if (lane == 0) st_rel(&status[t], kFlagPre | (excl + agg));
    return excl;
}

template <int W>
__global__ __launch_bounds__(kThreads) void k_level(LevelArgs a) {
    typedef typename ElemT<W>::T T;
    constexpr int CH = 16 / W;  // symbols per 16-byte chunk

    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_vfirst, s_vlast;
    __shared__ unsigned long long s_prefix;
    __shared__ uint32_t s_wtot[kThreads / 64];
    __shared__ uint32_t s_red[2][kThreads / 64];
    __shared__ uint16_t s_m16[kThreads];
    // zeros at [a0, a0+Z), ones at [a1, a1+O): a1 + O <= kTile + 3*CH - 3
    __shared__ __align__(16) T s_stage[kTile + 4 * CH];
    __shared__ uint32_t s_cnt[2 * kNodeCap];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) s_tile = atomicAdd(a.ticket, 1u);
    __syncthreads();
    const uint64_t t = s_tile;
    if (t >= a.ntiles) return;  // tickets are zeroed per build, so never taken
    const uint64_t base = t * kTile;
    const uint64_t pos0 = base + (uint64_t)tid * kEPT;
    const uint64_t nvalid = (a.n - base < kTile) ? a.n - base : kTile;  // base < n

    uint32_t x[16];
    const int nval = load16<W>(a.tin, pos0, a.n, x);
    const uint32_t sh = a.levels - 1 - a.level;  // bit of this level
    const uint32_t nsh = a.levels - a.level;     // node shift (Proposition 1)
    uint32_t mb = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        x[k] &= a.symmask;  // keeps every node index in range even for bad input
        mb |= ((x[k] >> sh) & 1u) << k;
    }

    // node span of the tile (T_i is sorted by node)
    if (tid == 0) s_vfirst = x[0] >> nsh;
    {
        const uint64_t last = nvalid - 1;
        if ((uint64_t)tid == last / kEPT) {
            const int kl = (int)(last % kEPT);
            uint32_t xv = 0;
#pragma unroll
            for (int k = 0; k < 16; k++) xv = (k == kl) ? x[k] : xv;
            s_vlast = xv >> nsh;
        }
    }

    s_m16[tid] = (uint16_t)mb;
    const uint32_t pc = __popc(mb);
    const uint32_t incl = wave_incl_scan(pc);
    if (lane == 63) s_wtot[wv] = incl;
    __syncthreads();

    uint32_t agg = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; w++) agg += s_wtot[w];

    if (wv == 0) {
        // bitmap words: word q of the tile = 4 threads x 16 bits
        const uint64_t wd = (uint64_t)s_m16[4 * lane] | ((uint64_t)s_m16[4 * lane + 1] << 16) |
                            ((uint64_t)s_m16[4 * lane + 2] << 32) | ((uint64_t)s_m16[4 * lane + 3] << 48);
        const uint64_t widx = base / 64 + lane;
        if (widx < a.words) a.bits[widx] = wd;
        const unsigned long long ex = lookback(a.status, t, agg);
        if (lane == 0) s_prefix = ex;
    }
    __syncthreads();
    const unsigned long long prefix = s_prefix;
    uint32_t wex = 0;
    for (int w = 0; w < wv; w++) wex += s_wtot[w];
    const uint32_t lr1_thread = wex + incl - pc;  // ones in the tile before this thread
    const unsigned long long r_thread = prefix + lr1_thread;

    // rank directory: entry k = ones before position 512k (every 32nd thread)
    if ((tid & 31) == 0) {
        const uint64_t k = pos0 >> 9;
        if (k < a.rank_stride) a.ranks[k] = (k < a.rank_entries) ? r_thread : 0ull;
    }
    if (t == a.ntiles - 1 && tid < 8) {  // entries past the last tile
        const uint64_t k = (base + kTile) / 512 + tid;
        if (k < a.rank_stride) a.ranks[k] = (k < a.rank_entries) ? prefix + agg : 0ull;
    }

    if (a.tout == nullptr) return;  // last level: no next order, no counts

    T *tout = reinterpret_cast<T *>(a.tout);
    const uint32_t vf = s_vfirst, vl = s_vlast;
    if (vf == vl) {
        // Single node: zeros keep their order at g0.., ones at g1...
        const ulonglong2 zo = a.zo[vf];
        const uint64_t Z = nvalid - agg, O = agg;
        const uint64_t g0 = base - prefix + zo.x;
        const uint64_t g1 = zo.y + prefix;
        const uint32_t a0 = (uint32_t)(g0 % CH);
        const uint32_t r1 = (uint32_t)round_up(a0 + Z, CH);
        const uint32_t a1 = r1 + (uint32_t)(g1 % CH);
#pragma unroll
        for (int k = 0; k < 16; k++) {
            if (k < nval) {
                const uint32_t lr1 = lr1_thread + __popc(mb & ((1u << k) - 1u));
                const uint32_t lidx = (uint32_t)tid * kEPT + k;
                if ((mb >> k) & 1u) s_stage[a1 + lr1] = (T)x[k];
                else s_stage[a0 + (lidx - lr1)] = (T)x[k];
            }
        }
        __syncthreads();
        const uint32_t nch = (a1 + (uint32_t)O + CH - 1) / CH;
        for (uint32_t c = tid; c < nch; c += kThreads) {
            const uint32_t s = c * CH;
            uint64_t gb;
            uint32_t lo, hi;
            if (s < r1) { gb = g0 - a0; lo = a0; hi = a0 + (uint32_t)Z; }
            else        { gb = g1 - a1; lo = a1; hi = a1 + (uint32_t)O; }
            // (destinations beyond n only arise from inconsistent tables; they
            // are dropped rather than written)
            if (s >= lo && s + CH <= hi && gb + s + CH <= a.n) {
                *reinterpret_cast<uint4 *>(tout + (gb + s)) = *reinterpret_cast<const uint4 *>(&s_stage[s]);
            } else {
#pragma unroll
                for (int e = 0; e < CH; e++)
                    if (s + e >= lo && s + e < hi && gb + s + e < a.n) tout[gb + s + e] = s_stage[s + e];
            }
        }
    } else {
        // Several nodes: every symbol goes straight to its destination.
#pragma unroll
        for (int k = 0; k < 16; k++) {
            if (k < nval) {
                const uint32_t v = x[k] >> nsh;
                const ulonglong2 zo = a.zo[v];
                const unsigned long long r1 = r_thread + __popc(mb & ((1u << k) - 1u));
                const uint64_t p = pos0 + k;
                const uint64_t dst = ((mb >> k) & 1u) ? zo.y + r1 : p - r1 + zo.x;
                if (dst < a.n) tout[dst] = (T)x[k];
            }
        }
    }

    if (a.ones_next == nullptr) return;

    // Ones of the next level, per next-level node 2v + bit.
    const uint32_t sh2 = sh - 1;
    uint32_t mb2 = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) mb2 |= ((x[k] >> sh2) & 1u) << k;  // invalid symbols are 0
    if (vf == vl) {
        uint32_t c0 = wave_sum32(__popc(~mb & mb2 & 0xffffu));
        uint32_t c1 = wave_sum32(__popc(mb & mb2));
        if (lane == 0) { s_red[0][wv] = c0; s_red[1][wv] = c1; }
        __syncthreads();
        if (tid == 0) {
            uint32_t t0 = 0, t1 = 0;
            for (int w = 0; w < kThreads / 64; w++) { t0 += s_red[0][w]; t1 += s_red[1][w]; }
            if (t0) atomicAdd(&a.ones_next[2ull * vf], (unsigned long long)t0);
            if (t1) atomicAdd(&a.ones_next[2ull * vf + 1], (unsigned long long)t1);
        }
    } else if (vl - vf < kNodeCap) {
        const uint32_t nc = 2 * (vl - vf + 1);
        for (uint32_t q = tid; q < nc; q += kThreads) s_cnt[q] = 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; k++)
            if (k < nval && ((mb2 >> k) & 1u) && (x[k] >> nsh) - vf <= vl - vf)
                atomicAdd(&s_cnt[2 * ((x[k] >> nsh) - vf) + ((mb >> k) & 1u)], 1u);
        __syncthreads();
        for (uint32_t q = tid; q < nc; q += kThreads)
            if (s_cnt[q]) atomicAdd(&a.ones_next[2ull * vf + q], (unsigned long long)s_cnt[q]);
    } else {
#pragma unroll
        for (int k = 0; k < 16; k++)
            if (k < nval && ((mb2 >> k) & 1u))
                atomicAdd(&a.ones_next[2ull * (x[k] >> nsh) + ((mb >> k) & 1u)], 1ull);
    }
}

}  // namespace

// ------------------------------------------------------------- launchers --

static inline uint32_t grid_for(uint64_t items, uint64_t per_block, uint32_t cap) {
    uint64_t g = ceil_div(items, per_block);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

hipError_t launch_zero(void *p, uint64_t bytes, uint32_t *tree_status, uint64_t *tree_ranks,
                       uint64_t tree_ranks_count, hipStream_t s) {
    const uint64_t words = bytes / 8;
    const uint64_t items = words > tree_ranks_count ? words : tree_ranks_count;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(items, 256, 4096)), dim3(256), 0, s, (uint64_t *)p, words,
                       tree_status, tree_ranks, tree_ranks_count);
    return hipGetLastError();
}

hipError_t launch_hist(const HistArgs &a, uint32_t width, uint64_t ntiles, hipStream_t s) {
    const uint32_t g = grid_for(ntiles, 1, 2048);
    if (width == 1) hipLaunchKernelGGL(k_hist<1>, dim3(g), dim3(kThreads), 0, s, a);
    else if (width == 2) hipLaunchKernelGGL(k_hist<2>, dim3(g), dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL(k_hist<4>, dim3(g), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_top(const TopArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_top, dim3(1), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_plan(const PlanArgs &a, hipStream_t s) {
    const uint64_t nb = ceil_div(a.nodes, kScanChunk);
    if (nb > 1) {
        hipLaunchKernelGGL(k_plan_reduce, dim3((uint32_t)nb), dim3(kThreads), 0, s, a);
        hipLaunchKernelGGL(k_plan_partials, dim3(1), dim3(kThreads), 0, s, a, nb);
    }
    hipLaunchKernelGGL(k_plan_apply, dim3((uint32_t)nb), dim3(kThreads), 0, s, a, nb > 1 ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_level(const LevelArgs &a, uint32_t width, hipStream_t s) {
    const dim3 g((uint32_t)a.ntiles);
    if (width == 1) hipLaunchKernelGGL(k_level<1>, g, dim3(kThreads), 0, s, a);
    else if (width == 2) hipLaunchKernelGGL(k_level<2>, g, dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL(k_level<4>, g, dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace wt
