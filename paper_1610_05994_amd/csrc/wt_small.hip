// One-workgroup construction of a short sequence, every level in LDS.
// Two sizes: 512 threads under 64 KB of LDS, 1024 threads up to 160 KB.
//
// Same level split as the tiled passes (T_0 = S, T_{i+1} = T_i stably
// partitioned inside every level-i node by the level-i bit, Proposition 1
// giving the node of s at level i as s >> (l-i)), but the whole of T_i sits
// in LDS and one workgroup runs all l levels back to back, so a build is a
// single launch and a batch of short sequences is a single launch with one
// workgroup per sequence.
//
// Node tables are not used.  Because T_i is sorted by node, the nodes of T_i
// are its maximal runs of equal s >> (l-i); a segmented scan finds, for every
// position p, the run [s, e) that holds it.  With rank1 the ones before a
// position at this level, the destinations of the split are
//     bit 0 at p  ->  p - rank1(p) + rank1(s)
//     bit 1 at p  ->  e - rank1(e) + rank1(p)
// (the counts of Algorithm pwt restricted to one node, Section 3.1), so the
// work per level is O(n) whatever sigma is, and rank1 is only ever needed at
// run starts and at n.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wt_check.h"
#include "wt_internal.h"

namespace wt {

namespace {

template <int W> struct SElem;
template <> struct SElem<1> { typedef uint8_t T; };
template <> struct SElem<2> { typedef uint16_t T; };
template <> struct SElem<4> { typedef uint32_t T; };

// Block-wide exclusive scans of one value per thread: sum, max (from the
// left) and min (from the right).  Each synchronises the workgroup twice.
struct Scans {
    uint32_t sum_excl, total, max_excl, min_excl_right;
};

template <int kSW>
__device__ __forceinline__ Scans block_scans(uint32_t c, uint32_t mx, uint32_t mn, uint32_t mn_identity,
                                             uint32_t (*s_w)[kSW]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t inc = c, imx = mx, imn = mn;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t a = __shfl_up(inc, d, 64);
        const uint32_t b = __shfl_up(imx, d, 64);
        const uint32_t e = __shfl_down(imn, d, 64);
        if (lane >= d) {
            inc += a;
            imx = imx > b ? imx : b;
        }
        if (lane + d < 64) imn = imn < e ? imn : e;
    }
    if (lane == 63) {
        s_w[0][wv] = inc;
        s_w[1][wv] = imx;
    }
    if (lane == 0) s_w[2][wv] = imn;
    __syncthreads();
    uint32_t off = 0, tot = 0, wmx = 0, wmn = mn_identity;
#pragma unroll
    for (int w = 0; w < kSW; w++) {
        const uint32_t sw = s_w[0][w];
        tot += sw;
        if (w < wv) {
            off += sw;
            wmx = wmx > s_w[1][w] ? wmx : s_w[1][w];
        }
        if (w > wv) wmn = wmn < s_w[2][w] ? wmn : s_w[2][w];
    }
    __syncthreads();
    Scans r;
    r.sum_excl = off + inc - c;
    r.total = tot;
    const uint32_t pmx = __shfl_up(imx, 1, 64);
    r.max_excl = (lane > 0) ? (pmx > wmx ? pmx : wmx) : wmx;
    const uint32_t nmn = __shfl_down(imn, 1, 64);
    r.min_excl_right = (lane < 63) ? (nmn < wmn ? nmn : wmn) : wmn;
    return r;
}

// Symbol k of a thread's chunk held as dwords.
template <int W>
__device__ __forceinline__ uint32_t sym_of(const uint32_t *d, int k) {
    if (W == 4) return d[k];
    if (W == 2) return (d[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
    return (d[k >> 2] >> (8 * (k & 3))) & 0xFFu;
}

// Whole build of one sequence; each of the NT threads owns E consecutive
// positions.
template <int W, int NT, int E, uint32_t CAP>
__device__ void small_levels(const SmallJob &j, typename SElem<W>::T (*s_buf)[CAP], uint16_t *s_rank,
                             uint32_t (*s_w)[NT / 64]) {
    typedef typename SElem<W>::T T;
    constexpr int D = E * W / 4;  // dwords per chunk (E * W >= 8)
    const uint32_t n = j.n, l = j.levels, tid = threadIdx.x;
    const int lane = tid & 63;
    uint64_t *bits = reinterpret_cast<uint64_t *>(j.tree + j.bits_off);
    uint64_t *ranks = reinterpret_cast<uint64_t *>(j.tree + j.ranks_off);
    const uint32_t p0 = tid * E;
    const uint32_t cnt = p0 < n ? ((n - p0) < (uint32_t)E ? n - p0 : (uint32_t)E) : 0u;
    const uint32_t kfull = ceil_div(n, 512);  // rank entries at positions < n

    int cur = 0;
    for (uint32_t i = 0; i < l; i++) {
        const T *tin = s_buf[cur];
        T *tout = s_buf[cur ^ 1];
        const uint32_t sh = l - 1 - i;  // bit of this level
        const uint32_t nsh = l - i;     // node shift (Proposition 1)

        uint32_t d[D];
        if (cnt) {
            // p0 + E <= capacity, so the whole chunk is inside the buffer
            if (D >= 4) {
#pragma unroll
                for (int q = 0; q < D / 4; q++) {
                    const uint4 v = reinterpret_cast<const uint4 *>(tin + p0)[q];
                    d[4 * q] = v.x;
                    d[4 * q + 1] = v.y;
                    d[4 * q + 2] = v.z;
                    d[4 * q + 3] = v.w;
                }
            } else {
                const uint2 v = *reinterpret_cast<const uint2 *>(tin + p0);
                d[0] = v.x;
                d[1] = v.y;
            }
        } else {
#pragma unroll
            for (int q = 0; q < D; q++) d[q] = 0;
        }
        // level bits (bm) and run starts (fm) of the chunk
        uint32_t vprev = (cnt && p0 > 0) ? (j.matrix ? 0u : ((uint32_t)tin[p0 - 1] >> nsh)) : 0xFFFFFFFFu;
        uint32_t bm = 0, fm = 0;
#pragma unroll
        for (int k = 0; k < E; k++) {
            if ((uint32_t)k < cnt) {
                const uint32_t x = sym_of<W>(d, k);
                const uint32_t v = j.matrix ? 0u : x >> nsh;  // a matrix level is one node
                bm |= ((x >> sh) & 1u) << k;
                fm |= (v != vprev ? 1u : 0u) << k;
                vprev = v;
            }
        }
        const uint32_t last_start = fm ? p0 + 31 - __clz(fm) : 0u;  // position 0 always starts a run
        const uint32_t first_start = fm ? p0 + __ffs(fm) - 1 : n;
        const Scans sc = block_scans<NT / 64>(__popc(bm), last_start, first_start, n, s_w);
        const uint32_t base = sc.sum_excl;

        // rank1 at every run start of the chunk, and at n
#pragma unroll
        for (int k = 0; k < E; k++)
            if ((fm >> k) & 1u) s_rank[p0 + k] = (uint16_t)(base + __popc(bm & ((1u << k) - 1u)));
        if (tid == 0) {
            s_rank[n] = (uint16_t)sc.total;
            if (j.matrix) reinterpret_cast<unsigned long long *>(j.tree + kZerosOff)[i] = n - sc.total;
        }

        // bitmap words: 64 / E consecutive threads form one word (chunks of
        // positions >= n contribute zeros, so padding words are written too)
        {
            uint64_t wd = bm;
#pragma unroll
            for (int q = 1; q < 64 / E; q++) wd |= (uint64_t)__shfl_down(bm, q, 64) << (q * E);
            const uint32_t widx = p0 / 64;
            if ((lane % (64 / E)) == 0 && widx < j.words) {
                bits[(uint64_t)i * j.words + widx] = wd;
                note_write(&bits[(uint64_t)i * j.words + widx], 8);
            }
        }
        // rank directory: entry k = ones before min(512k, n); padding zero
        uint64_t *rk = ranks + (uint64_t)i * j.rank_stride;
        if ((p0 & 511) == 0 && p0 < n) rk[p0 / 512] = base;
        if (tid < 8 && kfull + tid < j.rank_stride) rk[kfull + tid] = (kfull + tid < j.rank_entries) ? sc.total : 0ull;

        if (i + 1 == l) break;
        __syncthreads();  // s_rank complete
        uint32_t r = base, o1 = 0, zb = 0;
#pragma unroll
        for (int k = 0; k < E; k++) {
            if ((uint32_t)k < cnt) {
                if (k == 0 || ((fm >> k) & 1u)) {
                    const uint32_t s = ((fm >> k) & 1u) ? p0 + k : sc.max_excl;
                    const uint64_t above = (uint64_t)fm >> (k + 1);
                    const uint32_t e = above ? p0 + k + 1 + (uint32_t)__builtin_ctzll(above) : sc.min_excl_right;
                    o1 = s_rank[s];
                    zb = e - s_rank[e];
                }
                const uint32_t b = (bm >> k) & 1u;
                const uint32_t p = p0 + k;
                const uint32_t dst = b ? zb + r : p - r + o1;  // inside [s, e)
                tout[dst] = (T)sym_of<W>(d, k);
                r += b;
            }
        }
        __syncthreads();  // T_{i+1} complete, s_rank free
        cur ^= 1;
    }
}

template <int W, uint32_t GEOM>
__device__ void small_build(const SmallJob &j) {
    typedef typename SElem<W>::T T;
    constexpr int NT = one_wg_threads(GEOM);
    constexpr uint32_t CAP = one_wg_cap(W, GEOM);
    static_assert(CAP % 32 == 0 && CAP <= 32u * NT, "capacity must fit the chunks");
    __shared__ __align__(16) T s_buf[2][CAP];
    __shared__ uint16_t s_rank[CAP + 1];
    __shared__ uint32_t s_w[3][NT / 64];
    const uint32_t n = j.n, tid = threadIdx.x;
    if (n > CAP) return;  // the host never sends these
    const uint32_t mask = (uint32_t)((1ull << j.levels) - 1);

    // T_0 = S, masked to l bits; symbols >= sigma are flagged
    bool bad = false;
    const T *S = reinterpret_cast<const T *>(j.S);
    const uint32_t nvec = (n * W) / 16;
    const uint32_t mrep = (W == 1) ? mask * 0x01010101u : (W == 2) ? mask * 0x00010001u : mask;
    for (uint32_t q = tid; q < nvec; q += NT) {
        uint4 v = reinterpret_cast<const uint4 *>(S)[q];
        const uint32_t dw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 16 / W; k++) bad |= sym_of<W>(dw, k) >= j.sigma;
        v.x &= mrep;
        v.y &= mrep;
        v.z &= mrep;
        v.w &= mrep;
        reinterpret_cast<uint4 *>(s_buf[0])[q] = v;
    }
    for (uint32_t p = nvec * (16 / W) + tid; p < n; p += NT) {
        const uint32_t x = S[p];
        bad |= x >= j.sigma;
        s_buf[0][p] = (T)(x & mask);
    }
    bad = __syncthreads_or(bad);
    if (tid == 0) *reinterpret_cast<uint32_t *>(j.tree) = bad ? 1u : 0u;

    if (n <= NT * 8) small_levels<W, NT, 8, CAP>(j, s_buf, s_rank, s_w);
    else if (n <= NT * 16) small_levels<W, NT, 16, CAP>(j, s_buf, s_rank, s_w);
    else small_levels<W, NT, 32, CAP>(j, s_buf, s_rank, s_w);
}

template <int W, uint32_t GEOM>
__global__ __launch_bounds__(one_wg_threads(GEOM)) void k_small_one(SmallJob j) {
    small_build<W, GEOM>(j);
}

template <int W, uint32_t GEOM>
__global__ __launch_bounds__(one_wg_threads(GEOM)) void k_small_batch(const SmallJob *jobs) {
    const SmallJob j = jobs[blockIdx.x];
    small_build<W, GEOM>(j);
}

}  // namespace

#define WT_SMALL_LAUNCH(KERNEL, WIDTH, GEOM, GRID, ...)                                                 \
    do {                                                                                                 \
        const dim3 blk_s(one_wg_threads(kGeomSmall)), blk_m(one_wg_threads(kGeomMid));                 \
        switch ((WIDTH) * 10 + (GEOM)) {                                                                 \
            case 11: hipLaunchKernelGGL((KERNEL<1, kGeomSmall>), GRID, blk_s, 0, __VA_ARGS__); break;    \
            case 21: hipLaunchKernelGGL((KERNEL<2, kGeomSmall>), GRID, blk_s, 0, __VA_ARGS__); break;    \
            case 41: hipLaunchKernelGGL((KERNEL<4, kGeomSmall>), GRID, blk_s, 0, __VA_ARGS__); break;    \
            case 12: hipLaunchKernelGGL((KERNEL<1, kGeomMid>), GRID, blk_m, 0, __VA_ARGS__); break;      \
            case 22: hipLaunchKernelGGL((KERNEL<2, kGeomMid>), GRID, blk_m, 0, __VA_ARGS__); break;      \
            case 42: hipLaunchKernelGGL((KERNEL<4, kGeomMid>), GRID, blk_m, 0, __VA_ARGS__); break;      \
            default: return hipErrorInvalidValue;                                                        \
        }                                                                                                \
    } while (0)

hipError_t launch_small_one(const SmallJob &j, uint32_t width, uint32_t geom, hipStream_t s) {
    WT_SMALL_LAUNCH(k_small_one, width, geom, dim3(1), s, j);
    return hipGetLastError();
}

hipError_t launch_small_batch(const SmallJob *d_jobs, uint32_t count, uint32_t width, uint32_t geom, hipStream_t s) {
    if (count == 0) return hipSuccess;
    WT_SMALL_LAUNCH(k_small_batch, width, geom, dim3(count), s, d_jobs);
    return hipGetLastError();
}

#ifdef WT_WRITE_CHECK
hipError_t write_check_small(uint32_t *cnt, uint64_t base, uint64_t bytes) {
    return set_write_check_here(cnt, base, bytes);
}
#endif

}  // namespace wt
