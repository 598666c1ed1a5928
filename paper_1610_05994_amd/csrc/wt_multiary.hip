// Directories of the 4-ary tree's digit levels.  Entry k of a level holds
// the counts of digits 0, 1, 2 and 3 in positions [0, min(512 k, n)): the
// rank structure of the one-pointer-per-level representation (Section 2.2)
// with four symbols per level instead of two.
//
// Sixteen lanes count one 512-position block (sixteen 32-digit words) with
// popcounts over the two bit planes of the words; each wave scans the counts
// of its 64 blocks, the workgroup combines its waves, the workgroup totals
// of a level are scanned by one workgroup, and a last pass adds each
// workgroup's base.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wt_internal.h"

namespace wt {

namespace {

constexpr int kDT = 256;  // threads per workgroup
constexpr uint64_t kEven = 0x5555555555555555ull;

// Exclusive scan of one u64 per thread over the workgroup (wave shuffles,
// one barrier pair); s holds kDT / 64 entries.
__device__ __forceinline__ unsigned long long excl_scan(unsigned long long x, unsigned long long *s,
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
    for (int w = 0; w < kDT / 64; w++) {
        const unsigned long long v = s[w];
        before += (w < wv) ? v : 0ull;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return before + inc - x;
}

// Block counts and their workgroup-local prefixes.  Each wave covers 64
// blocks (1024 words): lane l reads words l, l + 64, ... (coalesced), counts
// digits 1, 2, 3 of each word (packed in 16-bit fields), and the 16 lanes
// holding one block's words add their counts with shuffles.  Lane b then
// scans block b's counts across the wave, counts (0, 1) and (2, 3)
// travelling as the two 32-bit halves of a u64, and the four waves' totals
// give each wave its base inside the workgroup.
constexpr int kWaveBlocks = 64;
constexpr int kWordsPerLane = kWaveBlocks * 16 / 64;
static_assert(kDirBlocksPerWG == (uint64_t)(kDT / 64) * kWaveBlocks, "directory tiling");

__global__ __launch_bounds__(kDT) void k_digit_dir(DigitDirArgs a) {
    __shared__ unsigned long long s_blk[kDT / 64][kWaveBlocks];
    __shared__ unsigned long long s_tot[kDT / 64][2];
    const uint32_t i = blockIdx.y;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t *D = a.digits + (uint64_t)i * a.dwords;
    const uint64_t blk0 = (uint64_t)blockIdx.x * kDirBlocksPerWG + (uint64_t)wv * kWaveBlocks;
    const uint64_t w0 = blk0 * 16;
    uint64_t x[kWordsPerLane];
#pragma unroll
    for (int u = 0; u < kWordsPerLane; u++) {
        const uint64_t w = w0 + (uint64_t)u * 64 + lane;
        x[u] = (w < a.dwords) ? D[w] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < kWordsPerLane; u++) {
        const uint64_t lo = x[u] & kEven, hi = (x[u] >> 1) & kEven;
        unsigned long long c = (unsigned long long)__popcll(lo & ~hi) |
                               ((unsigned long long)__popcll(hi & ~lo) << 16) |
                               ((unsigned long long)__popcll(lo & hi) << 32);
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) c += __shfl_xor(c, off, 64);
        if ((lane & 15) == 0) s_blk[wv][u * 4 + (lane >> 4)] = c;
    }
    __syncthreads();
    const uint64_t blk = blk0 + lane;
    const unsigned long long c = s_blk[wv][lane];
    const uint64_t c1 = c & 0xFFFF, c2 = (c >> 16) & 0xFFFF, c3 = (c >> 32) & 0xFFFF;
    uint64_t valid = 0;
    if (blk < a.nblk) valid = (a.n - blk * 512 < 512) ? a.n - blk * 512 : 512;
    const uint64_t c0 = valid - c1 - c2 - c3;  // padding digits are 0 and never counted
    const unsigned long long v01 = c0 | (c1 << 32), v23 = c2 | (c3 << 32);
    unsigned long long i01 = v01, i23 = v23;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long y01 = __shfl_up(i01, d, 64), y23 = __shfl_up(i23, d, 64);
        if (lane >= d) {
            i01 += y01;
            i23 += y23;
        }
    }
    if (lane == 63) {
        s_tot[wv][0] = i01;
        s_tot[wv][1] = i23;
    }
    __syncthreads();
    unsigned long long base01 = 0, base23 = 0, t01 = 0, t23 = 0;
#pragma unroll
    for (int w = 0; w < kDT / 64; w++) {
        base01 += (w < wv) ? s_tot[w][0] : 0ull;
        base23 += (w < wv) ? s_tot[w][1] : 0ull;
        t01 += s_tot[w][0];
        t23 += s_tot[w][1];
    }
    const unsigned long long b01 = base01 + i01 - v01, b23 = base23 + i23 - v23;
    if (blk < a.nblk) {
        uint64_t *E = a.dir + ((uint64_t)i * a.dir_stride + blk) * 4;
        E[0] = b01 & 0xFFFFFFFFull;
        E[1] = b01 >> 32;
        E[2] = b23 & 0xFFFFFFFFull;
        E[3] = b23 >> 32;
    }
    if (threadIdx.x == 0) {
        unsigned long long *ws = a.wsum + ((uint64_t)i * a.wg_per_level + blockIdx.x) * 4;
        ws[0] = t01 & 0xFFFFFFFFull;
        ws[1] = t01 >> 32;
        ws[2] = t23 & 0xFFFFFFFFull;
        ws[3] = t23 >> 32;
    }
}

// One workgroup per level: exclusive scan of the workgroup totals of each
// digit, in place; the level totals at entry nblk and zero padding entries.
__global__ __launch_bounds__(kDT) void k_digit_dir_fix(DigitDirArgs a) {
    __shared__ unsigned long long s_scan[kDT / 64];
    const uint32_t i = blockIdx.x;
    unsigned long long *ws = a.wsum + (uint64_t)i * a.wg_per_level * 4;
    const uint64_t per = (a.wg_per_level + kDT - 1) / kDT;
    const uint64_t k0 = (uint64_t)threadIdx.x * per;
    unsigned long long tot[4];
    constexpr uint64_t kFixPer = 16;
    if (per <= kFixPer) {
        // up to 2^29 positions per level: every sum of the thread loaded at
        // once (a loop of unknown length would wait for them one by one)
        unsigned long long v[kFixPer][4];
#pragma unroll
        for (uint64_t q = 0; q < kFixPer; q++)
#pragma unroll
            for (int d = 0; d < 4; d++) v[q][d] = (q < per && k0 + q < a.wg_per_level) ? ws[(k0 + q) * 4 + d] : 0ull;
#pragma unroll
        for (int d = 0; d < 4; d++) {
            unsigned long long sum = 0;
#pragma unroll
            for (uint64_t q = 0; q < kFixPer; q++) sum += v[q][d];
            unsigned long long off = excl_scan(sum, s_scan, &tot[d]);
#pragma unroll
            for (uint64_t q = 0; q < kFixPer; q++) {
                if (q < per && k0 + q < a.wg_per_level) ws[(k0 + q) * 4 + d] = off;
                off += v[q][d];
            }
        }
        uint64_t *E = a.dir + (uint64_t)i * a.dir_stride * 4;
        for (uint64_t t = a.nblk + threadIdx.x; t < a.dir_stride; t += kDT)
#pragma unroll
            for (int d = 0; d < 4; d++) E[t * 4 + d] = (t == a.nblk) ? tot[d] : 0ull;
        return;
    }
#pragma unroll
    for (int d = 0; d < 4; d++) {
        unsigned long long sum = 0;
        for (uint64_t t = k0; t < k0 + per && t < a.wg_per_level; t++) sum += ws[t * 4 + d];
        unsigned long long off = excl_scan(sum, s_scan, &tot[d]);
        for (uint64_t t = k0; t < k0 + per && t < a.wg_per_level; t++) {
            const unsigned long long v = ws[t * 4 + d];
            ws[t * 4 + d] = off;
            off += v;
        }
    }
    uint64_t *E = a.dir + (uint64_t)i * a.dir_stride * 4;
    for (uint64_t t = a.nblk + threadIdx.x; t < a.dir_stride; t += kDT)
#pragma unroll
        for (int d = 0; d < 4; d++) E[t * 4 + d] = (t == a.nblk) ? tot[d] : 0ull;
}

// Adds each directory workgroup's base to its blocks' entries.
__global__ __launch_bounds__(kDT) void k_digit_dir_apply(DigitDirArgs a) {
    const uint32_t i = blockIdx.y;
    const uint64_t blk = (uint64_t)blockIdx.x * kDT + threadIdx.x;
    if (blk >= a.nblk) return;
    const unsigned long long *ws = a.wsum + ((uint64_t)i * a.wg_per_level + blk / kDirBlocksPerWG) * 4;
    uint64_t *E = a.dir + ((uint64_t)i * a.dir_stride + blk) * 4;
#pragma unroll
    for (int d = 0; d < 4; d++) E[d] += ws[d];
}

}  // namespace

hipError_t launch_digit_dir(const DigitDirArgs &a, hipStream_t s) {
    if (a.levels == 0) return hipSuccess;
    hipError_t err;
    if (a.nblk) {
        hipLaunchKernelGGL(k_digit_dir, dim3((unsigned)a.wg_per_level, a.levels), dim3(kDT), 0, s, a);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    hipLaunchKernelGGL(k_digit_dir_fix, dim3(a.levels), dim3(kDT), 0, s, a);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (a.nblk) {
        hipLaunchKernelGGL(k_digit_dir_apply, dim3((unsigned)ceil_div(a.nblk, kDT), a.levels), dim3(kDT), 0, s, a);
        err = hipGetLastError();
    }
    return err;
}

}  // namespace wt
