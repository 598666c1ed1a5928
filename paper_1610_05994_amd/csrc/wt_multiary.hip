// Directories of the 4-ary tree's digit levels.  Entry k of a level holds
// the counts of digits 0, 1, 2 and 3 in positions [0, min(512 k, n)): the
// rank structure of the one-pointer-per-level representation (Section 2.3)
// with four symbols per level instead of two.
//
// One thread per 512-position block (sixteen 32-digit words) counts its
// digits with popcounts over the two bit planes of the words; the workgroup
// scans the counts of its blocks, the workgroup totals of a level are scanned
// by one workgroup, and a last pass adds each workgroup's base.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wt_internal.h"

namespace wt {

namespace {

constexpr int kDT = (int)kDirBlocksPerWG;  // threads per workgroup
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

// Counts of digits 1, 2, 3 in a 32-digit word (padding digits are 0).
__device__ __forceinline__ void count123(uint64_t w, uint32_t &c1, uint32_t &c2, uint32_t &c3) {
    const uint64_t lo = w & kEven, hi = (w >> 1) & kEven;
    c1 += (uint32_t)__popcll(lo & ~hi);
    c2 += (uint32_t)__popcll(hi & ~lo);
    c3 += (uint32_t)__popcll(lo & hi);
}

// Block counts and their workgroup-local prefixes: counts (0, 1) and (2, 3)
// travel packed as two 32-bit halves of a u64 (a workgroup holds at most
// kDT * 512 < 2^32 positions).
__global__ __launch_bounds__(kDT) void k_digit_dir(DigitDirArgs a) {
    __shared__ unsigned long long s_scan[kDT / 64];
    const uint32_t i = blockIdx.y;
    const uint64_t blk = (uint64_t)blockIdx.x * kDT + threadIdx.x;
    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    if (blk < a.nblk) {
        const uint64_t *D = a.digits + (uint64_t)i * a.dwords;
#pragma unroll 4
        for (int q = 0; q < 16; q++) {
            const uint64_t w = blk * 16 + q;
            if (w < a.dwords) count123(D[w], c1, c2, c3);
        }
        const uint64_t valid = (a.n - blk * 512 < 512) ? a.n - blk * 512 : 512;
        c0 = (uint32_t)valid - c1 - c2 - c3;
    }
    unsigned long long t01, t23;
    const unsigned long long b01 = excl_scan((unsigned long long)c0 | ((unsigned long long)c1 << 32), s_scan, &t01);
    const unsigned long long b23 = excl_scan((unsigned long long)c2 | ((unsigned long long)c3 << 32), s_scan, &t23);
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
    const unsigned long long *ws = a.wsum + ((uint64_t)i * a.wg_per_level + blockIdx.x) * 4;
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
        hipLaunchKernelGGL(k_digit_dir_apply, dim3((unsigned)a.wg_per_level, a.levels), dim3(kDT), 0, s, a);
        err = hipGetLastError();
    }
    return err;
}

}  // namespace wt
