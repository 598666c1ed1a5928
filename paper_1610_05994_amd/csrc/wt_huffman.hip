// Huffman-shaped wavelet tree kernels (compressed wavelet trees are future
// work in Section 5): the symbol histogram and the map of every symbol to
// its canonical code left-aligned to L bits.  The tree is then built by the
// level split of those codes (wt_build.hip) with every level compacted.
//
// With canonical codes, a code of length d (left-aligned) is smaller than
// the first d bits of every longer code, so in the order of the first d
// code bits the symbols whose code ends by depth d come first.  The level
// split over the left-aligned codes (T_d = the codes stably sorted by their
// first d bits, level d = bit d of T_d, Proposition 1 with L levels) thus
// lists at level d first the finished symbols, then, node after node, the
// internal nodes at depth d of the Huffman-shaped tree with their symbols
// in input order: depth d is level d without its first n - n_d positions,
// and the split keeps only those (its node tables shifted down by the
// symbols that finish at the next depth).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wt_internal.h"

namespace wt {

namespace {

#include "wt_wave.h"

constexpr int kHThreads = 256;
constexpr uint32_t kHistLds = 8192;  // alphabets up to this size count in LDS first

template <int W>
__device__ __forceinline__ uint32_t sym_load(const void *S, uint64_t j) {
    if (W == 1) return reinterpret_cast<const uint8_t *>(S)[j];
    if (W == 2) return reinterpret_cast<const uint16_t *>(S)[j];
    return reinterpret_cast<const uint32_t *>(S)[j];
}

__global__ __launch_bounds__(kHThreads) void k_hist_zero(unsigned long long *counts, uint32_t sigma) {
    for (uint64_t c = (uint64_t)blockIdx.x * kHThreads + threadIdx.x; c < sigma; c += (uint64_t)gridDim.x * kHThreads)
        counts[c] = 0;
}

// Symbols >= sigma are not counted (the build reports them).
template <int W, bool kLds>
__global__ __launch_bounds__(kHThreads) void k_hist(const void *S, uint64_t n, uint32_t sigma,
                                                    unsigned long long *counts) {
    __shared__ uint32_t s_h[kLds ? kHistLds : 1];
    if (kLds) {
        for (uint32_t c = threadIdx.x; c < sigma; c += kHThreads) s_h[c] = 0;
        __syncthreads();
    }
    const uint64_t stride = (uint64_t)gridDim.x * kHThreads;
    for (uint64_t j = (uint64_t)blockIdx.x * kHThreads + threadIdx.x; j < n; j += stride) {
        const uint32_t s = sym_load<W>(S, j);
        if (s < sigma) {
            if (kLds) atomicAdd(&s_h[s], 1u);
            else atomicAdd(&counts[s], 1ull);
        }
    }
    if (kLds) {
        __syncthreads();
        for (uint32_t c = threadIdx.x; c < sigma; c += kHThreads)
            if (s_h[c]) atomicAdd(&counts[c], (unsigned long long)s_h[c]);
    }
}

// One 16-byte chunk of S per thread (16 / W symbols), its codes stored as
// one run of 16 / W values of WO bytes; a chunk reaching past n goes symbol
// by symbol.
template <int W, int WO>
__global__ __launch_bounds__(kHThreads) void k_huff_map(const void *S, uint64_t n, const uint32_t *code_tab,
                                                        uint32_t sigma, uint32_t levels, void *K,
                                                        uint32_t *status) {
    constexpr int CH = 16 / W;
    const uint64_t chunks = (n + CH - 1) / CH;
    const uint64_t stride = (uint64_t)gridDim.x * kHThreads;
    bool bad = false;
    for (uint64_t c = (uint64_t)blockIdx.x * kHThreads + threadIdx.x; c < chunks; c += stride) {
        const uint64_t j0 = c * CH;
        const int cnt = (j0 + CH <= n) ? CH : (int)(n - j0);
        uint4 v = make_uint4(0, 0, 0, 0);
        if (cnt == CH) {
            v = reinterpret_cast<const uint4 *>(S)[c];
        } else {
            uint32_t d[4] = {0, 0, 0, 0};
            for (int e = 0; e < cnt; e++) {
                const uint32_t x = sym_load<W>(S, j0 + e);
                d[(e * W) >> 2] |= (W == 4) ? x : (x << (8 * ((e * W) & 3)));
            }
            v = make_uint4(d[0], d[1], d[2], d[3]);
        }
        constexpr int NW = (CH * WO) / 4;  // 32-bit words of the chunk's codes (CH * WO >= 4)
        uint32_t wd[NW];
#pragma unroll
        for (int q = 0; q < NW; q++) wd[q] = 0;
#pragma unroll
        for (int e = 0; e < CH; e++) {
            const uint32_t s = chunk_elem<W>(v, e);
            uint32_t k = 0;
            if (e < cnt) {
                if (s >= sigma) {
                    bad = true;
                } else {
                    const uint32_t ent = code_tab[s];
                    const uint32_t len = ent & 31u;
                    if (!(ent & kHuffPresent)) bad = true;
                    else if (len) k = (ent >> 8) << (levels - len);
                }
            }
            wd[(e * WO) >> 2] |= (WO == 4) ? k : (k << (8 * ((e * WO) & 3)));
        }
        if (K == nullptr) continue;  // (no levels: the symbols are only checked)
        uint8_t *dst = reinterpret_cast<uint8_t *>(K) + j0 * WO;  // CH * WO-byte aligned
        if (cnt == CH) {
            if (NW >= 4) {
#pragma unroll
                for (int q = 0; q < NW / 4; q++)
                    reinterpret_cast<uint4 *>(dst)[q] = make_uint4(wd[4 * q], wd[4 * q + 1], wd[4 * q + 2], wd[4 * q + 3]);
            } else if (NW == 2) {
                *reinterpret_cast<uint2 *>(dst) = make_uint2(wd[0], wd[NW - 1]);
            } else {
                *reinterpret_cast<uint32_t *>(dst) = wd[0];
            }
        } else {
            for (int e = 0; e < cnt; e++) {
                const uint32_t k = (WO == 4) ? wd[e] : ((wd[(e * WO) >> 2] >> (8 * ((e * WO) & 3))) & ((1u << (8 * WO)) - 1u));
                if (WO == 1) dst[e] = (uint8_t)k;
                else if (WO == 2) reinterpret_cast<uint16_t *>(dst)[e] = (uint16_t)k;
                else reinterpret_cast<uint32_t *>(dst)[e] = k;
            }
        }
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(status, 1u);
}

}  // namespace

hipError_t launch_histogram(const void *S, uint64_t n, uint32_t width, uint32_t sigma, unsigned long long *counts,
                            hipStream_t s) {
    const uint32_t zb = (uint32_t)(ceil_div(sigma, kHThreads) < 4096 ? ceil_div(sigma, kHThreads) : 4096);
    hipLaunchKernelGGL(k_hist_zero, dim3(zb ? zb : 1), dim3(kHThreads), 0, s, counts, sigma);
    if (n == 0) return hipGetLastError();
    const uint64_t want = ceil_div(n, (uint64_t)kHThreads * 16);
    const uint32_t g = (uint32_t)(want < 2048 ? (want ? want : 1) : 2048);
    const bool lds = sigma <= kHistLds;
#define WT_HIST(W_)                                                                                    \
    if (lds) hipLaunchKernelGGL((k_hist<W_, true>), dim3(g), dim3(kHThreads), 0, s, S, n, sigma, counts); \
    else hipLaunchKernelGGL((k_hist<W_, false>), dim3(g), dim3(kHThreads), 0, s, S, n, sigma, counts)
    if (width == 1) { WT_HIST(1); }
    else if (width == 2) { WT_HIST(2); }
    else if (width == 4) { WT_HIST(4); }
    else return hipErrorInvalidValue;
#undef WT_HIST
    return hipGetLastError();
}

hipError_t launch_huff_map(const void *S, uint64_t n, uint32_t width, const uint32_t *code_tab, uint32_t sigma,
                           uint32_t levels, void *K, uint32_t wout, uint32_t *status, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t want = ceil_div(ceil_div(n, 16 / width), (uint64_t)kHThreads);
    const dim3 g((uint32_t)(want < 16384 ? (want ? want : 1) : 16384));
    switch (width * 10 + wout) {
        case 11: hipLaunchKernelGGL((k_huff_map<1, 1>), g, dim3(kHThreads), 0, s, S, n, code_tab, sigma, levels, K, status); break;
        case 12: hipLaunchKernelGGL((k_huff_map<1, 2>), g, dim3(kHThreads), 0, s, S, n, code_tab, sigma, levels, K, status); break;
        case 14: hipLaunchKernelGGL((k_huff_map<1, 4>), g, dim3(kHThreads), 0, s, S, n, code_tab, sigma, levels, K, status); break;
        case 21: hipLaunchKernelGGL((k_huff_map<2, 1>), g, dim3(kHThreads), 0, s, S, n, code_tab, sigma, levels, K, status); break;
        case 22: hipLaunchKernelGGL((k_huff_map<2, 2>), g, dim3(kHThreads), 0, s, S, n, code_tab, sigma, levels, K, status); break;
        case 24: hipLaunchKernelGGL((k_huff_map<2, 4>), g, dim3(kHThreads), 0, s, S, n, code_tab, sigma, levels, K, status); break;
        case 41: hipLaunchKernelGGL((k_huff_map<4, 1>), g, dim3(kHThreads), 0, s, S, n, code_tab, sigma, levels, K, status); break;
        case 42: hipLaunchKernelGGL((k_huff_map<4, 2>), g, dim3(kHThreads), 0, s, S, n, code_tab, sigma, levels, K, status); break;
        case 44: hipLaunchKernelGGL((k_huff_map<4, 4>), g, dim3(kHThreads), 0, s, S, n, code_tab, sigma, levels, K, status); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace wt
