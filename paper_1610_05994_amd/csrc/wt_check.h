// Write counting for the debug build (compiled with -DWT_WRITE_CHECK; the
// product build compiles note_write to nothing).
//
// Every store of bitmap or digit words also counts, per 16-bit granule of a
// span of device memory set by wt_debug_write_counters, how many times the
// granule was stored.  A build keeps its promise of one writer per word (no
// atomics on the bitmaps) when every granule of its bitmaps is stored
// exactly once, padding included.  Each translation unit keeps its own copy
// of the span (a static device variable: the library is built without
// relocatable device code) and exports one setter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wt {

#ifdef WT_WRITE_CHECK
struct WriteCheck {
    uint32_t *cnt;   // one counter per 16-bit granule of [base, base + bytes)
    uint64_t base, bytes;
};
static __device__ WriteCheck g_write_check;

__device__ __forceinline__ void note_write(const void *p, uint32_t bytes) {
    const WriteCheck w = g_write_check;
    const uint64_t off = (uint64_t)(uintptr_t)p - w.base;
    if (w.cnt != nullptr && off < w.bytes)
        for (uint32_t q = 0; q < bytes / 2; q++) atomicAdd(&w.cnt[off / 2 + q], 1u);
}

static inline hipError_t set_write_check_here(uint32_t *cnt, uint64_t base, uint64_t bytes) {
    const WriteCheck w{cnt, base, bytes};
    return hipMemcpyToSymbol(HIP_SYMBOL(g_write_check), &w, sizeof(w));
}
#else
__device__ __forceinline__ void note_write(const void *, uint32_t) {}
#endif

}  // namespace wt
