// Wave-level helpers shared by the level-split kernels (included inside
// namespace wt { namespace { ... } } of each kernel file, so every
// translation unit keeps its own internal copies): symbol extraction from
// 16-byte lane loads, DPP wave scans, the block scan, and level bits.
#pragma once

template <int W> struct ElemT;
template <> struct ElemT<1> { typedef uint8_t T; };
template <> struct ElemT<2> { typedef uint16_t T; };
template <> struct ElemT<4> { typedef uint32_t T; };

// Wave-wide operations on DPP (register-to-register lane moves; GFX9 row
// shifts and row broadcasts), not the LDS crossbar.  The whole wave must be
// active.  DPP controls: row_shr:n = 0x110 + n, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143, wave_shr:1 = 0x138.
__device__ __forceinline__ uint32_t dpp_row_shr(uint32_t v, int n) {
    switch (n) {
        case 1: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);
        case 2: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);
        case 4: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);
        default: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);
    }
}

// Inclusive prefix sum over the 64 lanes: a scan inside each row of 16,
// then row 0's total into row 1 and row 2's into row 3, then lane 31's
// into rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += dpp_row_shr(v, 1);
    v += dpp_row_shr(v, 2);
    v += dpp_row_shr(v, 4);
    v += dpp_row_shr(v, 8);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
    return v;
}

// Value of the previous lane (lane 0 gets `first`).
__device__ __forceinline__ uint32_t wave_prev_lane(uint32_t v, uint32_t first) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)first, (int)v, 0x138, 0xf, 0xf, false);
}

// Inclusive prefix maximum over the 64 lanes (DPP; lanes shifted in read 0).
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
    uint32_t t;
    t = dpp_row_shr(v, 1); v = v > t ? v : t;
    t = dpp_row_shr(v, 2); v = v > t ? v : t;
    t = dpp_row_shr(v, 4); v = v > t ? v : t;
    t = dpp_row_shr(v, 8); v = v > t ? v : t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false); v = v > t ? v : t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false); v = v > t ? v : t;
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
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(v), 63);
}

// Exclusive scan of one value per thread over the block (kThreads threads);
// *total receives the sum.  Uses s_w (kWaves entries) and synchronises.
__device__ __forceinline__ unsigned long long block_excl_scan64(unsigned long long v, unsigned long long *s_w,
                                                                unsigned long long *total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long incl = wave_incl_scan64(v);
    if (lane == 63) s_w[wv] = incl;
    __syncthreads();
    unsigned long long off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) {
        off += (w < wv) ? s_w[w] : 0ull;
        tot += s_w[w];
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

// Symbol e (0 <= e < 16/W) of a 16-byte chunk.
template <int W>
__device__ __forceinline__ uint32_t chunk_elem(const uint4 &v, int e) {
    const uint32_t d4[4] = {v.x, v.y, v.z, v.w};
    const uint32_t d = d4[(e * W) >> 2];
    return (W == 4) ? d : ((d >> (8 * ((e * W) & 3))) & ((1u << (8 * W)) - 1u));
}

// Symbol k (0 <= k < B/W) of one lane's B bytes.
template <int W, int B>
__device__ __forceinline__ uint32_t raw_elem(const uint4 (&raw)[B / 16], int k) {
    return chunk_elem<W>(raw[k / (16 / W)], k % (16 / W));
}

// Load the B/W symbols of one lane starting at position pos (a multiple of
// B/W, so full loads are 16-byte aligned).  Positions >= n read as 0;
// returns the number of symbols below n.
template <int W, int B>
__device__ __forceinline__ int load_lane(const void *src, uint64_t pos, uint64_t n, uint4 (&raw)[B / 16]) {
    typedef typename ElemT<W>::T T;
    constexpr int E = B / W;
    constexpr int Q = B / 16;
    const T *s = reinterpret_cast<const T *>(src);
    if (pos + E <= n) {
        const uint4 *p = reinterpret_cast<const uint4 *>(s + pos);
#pragma unroll
        for (int q = 0; q < Q; q++) raw[q] = p[q];
        return E;
    }
    const int nval = pos < n ? (int)(n - pos) : 0;
    uint32_t d[4 * Q];
#pragma unroll
    for (int q = 0; q < 4 * Q; q++) d[q] = 0;
#pragma unroll
    for (int k = 0; k < E; k++) {
        const uint32_t v = (k < nval) ? (uint32_t)s[pos + k] : 0u;
        d[(k * W) >> 2] |= (W == 4) ? v : (v << (8 * ((k * W) & 3)));
    }
#pragma unroll
    for (int q = 0; q < Q; q++) raw[q] = make_uint4(d[4 * q], d[4 * q + 1], d[4 * q + 2], d[4 * q + 3]);
    return nval;
}

template <int E> struct MaskT { typedef uint32_t T; };  // E <= 32
template <> struct MaskT<64> { typedef uint64_t T; };

// Orders this wave's LDS accesses (a wave's LDS operations execute in order).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Level bits (bit sh) of one lane's E = B/W symbols, symbol k at bit k.
template <int W, int B>
__device__ __forceinline__ typename MaskT<B / W>::T level_bits(const uint4 (&raw)[B / 16], uint32_t sh) {
    typedef typename MaskT<B / W>::T M;
    constexpr int D = B / 4;  // dwords per lane
    M mb = 0;
#pragma unroll
    for (int q = 0; q < D; q++) {
        const uint4 &c = raw[q / 4];
        const uint32_t d = (q % 4 == 0) ? c.x : (q % 4 == 1) ? c.y : (q % 4 == 2) ? c.z : c.w;
        if (W == 1) {
            // gather bit sh of the four bytes into a nibble (no carries: the
            // sixteen partial products land on distinct bits)
            const uint32_t nib = (((d >> sh) & 0x01010101u) * 0x10204080u) >> 28;
            mb |= (M)nib << (4 * q);
        } else if (W == 2) {
            const uint32_t two = ((d >> sh) & 1u) | (((d >> (16 + sh)) & 1u) << 1);
            mb |= (M)two << (2 * q);
        } else {
            mb |= (M)((d >> sh) & 1u) << q;
        }
    }
    return mb;
}

