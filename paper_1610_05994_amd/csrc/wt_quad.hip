// Four-way level split: one pass over T_i writes T_{i+2}.
//
// T_i is S stably sorted by its top i bits (Proposition 1), so the symbols of
// a level-i node v are a range of T_i, and its four grandchildren 4v + d
// (d = 2a + b, a = bit l-1-i, b = bit l-2-i) follow each other at level i + 2
// inside that range.  A symbol with digit d at position p goes to
//   start_{i+2}(4v + d) + (symbols of v with digit d before p),
// and with A(p), B(p), AB(p) the numbers of a-ones, b-ones and symbols with
// both bits set before p (over all of T_i), the count of digit d before p
// inside v is a fixed combination of p, A, B, AB minus its value at the
// node's start.  So one table entry per node, K(v), and the three prefix
// counts at the tile start give every destination:
//   digit 0: K0 + p - A - B + AB,  digit 1: K1 + B - AB,
//   digit 2: K2 + A - AB,          digit 3: K3 + AB.
// This is Algorithm pwt's count / prefix-sum / place, done for two bits of a
// node at once (the quaternary node of a 4-ary tree, Section 5), and the
// tile counts are Algorithm dd's per-segment counts (Section 3.2).
//
// Tiles inside one node stage their four runs in LDS, each at its
// destination's 16-byte phase, and write them out in aligned chunks; tiles
// spanning several nodes place every symbol directly.  The pass counts, for
// the next four-way level, the two following bits of every symbol per
// destination tile and per node.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wt_check.h"
#include "wt_internal.h"

namespace wt {

namespace {

#include "wt_wave.h"

// Counts before tile t of one count array: its superchunk's prefix plus the
// earlier tiles of the superchunk, four counts per lane (16-byte loads; the
// array holds round_up(ntiles, 4) entries).
__device__ __forceinline__ unsigned long long tile_prefix(const uint32_t *cnt, const unsigned long long *sup,
                                                          uint64_t t, int lane) {
    uint32_t pv = 0;
    const uint64_t q = t - t % kSup + 4 * (uint64_t)lane;
    if (q < t) {
        const uint4 c = *reinterpret_cast<const uint4 *>(cnt + q);
        pv = c.x + (q + 1 < t ? c.y : 0u) + (q + 2 < t ? c.z : 0u) + (q + 3 < t ? c.w : 0u);
    }
    return sup[t / kSup] + wave_sum32(pv);
}

template <typename M>
__device__ __forceinline__ uint32_t popm(M m) {
    return (sizeof(M) == 8) ? (uint32_t)__popcll((uint64_t)m) : (uint32_t)__popc((uint32_t)m);
}

// Counts of bit shc, of bit shd and of both over the symbols of a 16-byte chunk.
template <int W>
__device__ __forceinline__ uint3 chunk_counts(const uint4 &v, uint32_t shc, uint32_t shd) {
    const uint32_t lowbits = (W == 1) ? 0x01010101u : (W == 2) ? 0x00010001u : 1u;
    const uint32_t d4[4] = {v.x, v.y, v.z, v.w};
    uint3 r = make_uint3(0, 0, 0);
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint32_t c = (d4[q] >> shc) & lowbits, d = (d4[q] >> shd) & lowbits;
        r.x += __popc(c);
        r.y += __popc(d);
        r.z += __popc(c & d);
    }
    return r;
}

// Tiles over fewer nodes than this gather their next-level counts in LDS.
constexpr uint32_t kQuadNodeCap = 16;

template <int W, int B>
__host__ __device__ constexpr uint32_t quad_wave_bytes() {
    // four runs, each starting at its destination's phase inside a chunk; or
    // the direct path's counters (8 keys per node, three counts and a tile each)
    constexpr uint32_t stage = (uint32_t)(((tile_syms(W, B) + 8 * (16 / W)) * W + 15) / 16 * 16);
    constexpr uint32_t counters = 4 * 8 * kQuadNodeCap * 4;
    return stage > counters ? stage : counters;
}

// A single-node tile's next-level node counts (per run r: a'-ones, b'-ones
// with a' = 0, b'-ones with a' = 1), added up over the workgroup's tiles of
// the same node before they go out: consecutive tiles mostly share a node,
// and one atomic per tile on a few counters would serialise.
struct QuadRec {
    uint32_t v;  // the tile's node, or ~0u: no record
    uint32_t c[4][3];
};

template <int W, int B>
__device__ __forceinline__ void quad_tile(const QuadArgs &a, uint64_t t, uint8_t *s_wave, QuadRec *rec) {
    typedef typename ElemT<W>::T T;
    constexpr int E = B / W;
    constexpr uint32_t CH = 16 / W;
    constexpr uint64_t TILE = tile_syms(W, B);
    typedef typename MaskT<E>::T M;
    const int lane = threadIdx.x & 63;
    T *s_stage = reinterpret_cast<T *>(s_wave);

    const uint32_t sha = a.levels - 1 - a.level, shb = sha - 1;  // the digit's two bits
    const uint32_t nsh = a.levels - a.level;                       // node shift
    const uint64_t base = t * TILE;
    const uint64_t pos0 = base + (uint64_t)lane * E;
    const uint64_t nvalid = (a.n - base < TILE) ? a.n - base : TILE;

    uint4 raw[B / 16];
    const int nval = load_lane<W, B>(a.tin, pos0, a.n, raw);  // positions >= n read as 0
    const M ma = level_bits<W, B>(raw, sha), mb = level_bits<W, B>(raw, shb);
    const M mab = ma & mb;
    const uint32_t pa = popm(ma), pb = popm(mb), pab = popm(mab);
    const uint32_t ia = wave_incl_scan(pa), ib = wave_incl_scan(pb), iab = wave_incl_scan(pab);
    const uint32_t Ta = (uint32_t)__builtin_amdgcn_readlane((int)ia, 63);
    const uint32_t Tb = (uint32_t)__builtin_amdgcn_readlane((int)ib, 63);
    const uint32_t Tab = (uint32_t)__builtin_amdgcn_readlane((int)iab, 63);
    const uint32_t la = ia - pa, lb = ib - pb, lab = iab - pab;  // before this lane, inside the tile
    const unsigned long long PA = tile_prefix(a.cnt[0], a.sup[0], t, lane);
    const unsigned long long PB = tile_prefix(a.cnt[1], a.sup[1], t, lane);
    const unsigned long long PAB = tile_prefix(a.cnt[2], a.sup[2], t, lane);

    if (a.digits) {
        // 4-ary tree: digit level i / 2 lists the digit of every symbol of T_i
        constexpr int DPW = 32;
        if (E >= DPW) {
#pragma unroll
            for (int w = 0; w < E / DPW; w++) {
                uint64_t wd = 0;
#pragma unroll
                for (int k = 0; k < DPW; k++)
                    wd |= (uint64_t)((raw_elem<W, B>(raw, w * DPW + k) >> shb) & 3u) << (2 * k);
                const uint64_t widx = pos0 / DPW + w;
                if (widx < a.dwords) {
                    a.digits[widx] = wd;
                    note_write(&a.digits[widx], 8);
                }
            }
        } else {
            uint32_t part = 0;
#pragma unroll
            for (int k = 0; k < E; k++) part |= ((raw_elem<W, B>(raw, k) >> shb) & 3u) << (2 * k);
            uint64_t wd = part;
#pragma unroll
            for (int d = 1; d < DPW / E; d++) wd |= (uint64_t)__shfl_down(part, d, 64) << (d * 2 * E);
            if ((lane % (DPW / E)) == 0) {
                const uint64_t widx = pos0 / DPW;
                if (widx < a.dwords) {
                    a.digits[widx] = wd;
                    note_write(&a.digits[widx], 8);
                }
            }
        }
    }
    if (a.tout == nullptr) return;

    // node span of the tile (T_i is sorted by node)
    const uint32_t vf =
        (uint32_t)__builtin_amdgcn_readlane((int)((raw_elem<W, B>(raw, 0) & a.symmask) >> nsh), 0);
    uint32_t vl;
    {
        const uint64_t last = nvalid - 1;
        const int kl = (int)(last % E);
        uint32_t xv = 0;
#pragma unroll
        for (int k = 0; k < E; k++) xv = (k == kl) ? raw_elem<W, B>(raw, k) : xv;
        vl = (uint32_t)__builtin_amdgcn_readlane((int)((xv & a.symmask) >> nsh), (int)(last / E));
        vl = __builtin_amdgcn_readfirstlane(vl);
    }
    T *tout = reinterpret_cast<T *>(a.tout);
    const bool counting = a.cnt_next[0] != nullptr;
    const uint32_t shc = sha - 2, shd = sha - 3;  // the next digit's bits (when counting)
    const bool count_b = counting && a.ones_b_next != nullptr;
    // (counter slots by workgroup, as the workgroup merge below uses)
    const uint64_t tw = t - t % kWaves;
    const uint64_t slot_a = counting ? (tw & (a.slots_a_next - 1)) * a.nodes_a_next : 0;
    const uint64_t slot_b = count_b ? (tw & (a.slots_b_next - 1)) * a.nodes_b_next : 0;

    if (vf == vl) {
        const ulonglong2 k01 = a.K[2 * (uint64_t)vf], k23 = a.K[2 * (uint64_t)vf + 1];
        const uint32_t N0 = (uint32_t)nvalid - Ta - Tb + Tab, N1 = Tb - Tab, N2 = Ta - Tab, N3 = Tab;
        // destination of the tile's first symbol of each digit
        const uint64_t G0 = k01.x + base - PA - PB + PAB, G1 = k01.y + PB - PAB;
        const uint64_t G2 = k23.x + PA - PAB, G3 = k23.y + PAB;
        // staging: run d at slots [lo_d, lo_d + N_d), lo_d = the phase of G_d
        const uint32_t lo0 = (uint32_t)(G0 % CH);
        const uint32_t lo1 = (uint32_t)round_up(lo0 + N0, CH) + (uint32_t)(G1 % CH);
        const uint32_t lo2 = (uint32_t)round_up(lo1 + N1, CH) + (uint32_t)(G2 % CH);
        const uint32_t lo3 = (uint32_t)round_up(lo2 + N2, CH) + (uint32_t)(G3 % CH);
        {
            // this lane's first slot of each run
            const uint32_t before = (uint32_t)((uint64_t)lane * E < nvalid ? (uint64_t)lane * E : nvalid);
            uint32_t s0 = lo0 + before - la - lb + lab, s1 = lo1 + lb - lab, s2 = lo2 + la - lab, s3 = lo3 + lab;
#pragma unroll
            for (int k = 0; k < E; k++) {
                if (k < nval) {
                    const uint32_t x = raw_elem<W, B>(raw, k);
                    const uint32_t d = (x >> shb) & 3u;
                    const uint32_t sl = d == 0 ? s0 : (d == 1 ? s1 : (d == 2 ? s2 : s3));
                    s_stage[sl] = (T)x;
                    s0 += d == 0;
                    s1 += d == 1;
                    s2 += d == 2;
                    s3 += d == 3;
                }
            }
        }
        wave_sync();
        // write the four runs out: whole chunks as 16-byte stores, the
        // partial chunks at the run edges one symbol per lane; next-level
        // counts per (run, destination-tile parity), a, b and a & b packed
        // two 16-bit halves per word (a run holds at most TILE < 2^16)
        uint32_t cp[4][3];
#pragma unroll
        for (int r = 0; r < 4; r++) cp[r][0] = cp[r][1] = cp[r][2] = 0;
        uint64_t dt0_r[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const uint32_t lo = r == 0 ? lo0 : (r == 1 ? lo1 : (r == 2 ? lo2 : lo3));
            const uint32_t len = r == 0 ? N0 : (r == 1 ? N1 : (r == 2 ? N2 : N3));
            const uint64_t gb = (r == 0 ? G0 : (r == 1 ? G1 : (r == 2 ? G2 : G3))) - lo;  // destination = gb + slot
            const uint32_t fb = (lo + CH - 1) / CH, fe = (lo + len) / CH;  // whole chunks [fb, fe)
            const uint64_t dt0 = (gb + lo) / TILE;
            dt0_r[r] = dt0;
            for (uint32_t c = fb + lane; c < fe; c += 64) {
                const uint32_t s = c * CH;
                const uint4 v = *reinterpret_cast<const uint4 *>(&s_stage[s]);
                const uint64_t d = gb + s;
                if (d + CH <= a.n) {
                    *reinterpret_cast<uint4 *>(tout + d) = v;
                    if (counting) {
                        const uint3 cc = chunk_counts<W>(v, shc, shd);
                        const uint32_t sh16 = (d / TILE != dt0) ? 16u : 0u;
                        cp[r][0] += cc.x << sh16;
                        cp[r][1] += cc.y << sh16;
                        cp[r][2] += cc.z << sh16;
                    }
                }
            }
            // edge symbols: [lo, head_end) and [tail_start, lo + len)
            const uint32_t head_end = (fb < fe) ? fb * CH : lo + len;
            const uint32_t tail_start = (fb < fe) ? fe * CH : lo + len;
            const uint32_t head = head_end - lo, tail = lo + len - tail_start;
            if ((uint32_t)lane < head + tail) {
                const uint32_t s = ((uint32_t)lane < head) ? lo + lane : tail_start + (lane - head);
                const uint64_t d = gb + s;
                if (d < a.n) {
                    const uint32_t x = (uint32_t)s_stage[s];
                    tout[d] = (T)x;
                    if (counting) {
                        const uint32_t sh16 = (d / TILE != dt0) ? 16u : 0u;
                        const uint32_t c1 = (x >> shc) & 1u, d1 = (x >> shd) & 1u;
                        cp[r][0] += c1 << sh16;
                        cp[r][1] += d1 << sh16;
                        cp[r][2] += (c1 & d1) << sh16;
                    }
                }
            }
        }
        if (!counting) return;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const uint32_t sa = wave_sum32(cp[r][0]), sb = wave_sum32(cp[r][1]), sab = wave_sum32(cp[r][2]);
            if (lane == 0) {
                const uint64_t dt0 = dt0_r[r];
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const uint64_t dt = dt0 + h;
                    const uint32_t va = (sa >> (16 * h)) & 0xFFFFu, vb = (sb >> (16 * h)) & 0xFFFFu,
                                   vab = (sab >> (16 * h)) & 0xFFFFu;
                    if (va) atomicAdd(&a.cnt_next[0][dt], va);
                    if (vb) atomicAdd(&a.cnt_next[1][dt], vb);
                    if (vab) atomicAdd(&a.cnt_next[2][dt], vab);
                }
                const uint32_t ta = (sa & 0xFFFFu) + (sa >> 16), tb = (sb & 0xFFFFu) + (sb >> 16),
                               tab = (sab & 0xFFFFu) + (sab >> 16);
                rec->c[r][0] = ta;
                rec->c[r][1] = tb - tab;
                rec->c[r][2] = tab;
            }
        }
        if (lane == 0) rec->v = vf;
        return;
    }

    // Several nodes: every symbol goes straight to its destination, its
    // node's table entry loaded where the node changes (a lane's nodes never
    // decrease).  Next-level counts of tiles spanning fewer than kQuadNodeCap
    // nodes gather in LDS per (child, destination-tile parity) first, the
    // others go out by atomics.
    uint32_t *s_cnt = reinterpret_cast<uint32_t *>(s_wave);  // [key][3], then [key] tiles
    uint32_t *s_tix = s_cnt + 3 * 8 * kQuadNodeCap;
    const bool lds_counts = counting && (vl - vf < kQuadNodeCap);
    if (lds_counts) {
        for (uint32_t q = lane; q < 4 * 8 * kQuadNodeCap; q += 64) s_cnt[q] = 0;
        wave_sync();
    }
    unsigned long long A = PA + la, Bc = PB + lb, AB = PAB + lab;
    uint32_t cv = (raw_elem<W, B>(raw, 0) & a.symmask) >> nsh;
    ulonglong2 k01 = a.K[2 * (uint64_t)(nval > 0 ? cv : vf)], k23 = a.K[2 * (uint64_t)(nval > 0 ? cv : vf) + 1];
#pragma unroll
    for (int k = 0; k < E; k++) {
        if (k < nval) {
            const uint32_t x = raw_elem<W, B>(raw, k) & a.symmask;
            const uint32_t v = x >> nsh;
            if (v != cv) {
                cv = v;
                k01 = a.K[2 * (uint64_t)v];
                k23 = a.K[2 * (uint64_t)v + 1];
            }
            const uint64_t p = pos0 + k;
            const uint32_t ab = (x >> shb) & 3u;
            uint64_t dst;
            if (ab == 0) dst = k01.x + p - A - Bc + AB;
            else if (ab == 1) dst = k01.y + Bc - AB;
            else if (ab == 2) dst = k23.x + A - AB;
            else dst = k23.y + AB;
            A += ab >> 1;
            Bc += ab & 1u;
            AB += ab == 3;
            if (dst < a.n) {
                tout[dst] = (T)x;
                if (counting) {
                    const uint32_t c1 = (x >> shc) & 1u, d1 = (x >> shd) & 1u;
                    const uint64_t dt = dst / TILE;
                    if (lds_counts) {
                        if (c1 | d1) {
                            const uint32_t key = 8 * (v - vf) + 2 * ab + (uint32_t)(dt & 1);
                            if (c1) atomicAdd(&s_cnt[3 * key], 1u);
                            if (d1) atomicAdd(&s_cnt[3 * key + 1], 1u);
                            if (c1 & d1) atomicAdd(&s_cnt[3 * key + 2], 1u);
                            s_tix[key] = (uint32_t)dt;
                        }
                    } else {
                        const uint64_t g = 4 * (uint64_t)v + ab;
                        if (c1) {
                            atomicAdd(&a.cnt_next[0][dt], 1u);
                            atomicAdd(&a.ones_a_next[slot_a + g], 1ull);
                        }
                        if (d1) {
                            atomicAdd(&a.cnt_next[1][dt], 1u);
                            if (count_b) atomicAdd(&a.ones_b_next[slot_b + 2 * g + c1], 1ull);
                        }
                        if (c1 & d1) atomicAdd(&a.cnt_next[2][dt], 1u);
                    }
                }
            }
        }
    }
    if (lds_counts) {
        wave_sync();
        for (uint32_t key = lane; key < 8 * (vl - vf + 1); key += 64) {
            const uint32_t c = s_cnt[3 * key], d = s_cnt[3 * key + 1], cd = s_cnt[3 * key + 2];
            if (c | d) {
                const uint64_t dt = s_tix[key];
                const uint64_t g = 4 * (uint64_t)(vf + key / 8) + (key / 2) % 4;
                if (c) {
                    atomicAdd(&a.cnt_next[0][dt], c);
                    atomicAdd(&a.ones_a_next[slot_a + g], (unsigned long long)c);
                }
                if (d) atomicAdd(&a.cnt_next[1][dt], d);
                if (cd) atomicAdd(&a.cnt_next[2][dt], cd);
                if (count_b) {
                    if (d - cd) atomicAdd(&a.ones_b_next[slot_b + 2 * g], (unsigned long long)(d - cd));
                    if (cd) atomicAdd(&a.ones_b_next[slot_b + 2 * g + 1], (unsigned long long)cd);
                }
            }
        }
    }
}

template <int W, int B>
__global__ __launch_bounds__(kThreads) void k_quad(QuadArgs a) {
    __shared__ __align__(16) uint8_t s_all[kWaves * quad_wave_bytes<W, B>()];
    __shared__ QuadRec s_rec[kWaves];
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t t0 = (uint64_t)blockIdx.x * kWaves, t = t0 + wv;
    if ((threadIdx.x & 63) == 0) s_rec[wv].v = ~0u;
    if (t < a.ntiles) quad_tile<W, B>(a, t, s_all + wv * quad_wave_bytes<W, B>(), &s_rec[wv]);
    __syncthreads();
    // node counts of the single-node tiles, one atomic per (node, run,
    // count): thread (w, r, c) adds the records w.. of w's node when w is the
    // first record of that node
    const uint32_t j = threadIdx.x;
    if (j >= kWaves * 12 || a.ones_a_next == nullptr) return;
    const uint32_t w = j / 12, r = (j / 3) % 4, c = j % 3;
    const uint32_t v = s_rec[w].v;
    if (v == ~0u) return;
    for (uint32_t u = 0; u < w; u++)
        if (s_rec[u].v == v) return;
    uint32_t sum = 0;
    for (uint32_t u = w; u < kWaves; u++)
        if (s_rec[u].v == v) sum += s_rec[u].c[r][c];
    if (sum == 0) return;
    const uint64_t g = 4 * (uint64_t)v + r;  // the level-(i+2) node
    if (c == 0) {
        atomicAdd(&a.ones_a_next[(t0 & (a.slots_a_next - 1)) * a.nodes_a_next + g], (unsigned long long)sum);
    } else if (a.ones_b_next) {
        atomicAdd(&a.ones_b_next[(t0 & (a.slots_b_next - 1)) * a.nodes_b_next + 2 * g + (c - 1)],
                  (unsigned long long)sum);
    }
}

// ------------------------------------------------------------- ingest ---
template <int W, int B>
__global__ __launch_bounds__(kThreads) void k_quad_ingest(QuadIngestArgs a) {
    constexpr int E = B / W;
    constexpr uint64_t TILE = tile_syms(W, B);
    typedef typename MaskT<E>::T M;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.start0[0] = 0;
        a.start0[1] = a.n;
    }
    const uint64_t t = (uint64_t)blockIdx.x * kWaves + wv;
    if (t >= a.ntiles) return;
    uint4 raw[B / 16];
    const int nval = load_lane<W, B>(a.S, t * TILE + (uint64_t)lane * E, a.n, raw);
    bool bad = false;
    if (a.check) {
#pragma unroll
        for (int k = 0; k < E; k++) bad |= (k < nval) && (raw_elem<W, B>(raw, k) >= a.sigma);
    }
    const uint32_t sha = a.levels - 1, shb = a.levels - 2;
    const M ma = level_bits<W, B>(raw, sha), mb = level_bits<W, B>(raw, shb);
    const uint32_t ca = wave_sum32(popm(ma)), cb = wave_sum32(popm(mb)), cab = wave_sum32(popm(ma & mb));
    if (lane == 0) {
        a.cnt[0][t] = ca;
        a.cnt[1][t] = cb;
        a.cnt[2][t] = cab;
        if (ca) atomicAdd(&a.ones_a0[t & (a.slots_a0 - 1)], (unsigned long long)ca);
        const uint64_t sb = (t & (a.slots_b1 - 1)) * 2;
        if (cb - cab) atomicAdd(&a.ones_b1[sb], (unsigned long long)(cb - cab));
        if (cab) atomicAdd(&a.ones_b1[sb + 1], (unsigned long long)cab);
    }
    if (__any(bad) && lane == 0) atomicOr(a.tree_status, 1u);
}

// --------------------------------------------------------------- prep ---
// Node tables for nodes [b0, b0 + cn) (cn <= kScanChunk), given the three
// counts before b0; returns the three totals of the chunk.  Per node: the
// a-ones qa (level i counters) and the b-ones of its two level-(i+1)
// children q01, q11, summed over their counter slots into LDS first.
struct Sums3 {
    unsigned long long a, b, ab;
};

constexpr uint32_t kQuadChunk = 1024;

__device__ Sums3 quad_chunk(const QuadPrepArgs &p, uint64_t b0, Sums3 before, bool write) {
    __shared__ unsigned long long s_qa[kQuadChunk], s_q01[kQuadChunk], s_q11[kQuadChunk];
    __shared__ unsigned long long s_w[kWaves];
    const uint32_t tid = threadIdx.x;
    const uint64_t cn = (p.nodes - b0 < kQuadChunk) ? p.nodes - b0 : kQuadChunk;
    for (uint64_t v = tid; v < cn; v += kThreads) s_qa[v] = s_q01[v] = s_q11[v] = 0;
    __syncthreads();
    // slot sums: one thread per node, or kThreads / cn threads per node (each
    // a share of its slots, added up in LDS) when the chunk has few nodes
    if (cn >= kThreads) {
        for (uint64_t v = tid; v < cn; v += kThreads) {
            unsigned long long qa = 0, q01 = 0, q11 = 0;
            for (uint64_t sl = 0; sl < p.slots_a; sl++) qa += p.ones_a[sl * p.nodes + b0 + v];
            for (uint64_t sl = 0; sl < p.slots_b; sl++) {
                q01 += p.ones_b[sl * 2 * p.nodes + 2 * (b0 + v)];
                q11 += p.ones_b[sl * 2 * p.nodes + 2 * (b0 + v) + 1];
            }
            s_qa[v] = qa;
            s_q01[v] = q01;
            s_q11[v] = q11;
        }
    } else {
        const uint64_t groups = kThreads / cn, v = tid % cn, g = tid / cn;
        if (g < groups) {
            unsigned long long qa = 0, q01 = 0, q11 = 0;
            for (uint64_t sl = g; sl < p.slots_a; sl += groups) qa += p.ones_a[sl * p.nodes + b0 + v];
            for (uint64_t sl = g; sl < p.slots_b; sl += groups) {
                q01 += p.ones_b[sl * 2 * p.nodes + 2 * (b0 + v)];
                q11 += p.ones_b[sl * 2 * p.nodes + 2 * (b0 + v) + 1];
            }
            if (qa) atomicAdd(&s_qa[v], qa);
            if (q01) atomicAdd(&s_q01[v], q01);
            if (q11) atomicAdd(&s_q11[v], q11);
        }
    }
    __syncthreads();
    // four consecutive nodes per thread
    constexpr uint32_t per = kQuadChunk / kThreads;
    const uint64_t k0 = (uint64_t)tid * per;
    unsigned long long ta = 0, tb = 0, tab = 0;
#pragma unroll
    for (uint32_t q = 0; q < per; q++) {
        if (k0 + q < cn) {
            ta += s_qa[k0 + q];
            tb += s_q01[k0 + q] + s_q11[k0 + q];
            tab += s_q11[k0 + q];
        }
    }
    Sums3 tot;
    unsigned long long oa = block_excl_scan64(ta, s_w, &tot.a) + before.a;
    unsigned long long ob = block_excl_scan64(tb, s_w, &tot.b) + before.b;
    unsigned long long oab = block_excl_scan64(tab, s_w, &tot.ab) + before.ab;
    if (write) {
#pragma unroll
        for (uint32_t q = 0; q < per; q++) {
            const uint64_t v = b0 + k0 + q;
            if (k0 + q < cn) {
                const unsigned long long qa = s_qa[k0 + q], q01 = s_q01[k0 + q], q11 = s_q11[k0 + q];
                const uint64_t s = p.start[v], e = p.start[v + 1];
                const uint64_t st1 = s + (e - s - qa - q01), st2 = st1 + q01, st3 = st2 + (qa - q11);
                p.K[2 * v] = make_ulonglong2(oa + ob - oab, st1 - ob + oab);
                p.K[2 * v + 1] = make_ulonglong2(st2 - oa + oab, st3 - oab);
                if (p.start_next) {
                    p.start_next[4 * v] = s;
                    p.start_next[4 * v + 1] = st1;
                    p.start_next[4 * v + 2] = st2;
                    p.start_next[4 * v + 3] = st3;
                }
                oa += qa;
                ob += q01 + q11;
                oab += q11;
            }
        }
        if (p.start_next && b0 == 0 && tid == 0) p.start_next[4 * p.nodes] = p.n;
    }
    __syncthreads();
    return tot;
}

// grid (nsup, 3): superchunk c of count array j
__global__ __launch_bounds__(kThreads) void k_quad_supsum(QuadPrepArgs p) {
    __shared__ uint32_t s_w[kWaves];
    const uint32_t j = blockIdx.y, tid = threadIdx.x;
    const uint64_t t = (uint64_t)blockIdx.x * kSup + tid;
    const uint32_t v = wave_sum32(t < p.ntiles ? p.cnt[j][t] : 0u);
    if ((tid & 63) == 0) s_w[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        unsigned long long tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; w++) tot += s_w[w];
        p.supsum[j][blockIdx.x] = tot;
    }
}

// one workgroup: the superchunk prefixes, and the node tables when the level
// has at most kScanChunk nodes
__global__ __launch_bounds__(kThreads) void k_quad_prep(QuadPrepArgs p) {
    __shared__ unsigned long long s_w[kWaves];
    for (int j = 0; j < 3; j++) {
        unsigned long long carry = 0;
        for (uint64_t c0 = 0; c0 < p.nsup; c0 += kThreads) {
            const uint64_t c = c0 + threadIdx.x;
            const unsigned long long v = (c < p.nsup) ? p.supsum[j][c] : 0ull;
            unsigned long long tot;
            const unsigned long long ex = block_excl_scan64(v, s_w, &tot);
            if (c < p.nsup) p.sup[j][c] = carry + ex;
            carry += tot;
        }
    }
    if (p.nodes > kScanChunk) return;
    Sums3 before = {0, 0, 0};
    for (uint64_t b0 = 0; b0 < p.nodes; b0 += kQuadChunk) {
        const Sums3 t = quad_chunk(p, b0, before, true);
        before.a += t.a;
        before.b += t.b;
        before.ab += t.ab;
    }
}

// levels above kScanChunk nodes: chunk totals, their scan, then the tables
__global__ __launch_bounds__(kThreads) void k_quad_plan_reduce(QuadPrepArgs p) {
    const Sums3 t = quad_chunk(p, (uint64_t)blockIdx.x * kQuadChunk, Sums3{0, 0, 0}, false);
    if (threadIdx.x == 0) {
        p.partials[3 * blockIdx.x] = t.a;
        p.partials[3 * blockIdx.x + 1] = t.b;
        p.partials[3 * blockIdx.x + 2] = t.ab;
    }
}

__global__ __launch_bounds__(kThreads) void k_quad_plan_partials(QuadPrepArgs p, uint64_t nchunks) {
    __shared__ unsigned long long s_w[kWaves];
    for (int j = 0; j < 3; j++) {
        unsigned long long carry = 0;
        for (uint64_t c0 = 0; c0 < nchunks; c0 += kThreads) {
            const uint64_t c = c0 + threadIdx.x;
            const unsigned long long v = (c < nchunks) ? p.partials[3 * c + j] : 0ull;
            unsigned long long tot;
            const unsigned long long ex = block_excl_scan64(v, s_w, &tot);
            __syncthreads();
            if (c < nchunks) p.partials[3 * c + j] = carry + ex;
            carry += tot;
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_quad_plan_apply(QuadPrepArgs p) {
    const uint64_t c = blockIdx.x;
    const Sums3 before = {p.partials[3 * c], p.partials[3 * c + 1], p.partials[3 * c + 2]};
    (void)quad_chunk(p, c * kQuadChunk, before, true);
}

}  // namespace

#define WT_QUAD_LAUNCH(KERNEL, W_, LB_, GRID, ...)                                                    \
    do {                                                                                              \
        switch ((W_) * 1000 + (LB_)) {                                                                \
            case 1032: hipLaunchKernelGGL((KERNEL<1, 32>), GRID, dim3(kThreads), 0, __VA_ARGS__); break; \
            case 1064: hipLaunchKernelGGL((KERNEL<1, 64>), GRID, dim3(kThreads), 0, __VA_ARGS__); break; \
            case 2032: hipLaunchKernelGGL((KERNEL<2, 32>), GRID, dim3(kThreads), 0, __VA_ARGS__); break; \
            case 2064: hipLaunchKernelGGL((KERNEL<2, 64>), GRID, dim3(kThreads), 0, __VA_ARGS__); break; \
            case 2128: hipLaunchKernelGGL((KERNEL<2, 128>), GRID, dim3(kThreads), 0, __VA_ARGS__); break; \
            case 4032: hipLaunchKernelGGL((KERNEL<4, 32>), GRID, dim3(kThreads), 0, __VA_ARGS__); break; \
            case 4064: hipLaunchKernelGGL((KERNEL<4, 64>), GRID, dim3(kThreads), 0, __VA_ARGS__); break; \
            case 4128: hipLaunchKernelGGL((KERNEL<4, 128>), GRID, dim3(kThreads), 0, __VA_ARGS__); break; \
            default: return hipErrorInvalidValue;                                                     \
        }                                                                                             \
    } while (0)

hipError_t launch_quad(const QuadArgs &a, uint32_t width, uint32_t lane_bytes, hipStream_t s) {
    if (a.ntiles == 0) return hipSuccess;
    WT_QUAD_LAUNCH(k_quad, width, lane_bytes, dim3((uint32_t)ceil_div(a.ntiles, kWaves)), s, a);
    return hipGetLastError();
}

hipError_t launch_quad_ingest(const QuadIngestArgs &a, uint32_t width, uint32_t lane_bytes, hipStream_t s) {
    if (a.ntiles == 0) return hipSuccess;
    WT_QUAD_LAUNCH(k_quad_ingest, width, lane_bytes, dim3((uint32_t)ceil_div(a.ntiles, kWaves)), s, a);
    return hipGetLastError();
}

hipError_t launch_quad_prep(const QuadPrepArgs &p, hipStream_t s) {
    if (p.nsup) hipLaunchKernelGGL(k_quad_supsum, dim3((uint32_t)p.nsup, 3), dim3(kThreads), 0, s, p);
    hipLaunchKernelGGL(k_quad_prep, dim3(1), dim3(kThreads), 0, s, p);
    if (p.nodes > kScanChunk) {
        const uint64_t nc = ceil_div(p.nodes, kQuadChunk);
        hipLaunchKernelGGL(k_quad_plan_reduce, dim3((uint32_t)nc), dim3(kThreads), 0, s, p);
        hipLaunchKernelGGL(k_quad_plan_partials, dim3(1), dim3(kThreads), 0, s, p, nc);
        hipLaunchKernelGGL(k_quad_plan_apply, dim3((uint32_t)nc), dim3(kThreads), 0, s, p);
    }
    return hipGetLastError();
}

#ifdef WT_WRITE_CHECK
hipError_t write_check_quad(uint32_t *cnt, uint64_t base, uint64_t bytes) {
    return set_write_check_here(cnt, base, bytes);
}
#endif

}  // namespace wt
