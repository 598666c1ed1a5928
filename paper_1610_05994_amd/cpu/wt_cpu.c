/*
 * Multicore CPU construction of the pointerless wavelet tree (OpenMP), the
 * paper's two parallel algorithms as a host-side comparator for the GPU
 * library:
 *
 *  - pwt (Section 3.1): every level is built independently from S, one level
 *    per thread: count the symbols of each level-i node (s >> (l-i),
 *    Proposition 1), turn the counts into node offsets by an exclusive
 *    prefix sum, then walk S in input order and write each symbol's level
 *    bit at its node's running offset.
 *  - dd (Section 3.2): S is cut into one segment per thread; each thread
 *    counts its segment's symbols per (level, node); a prefix sum over the
 *    segments gives each thread the global position of its part of every
 *    node; every thread then writes its bits there.  Only the first and
 *    last word of a thread's part of a node can be shared with a
 *    neighbouring thread, and those are written with atomic ORs.
 *
 * Output layout is the library's: per level round_up(ceil(n/64), 8) words,
 * LSB-first, zero past n, and a rank directory of ceil(n/512) + 1 absolute
 * counts in a slot of round_up(that, 8) entries (zero padding).
 *
 * This file shares nothing with the test oracle or the GPU kernels.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { WTC_OK = 0, WTC_EINVAL = 1, WTC_ERANGE = 2, WTC_ENOMEM = 3 };

static uint32_t levels_of(uint32_t sigma) {
    uint32_t l = 0;
    while (l < 32 && (1ull << l) < sigma) l++;
    return l;
}

uint64_t wtc_words(uint64_t n) { return ((n + 63) / 64 + 7) / 8 * 8; }
uint64_t wtc_rank_stride(uint64_t n) { return ((n + 511) / 512 + 1 + 7) / 8 * 8; }

static inline uint32_t sym_at(const void *S, uint32_t width, uint64_t k) {
    if (width == 1) return ((const uint8_t *)S)[k];
    if (width == 2) return ((const uint16_t *)S)[k];
    return ((const uint32_t *)S)[k];
}

static int check_args(const void *S, uint64_t n, uint32_t sigma, uint32_t width, const uint64_t *bits) {
    if ((n > 0 && !S) || !bits || sigma == 0 || sigma > (1u << 24)) return WTC_EINVAL;
    if (width != 1 && width != 2 && width != 4) return WTC_EINVAL;
    if (width < 4 && (uint64_t)sigma > (1ull << (8 * width))) return WTC_EINVAL;
    return WTC_OK;
}

static int any_out_of_range(const void *S, uint64_t n, uint32_t sigma, uint32_t width) {
    int bad = 0;
#pragma omp parallel for reduction(| : bad) schedule(static)
    for (uint64_t k = 0; k < n; k++) bad |= sym_at(S, width, k) >= sigma;
    return bad;
}

/* Rank directories of all levels from finished bitmaps (parallel over
 * levels and blocks of 512 positions). */
static void fill_ranks(const uint64_t *bits, uint64_t n, uint32_t l, uint64_t *ranks) {
    const uint64_t W = wtc_words(n), K = (n + 511) / 512 + 1, KS = wtc_rank_stride(n);
    const uint64_t nblk = (n + 511) / 512;
    uint64_t *blk = (uint64_t *)malloc(sizeof(uint64_t) * (nblk ? nblk : 1) * (l ? l : 1));
    if (!blk) return;
#pragma omp parallel for collapse(2) schedule(static)
    for (uint32_t i = 0; i < l; i++)
        for (uint64_t b = 0; b < nblk; b++) {
            const uint64_t *w = bits + (uint64_t)i * W + 8 * b;
            uint64_t c = 0;
            for (int k = 0; k < 8; k++) c += (uint64_t)__builtin_popcountll(w[k]);
            blk[(uint64_t)i * nblk + b] = c;
        }
#pragma omp parallel for schedule(static)
    for (uint32_t i = 0; i < l; i++) {
        uint64_t *R = ranks + (uint64_t)i * KS;
        uint64_t acc = 0;
        for (uint64_t b = 0; b < nblk; b++) {
            R[b] = acc;
            acc += blk[(uint64_t)i * nblk + b];
        }
        for (uint64_t k = nblk; k < KS; k++) R[k] = (k < K) ? acc : 0;
    }
    free(blk);
}

/* pwt: one level per thread. */
int wtc_build_pwt(const void *S, uint64_t n, uint32_t sigma, uint32_t width, uint64_t *bits, uint64_t *ranks,
                  int threads) {
    int rc = check_args(S, n, sigma, width, bits);
    if (rc != WTC_OK) return rc;
    const uint32_t l = levels_of(sigma);
    const uint64_t W = wtc_words(n);
    if (threads > 0) omp_set_num_threads(threads);
    if (any_out_of_range(S, n, sigma, width)) return WTC_ERANGE;
    memset(bits, 0, sizeof(uint64_t) * W * l);
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
    for (uint32_t i = 0; i < l; i++) {
        const uint32_t nsh = l - i, sh = l - 1 - i;
        const uint64_t nodes = 1ull << i;
        uint64_t *off = (uint64_t *)calloc(nodes, sizeof(uint64_t));
        if (!off) { fail = 1; continue; }
        for (uint64_t k = 0; k < n; k++) off[sym_at(S, width, k) >> nsh]++;
        uint64_t acc = 0;
        for (uint64_t v = 0; v < nodes; v++) {
            const uint64_t c = off[v];
            off[v] = acc;
            acc += c;
        }
        uint64_t *B = bits + (uint64_t)i * W;
        for (uint64_t k = 0; k < n; k++) {
            const uint32_t s = sym_at(S, width, k);
            const uint64_t p = off[s >> nsh]++;
            B[p >> 6] |= (uint64_t)((s >> sh) & 1u) << (p & 63);
        }
        free(off);
    }
    if (fail) return WTC_ENOMEM;
    if (ranks) fill_ranks(bits, n, l, ranks);
    return WTC_OK;
}

/* dd: one segment of S per thread. */
int wtc_build_dd(const void *S, uint64_t n, uint32_t sigma, uint32_t width, uint64_t *bits, uint64_t *ranks,
                 int threads) {
    int rc = check_args(S, n, sigma, width, bits);
    if (rc != WTC_OK) return rc;
    const uint32_t l = levels_of(sigma);
    const uint64_t W = wtc_words(n);
    if (threads > 0) omp_set_num_threads(threads);
    if (any_out_of_range(S, n, sigma, width)) return WTC_ERANGE;
    memset(bits, 0, sizeof(uint64_t) * W * l);
    if (l == 0 || n == 0) {
        if (ranks) fill_ranks(bits, n, l, ranks);
        return WTC_OK;
    }
    const int p = omp_get_max_threads();
    /* per (level, node) tables, node v of level i at entry (2^i - 1) + v:
     * cnt = the segment's symbols there, then the end of the thread's part
     * rounded down to a word; first = the part's first position, then the
     * running position; lo = the part's first position rounded up to a word.
     * Words in [lo, hi) are written by this thread only. */
    const uint64_t entries = (1ull << l) - 1;
    uint64_t *cnt = (uint64_t *)calloc((size_t)p * entries, sizeof(uint64_t));
    uint64_t *first = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)p * entries);
    uint64_t *lo = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)p * entries);
    if (!cnt || !first || !lo) {
        free(cnt);
        free(first);
        free(lo);
        return WTC_ENOMEM;
    }
#pragma omp parallel num_threads(p)
    {
        const int t = omp_get_thread_num();
        const uint64_t a = n * (uint64_t)t / p, b = n * (uint64_t)(t + 1) / p;
        uint64_t *c = cnt + (uint64_t)t * entries;
        uint64_t *cur = first + (uint64_t)t * entries;
        uint64_t *l0 = lo + (uint64_t)t * entries;
        /* local counts per (level, node) */
        for (uint64_t k = a; k < b; k++) {
            const uint32_t s = sym_at(S, width, k);
            for (uint32_t i = 0; i < l; i++) c[((1ull << i) - 1) + (s >> (l - i))]++;
        }
#pragma omp barrier
        /* global positions: node by node, segment by segment (levels over threads) */
#pragma omp for schedule(dynamic, 1)
        for (uint32_t i = 0; i < l; i++) {
            const uint64_t base = (1ull << i) - 1, nodes = 1ull << i;
            uint64_t acc = 0;
            for (uint64_t v = 0; v < nodes; v++)
                for (int q = 0; q < p; q++) {
                    first[(uint64_t)q * entries + base + v] = acc;
                    acc += cnt[(uint64_t)q * entries + base + v];
                }
        }
        for (uint64_t e = 0; e < entries; e++) {
            const uint64_t start = cur[e], end = start + c[e];
            l0[e] = (start + 63) & ~63ull;
            c[e] = end & ~63ull;
        }
        for (uint64_t k = a; k < b; k++) {
            const uint32_t s = sym_at(S, width, k);
            for (uint32_t i = 0; i < l; i++) {
                const uint64_t e = ((1ull << i) - 1) + (s >> (l - i));
                const uint64_t pos = cur[e]++;
                if ((s >> (l - 1 - i)) & 1u) {
                    uint64_t *w = bits + (uint64_t)i * W + (pos >> 6);
                    const uint64_t m = 1ull << (pos & 63);
                    if (pos >= l0[e] && pos < c[e]) *w |= m;
                    else __atomic_fetch_or(w, m, __ATOMIC_RELAXED);
                }
            }
        }
    }
    free(lo);
    free(cnt);
    free(first);
    if (ranks) fill_ranks(bits, n, l, ranks);
    return WTC_OK;
}
