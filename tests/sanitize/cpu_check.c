/*
 * The CPU code under AddressSanitizer and UndefinedBehaviorSanitizer: the
 * oracle (every variant, its queries and decode) and the multicore pwt / dd
 * comparator, on many small seeded inputs; pwt and dd are compared with the
 * oracle word by word.  Built and run by tests/test_sanitizers.py; exits
 * non-zero on the first mismatch (the sanitizers abort on their own
 * findings).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

uint32_t wto_levels(uint32_t sigma);
uint64_t wto_words_per_level(uint64_t n);
uint64_t wto_rank_stride(uint64_t n);
int wto_build(const void *S, uint64_t n, uint32_t sigma, uint32_t width, uint64_t *B, uint64_t *R);
int wto_access(const uint64_t *B, uint64_t n, uint32_t sigma, uint64_t i, uint32_t *sym, uint32_t *tb,
               uint64_t *ti);
int wto_rank(const uint64_t *B, uint64_t n, uint32_t sigma, uint32_t c, uint64_t i, uint64_t *out);
int wto_select(const uint64_t *B, uint64_t n, uint32_t sigma, uint32_t c, uint64_t j, uint64_t *out);
int wto_decode(const uint64_t *B, uint64_t n, uint32_t sigma, uint32_t *out);
int wto_build_matrix(const void *S, uint64_t n, uint32_t sigma, uint32_t width, uint64_t *B, uint64_t *R,
                     uint64_t *Z);
int wto_matrix_access(const uint64_t *B, const uint64_t *Z, uint64_t n, uint32_t sigma, uint64_t i, uint32_t *sym);
uint32_t wto_levels4(uint32_t sigma);
uint64_t wto_words4(uint64_t n);
int wto_build4(const void *S, uint64_t n, uint32_t sigma, uint32_t width, uint64_t *D, uint64_t *R);
int wto_access4(const uint64_t *D, uint64_t n, uint32_t sigma, uint64_t i, uint32_t *sym);
int wto_huffman_lengths(const uint64_t *counts, uint32_t sigma, uint8_t *len, uint32_t *maxlen);
int wto_huffman_codes(const uint8_t *len, uint32_t sigma, uint32_t maxlen, uint32_t *code);
int wto_build_huffman(const void *S, uint64_t n, uint32_t sigma, uint32_t width, const uint8_t *len,
                      const uint32_t *code, uint32_t maxlen, const uint64_t *bofs, const uint64_t *rofs,
                      uint64_t *B, uint64_t *R);
int wtc_build_pwt(const void *S, uint64_t n, uint32_t sigma, uint32_t width, uint64_t *bits, uint64_t *ranks,
                  int threads);
int wtc_build_dd(const void *S, uint64_t n, uint32_t sigma, uint32_t width, uint64_t *bits, uint64_t *ranks,
                 int threads);

static uint64_t rng = 88172645463325252ull;
static uint64_t next(void) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return rng;
}

static int fails = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            fails++;                                                      \
        }                                                                 \
    } while (0)

int main(void) {
    const uint32_t widths[3] = {1, 2, 4};
    for (int k = 0; k < 300 && !fails; k++) {
        const uint32_t w = widths[k % 3];
        const uint32_t maxs = w == 1 ? 256u : (w == 2 ? 65536u : (1u << 20));
        const uint32_t sigma = 1 + (uint32_t)(next() % (k % 2 ? 40 : maxs));
        const uint64_t n = next() % 3000;
        void *S = malloc(n * w + 1);
        uint32_t *syms = (uint32_t *)malloc((n + 1) * 4);
        const uint32_t skew = 1 + (uint32_t)(next() % 4);
        for (uint64_t j = 0; j < n; j++) {
            uint64_t v = next() % sigma;
            for (uint32_t q = 1; q < skew; q++) v = v * (next() % (sigma)) / sigma;  /* skewed towards 0 */
            syms[j] = (uint32_t)v;
            if (w == 1) ((uint8_t *)S)[j] = (uint8_t)v;
            else if (w == 2) ((uint16_t *)S)[j] = (uint16_t)v;
            else ((uint32_t *)S)[j] = (uint32_t)v;
        }
        const uint32_t l = wto_levels(sigma);
        const uint64_t W = wto_words_per_level(n), K = wto_rank_stride(n);
        uint64_t *B = calloc((size_t)(l ? l : 1) * W, 8), *R = calloc((size_t)(l ? l : 1) * K, 8);
        uint64_t *B2 = calloc((size_t)(l ? l : 1) * W, 8), *R2 = calloc((size_t)(l ? l : 1) * K, 8);
        CHECK(wto_build(S, n, sigma, w, B, R) == 0);
        for (int threads = 1; threads <= 3; threads += 2) {
            CHECK(wtc_build_pwt(S, n, sigma, w, B2, R2, threads) == 0);
            CHECK(memcmp(B, B2, (size_t)l * W * 8) == 0 && memcmp(R, R2, (size_t)l * K * 8) == 0);
            memset(B2, 0xAB, (size_t)(l ? l : 1) * W * 8);
            CHECK(wtc_build_dd(S, n, sigma, w, B2, R2, threads) == 0);
            CHECK(memcmp(B, B2, (size_t)l * W * 8) == 0 && memcmp(R, R2, (size_t)l * K * 8) == 0);
        }
        uint32_t *dec = malloc((n + 1) * 4);
        CHECK(wto_decode(B, n, sigma, dec) == 0);
        for (uint64_t j = 0; j < n; j++) CHECK(dec[j] == syms[j]);
        for (int q = 0; q < 20 && n; q++) {
            const uint64_t i = next() % n;
            uint32_t s;
            uint32_t tb[32];
            uint64_t ti[32], r, p;
            CHECK(wto_access(B, n, sigma, i, &s, tb, ti) == 0 && s == syms[i]);
            CHECK(wto_rank(B, n, sigma, syms[i], i + 1, &r) == 0 && r >= 1);
            CHECK(wto_select(B, n, sigma, syms[i], r, &p) == 0 && p == i);
        }
        /* wavelet matrix */
        uint64_t Z[32];
        CHECK(wto_build_matrix(S, n, sigma, w, B2, R2, Z) == 0);
        for (int q = 0; q < 10 && n; q++) {
            const uint64_t i = next() % n;
            uint32_t s;
            CHECK(wto_matrix_access(B2, Z, n, sigma, i, &s) == 0 && s == syms[i]);
        }
        /* 4-ary tree */
        const uint32_t l4 = wto_levels4(sigma);
        uint64_t *D = calloc((size_t)(l4 ? l4 : 1) * wto_words4(n), 8);
        uint64_t *DR = calloc((size_t)(l4 ? l4 : 1) * K * 4, 8);
        CHECK(wto_build4(S, n, sigma, w, D, DR) == 0);
        for (int q = 0; q < 10 && n; q++) {
            const uint64_t i = next() % n;
            uint32_t s;
            CHECK(wto_access4(D, n, sigma, i, &s) == 0 && s == syms[i]);
        }
        /* Huffman-shaped tree */
        uint64_t *cnt = calloc(sigma, 8);
        for (uint64_t j = 0; j < n; j++) cnt[syms[j]]++;
        uint8_t *len = malloc(sigma);
        uint32_t *code = malloc((size_t)sigma * 4), maxlen = 0;
        CHECK(wto_huffman_lengths(cnt, sigma, len, &maxlen) == 0);
        if (maxlen <= 32) {
            CHECK(wto_huffman_codes(len, sigma, maxlen, code) == 0);
            uint64_t bofs[64], rofs[64], tb = 0, tr = 0;
            for (uint32_t d = 0; d < maxlen; d++) {
                uint64_t nd = 0;
                for (uint32_t c = 0; c < sigma; c++)
                    if (len[c] > d) nd += cnt[c];
                bofs[d] = tb;
                rofs[d] = tr;
                tb += wto_words_per_level(nd);
                tr += wto_rank_stride(nd);
            }
            uint64_t *HB = calloc(tb ? tb : 1, 8), *HR = calloc(tr ? tr : 1, 8);
            CHECK(wto_build_huffman(S, n, sigma, w, len, code, maxlen, bofs, rofs, HB, HR) == 0);
            free(HB);
            free(HR);
        }
        free(cnt); free(len); free(code); free(D); free(DR); free(dec);
        free(B); free(R); free(B2); free(R2); free(S); free(syms);
    }
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("cpu checks: ok\n");
    return 0;
}
