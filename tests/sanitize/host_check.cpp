// Host-side checks of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer: the layout, batch, buffered, multiary and
// Huffman planning code and the argument checks, reached through the C ABI
// entry points that touch no device.  Built and run by
// tests/test_sanitizers.py; exits non-zero on the first failed check (the
// sanitizers abort on their own findings).
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "wtree.h"

static int fails = 0;
#define CHECK(c)                                                 \
    do {                                                         \
        if (!(c)) {                                              \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            fails++;                                             \
        }                                                        \
    } while (0)

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static uint64_t next() {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return rng;
}

int main() {
    const uint32_t widths[3] = {1, 2, 4};
    // single, multiary and buffered footprints over sizes and alphabets
    for (int k = 0; k < 4000; k++) {
        wt_desc d;
        d.width = widths[next() % 3];
        const uint32_t maxs = d.width == 1 ? 256u : (d.width == 2 ? 65536u : (1u << 24));
        d.sigma = 1 + (uint32_t)(next() % maxs);
        d.n = (k % 7 == 0) ? 0 : (next() % (1ull << (next() % 34)));
        uint64_t tb = 0, wb = 0;
        CHECK(wt_footprint(&d, &tb, &wb) == WT_OK);
        CHECK(tb >= 256 && wb >= 256 && wb % 256 == 0);
        CHECK(wt_multiary_footprint(&d, &tb, &wb) == WT_OK);
        const uint64_t buf = 1 + next() % (1ull << 26);
        const int rc = wt_buffered_footprint(&d, buf, &tb, &wb);
        CHECK(rc == WT_OK || (d.n / buf) >= (1ull << 20));
    }
    // invalid descriptors and null arguments
    wt_desc bad = {10, 0, 1};
    uint64_t tb, wb;
    CHECK(wt_footprint(&bad, &tb, &wb) == WT_EINVAL);
    bad = {10, 300, 1};
    CHECK(wt_footprint(&bad, &tb, &wb) == WT_EINVAL);
    bad = {10, 4, 3};
    CHECK(wt_footprint(&bad, &tb, &wb) == WT_EINVAL);
    CHECK(wt_footprint(nullptr, &tb, &wb) == WT_EINVAL);
    CHECK(wt_tree_status(nullptr) == WT_EINVAL);
    wt_free(nullptr);
    CHECK(strlen(wt_strerror(WT_ERANGE)) > 0 && strlen(wt_strerror(12345)) > 0);
    // batch plans: mixed widths, alphabets, lengths (with empty sequences)
    for (int k = 0; k < 200; k++) {
        const uint32_t m = 1 + (uint32_t)(next() % 300);
        std::vector<wt_desc> ds(m);
        for (auto &d : ds) {
            d.width = widths[next() % 3];
            const uint32_t maxs = d.width == 1 ? 256u : (d.width == 2 ? 65536u : (1u << 20));
            d.sigma = 1 + (uint32_t)(next() % maxs);
            d.n = (next() % 5 == 0) ? 0 : next() % (1ull << (8 + next() % 16));
        }
        uint64_t w = 0;
        CHECK(wt_batch_footprint(m, ds.data(), &w) == WT_OK);
    }
    // tuning table: every key, valid and invalid values
    for (uint32_t mode = 0; mode < 3; mode++)
        for (uint32_t w : {1u, 2u, 3u, 4u})
            for (uint32_t l = 0; l <= 25; l += 5)
                for (uint32_t lg = 0; lg <= 41; lg += 7) {
                    uint32_t v = 0;
                    const int rc = wt_tune_get(mode, w, l, lg, &v);
                    if (rc == WT_OK) CHECK(wt_tune_set(mode, w, l, lg, v) == WT_OK);
                    (void)wt_tune_set(mode, w, l, lg, 48);
                }
    // Huffman plans: random counts, ties, one symbol, a Fibonacci histogram
    // (code longer than 24 bits: refused), counts that are not S's
    for (int k = 0; k < 300; k++) {
        wt_desc d;
        d.width = widths[next() % 3];
        const uint32_t maxs = d.width == 1 ? 256u : (d.width == 2 ? 65536u : (1u << 20));
        d.sigma = 1 + (uint32_t)(next() % maxs);
        std::vector<uint64_t> c(d.sigma, 0);
        uint64_t n = 0;
        const uint32_t used = 1 + (uint32_t)(next() % (d.sigma < 5000 ? d.sigma : 5000));
        for (uint32_t q = 0; q < used; q++) {
            const uint64_t x = (k % 3 == 0) ? 7 : 1 + next() % 1000;
            c[next() % d.sigma] += x;
        }
        for (uint64_t x : c) n += x;
        d.n = n;
        CHECK(wt_huffman_footprint(c.data(), &d, &tb, &wb) == WT_OK);
        d.n = n + 1;
        CHECK(wt_huffman_footprint(c.data(), &d, &tb, &wb) == WT_EINVAL);
    }
    {
        std::vector<uint64_t> c(40, 0);
        uint64_t a = 1, b = 1, n = 0;
        for (int q = 0; q < 40; q++) {
            c[q] = a;
            n += a;
            const uint64_t t = a + b;
            a = b;
            b = t;
        }
        wt_desc d = {n, 40, 1};
        CHECK(wt_huffman_footprint(c.data(), &d, &tb, &wb) == WT_EINVAL);
    }
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("host checks: ok\n");
    return 0;
}
