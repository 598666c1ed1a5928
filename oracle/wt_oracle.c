/*
 * Sequential CPU oracle for pointerless (one-bitmap-per-level) wavelet-tree
 * construction.  TEST INFRASTRUCTURE ONLY: it is used by the tests, by the
 * smoke check and by the benchmark's CPU-baseline leg, never by the library's
 * product path.  It shares no code, header or table with the GPU library.
 *
 * What it follows (Fuentes-Sepulveda, Elejalde, Ferres, Seco, "Parallel
 * Construction of Wavelet Trees on Multicore Architectures"):
 *
 *  - Section 2.2 (wavelet trees): the balanced binary tree whose node
 *    bitmaps mark with 0 the symbols of the first half and with 1 those of
 *    the second half of the node's alphabet range, each child holding its
 *    half's symbols in their original order; the one-pointer-per-level
 *    representation, which concatenates the node bitmaps of every level from
 *    left to right; access / rank / select, with the navigation simulated by
 *    rank on each level's n-bit bitmap.  The construction below is that
 *    recursive definition carried out level by level (every node split into
 *    its two children in place).
 *  - Section 2.3 (problem statement): S of n symbols over an alphabet of
 *    sigma symbols in, the levels of the tree out.
 *  - Section 3, Proposition 1: the node of symbol s at level i is s >> (l-i),
 *    with l = ceil(lg sigma); the halves of a node's range are therefore
 *    taken by bit prefix, and the mark of level i is bit l-1-i.
 *
 * Readings taken where the paper is loose (each is listed in the design
 * notes): symbols are 0-based in [0, sigma); non-power-of-two alphabets split
 * by bit prefix over l bits (so "first half" of a node's range is the part
 * whose next bit is 0); positions are 0-based; rank(c, i) counts [0, i);
 * select(c, j) takes a 1-based j and returns a 0-based position.
 *
 * Conventions that the paper leaves open and that the library implements
 * independently (parity of these two is unpinned by the paper):
 *  - bitmap words are 64-bit, position p lives in word p/64 at bit p%64
 *    (least significant bit first); each level owns W = round_up(ceil(n/64),
 *    8) words, and every bit at a position >= n is zero;
 *  - the rank directory of a level holds K = ceil(n/512) + 1 absolute
 *    counts R[k] = number of ones in positions [0, min(512k, n)), stored as
 *    64-bit integers in a slot of round_up(K, 8) entries whose padding
 *    entries are zero.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define WTO_OK 0
#define WTO_EINVAL 1
#define WTO_ERANGE 2
#define WTO_ENOMEM 3
#define WTO_ENOTFOUND 4

static uint64_t round_up(uint64_t x, uint64_t m) { return (x + m - 1) / m * m; }

/* Number of levels: the smallest l with 2^l >= sigma (integer loop, no log2). */
uint32_t wto_levels(uint32_t sigma)
{
    uint32_t l = 0;
    while ((1ull << l) < (uint64_t)sigma) l++;
    return l;
}

uint64_t wto_words_per_level(uint64_t n) { return round_up((n + 63) / 64, 8); }
uint64_t wto_rank_entries(uint64_t n) { return (n + 511) / 512 + 1; }
uint64_t wto_rank_stride(uint64_t n) { return round_up(wto_rank_entries(n), 8); }

static uint64_t sym_at(const void *S, uint32_t width, uint64_t j)
{
    if (width == 1) return ((const uint8_t *)S)[j];
    if (width == 2) return ((const uint16_t *)S)[j];
    return ((const uint32_t *)S)[j];
}

static int get_bit(const uint64_t *B, uint64_t p) { return (int)((B[p >> 6] >> (p & 63)) & 1u); }

/* Rank directory of one level: ones before every multiple of 512, then the
 * total, then zero padding up to the slot size. */
static void rank_directory(const uint64_t *Bi, uint64_t n, uint64_t *Ri)
{
    uint64_t K = wto_rank_entries(n), KS = wto_rank_stride(n);
    memset(Ri, 0, KS * sizeof(uint64_t));
    uint64_t ones = 0;
    for (uint64_t p = 0; p < n; p++) {
        if ((p & 511) == 0) Ri[p >> 9] = ones;
        ones += (uint64_t)get_bit(Bi, p);
    }
    Ri[K - 1] = ones;
}

/*
 * Build every level bitmap (and, when R != NULL, every rank directory).
 * B holds l * wto_words_per_level(n) words, R holds l * wto_rank_stride(n)
 * entries.  Returns WTO_ERANGE if some symbol is >= sigma.
 *
 * Straight from the recursive definition of Section 2.2: the root node holds
 * all of S; a node's bitmap marks each of its symbols with 0 (lower half of
 * the node's alphabet range) or 1 (upper half); its left child holds, in
 * their original order, the symbols marked 0 and its right child those
 * marked 1.  The halves are taken by bit prefix (the node of level i
 * covering the symbols whose top i bits are v, Proposition 1), so the mark
 * at level i is bit l-1-i.  The pointerless tree concatenates, level by
 * level, the bitmaps of the nodes from left to right.  Here A holds that
 * concatenation of the level's node sequences and len[v] the length of node
 * v, so the level's bitmap is simply the mark of A[p] at position p, and the
 * next level's A is every node split, in place of its parent, into its marked
 * 0 and marked 1 symbols (each in order).
 */
int wto_build(const void *S, uint64_t n, uint32_t sigma, uint32_t width,
              uint64_t *B, uint64_t *R)
{
    if (sigma == 0 || (width != 1 && width != 2 && width != 4)) return WTO_EINVAL;
    if (width < 4 && (uint64_t)sigma > (1ull << (8 * width))) return WTO_EINVAL;
    for (uint64_t j = 0; j < n; j++)
        if (sym_at(S, width, j) >= sigma) return WTO_ERANGE;

    uint32_t l = wto_levels(sigma);
    uint64_t W = wto_words_per_level(n);
    uint64_t KS = wto_rank_stride(n);
    uint64_t maxnodes = 1ull << l;        /* nodes of the level below the last */
    uint32_t *A = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *Anext = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint64_t *len = (uint64_t *)malloc(maxnodes * sizeof(uint64_t));
    uint64_t *lennext = (uint64_t *)malloc(maxnodes * sizeof(uint64_t));
    if (!A || !Anext || !len || !lennext) {
        free(A); free(Anext); free(len); free(lennext);
        return WTO_ENOMEM;
    }
    for (uint64_t j = 0; j < n; j++) A[j] = (uint32_t)sym_at(S, width, j);
    len[0] = n;                           /* level 0: the root holds S */

    for (uint32_t i = 0; i < l; i++) {
        uint64_t nodes = 1ull << i;
        uint32_t mark = l - 1 - i;        /* level i marks with bit l-1-i */
        uint64_t *Bi = B + (uint64_t)i * W;
        memset(Bi, 0, W * sizeof(uint64_t));
        uint64_t p = 0;                   /* first position of node v */
        for (uint64_t v = 0; v < nodes; v++) {
            uint64_t end = p + len[v];
            uint64_t zeros = 0;
            for (uint64_t k = p; k < end; k++) {
                if ((A[k] >> mark) & 1u) Bi[k >> 6] |= 1ull << (k & 63);
                else zeros++;
            }
            /* children in place of the parent: the 0-marked symbols in
             * order, then the 1-marked ones in order */
            uint64_t zp = p, op = p + zeros;
            for (uint64_t k = p; k < end; k++) {
                if ((A[k] >> mark) & 1u) Anext[op++] = A[k];
                else Anext[zp++] = A[k];
            }
            lennext[2 * v] = zeros;
            lennext[2 * v + 1] = len[v] - zeros;
            p = end;
        }
        if (R) rank_directory(Bi, n, R + (uint64_t)i * KS);
        uint32_t *ta = A; A = Anext; Anext = ta;
        uint64_t *tl = len; len = lennext; lennext = tl;
    }
    free(A);
    free(Anext);
    free(len);
    free(lennext);
    return WTO_OK;
}

/* ------------------------------------------------------------ queries ---- */
/*
 * Queries walk the levels as Section 2.2 describes for the one-pointer-per-
 * level representation: the current node is a range [b, e) of the level's
 * bitmap; its left child occupies, at the next level, the first
 * zeros(b, e) positions of the same range and its right child the rest.
 * rank on a bitmap is counted plainly, bit by bit.
 */
static uint64_t ones_in(const uint64_t *Bi, uint64_t a, uint64_t b)
{
    uint64_t c = 0;
    for (uint64_t p = a; p < b; p++) c += (uint64_t)get_bit(Bi, p);
    return c;
}

/*
 * access(S, i): returns the symbol; trace_bits[k] receives the bit read at
 * level k and trace_idx[k] the position inside the node at level k+1 that the
 * walk moves to (the paper's "i = rank_b(B, i) - 1" values).
 */
int wto_access(const uint64_t *B, uint64_t n, uint32_t sigma, uint64_t i,
               uint32_t *sym, uint32_t *trace_bits, uint64_t *trace_idx)
{
    if (i >= n) return WTO_EINVAL;
    uint32_t l = wto_levels(sigma);
    uint64_t W = wto_words_per_level(n);
    uint64_t b = 0, e = n, p = i;      /* node range and absolute position */
    uint32_t s = 0;
    for (uint32_t k = 0; k < l; k++) {
        const uint64_t *Bk = B + (uint64_t)k * W;
        uint64_t zeros = (e - b) - ones_in(Bk, b, e);
        int bit = get_bit(Bk, p);
        uint64_t before_ones = ones_in(Bk, b, p);
        uint64_t before = bit ? before_ones : (p - b) - before_ones;
        if (bit) { b = b + zeros; }
        else     { e = b + zeros; }
        p = b + before;
        s = (s << 1) | (uint32_t)bit;
        if (trace_bits) trace_bits[k] = (uint32_t)bit;
        if (trace_idx) trace_idx[k] = before;
    }
    *sym = s;
    return WTO_OK;
}

/* rank(c, i): occurrences of c in S[0, i), i in [0, n]. */
int wto_rank(const uint64_t *B, uint64_t n, uint32_t sigma, uint32_t c, uint64_t i,
             uint64_t *out)
{
    if (c >= sigma || i > n) return WTO_EINVAL;
    uint32_t l = wto_levels(sigma);
    uint64_t W = wto_words_per_level(n);
    uint64_t b = 0, e = n, cnt = i;    /* cnt: node symbols that precede i */
    for (uint32_t k = 0; k < l; k++) {
        const uint64_t *Bk = B + (uint64_t)k * W;
        uint64_t zeros = (e - b) - ones_in(Bk, b, e);
        uint64_t ones_before = ones_in(Bk, b, b + cnt);
        if ((c >> (l - 1 - k)) & 1u) { cnt = ones_before; b = b + zeros; }
        else                         { cnt = cnt - ones_before; e = b + zeros; }
    }
    *out = cnt;
    return WTO_OK;
}

/* position of the m-th (1-based) bit equal to `bit` inside [b, e) */
static int select_in(const uint64_t *Bk, uint64_t b, uint64_t e, int bit, uint64_t m,
                     uint64_t *pos)
{
    uint64_t seen = 0;
    for (uint64_t p = b; p < e; p++) {
        if (get_bit(Bk, p) == bit && ++seen == m) { *pos = p; return WTO_OK; }
    }
    return WTO_ENOTFOUND;
}

/* select(c, j): 0-based position of the j-th (1-based) occurrence of c. */
int wto_select(const uint64_t *B, uint64_t n, uint32_t sigma, uint32_t c, uint64_t j,
               uint64_t *out)
{
    if (c >= sigma) return WTO_EINVAL;
    uint32_t l = wto_levels(sigma);
    uint64_t W = wto_words_per_level(n);
    uint64_t bs[32], es[32];
    uint64_t b = 0, e = n;
    for (uint32_t k = 0; k < l; k++) {       /* top-down: node ranges of c */
        const uint64_t *Bk = B + (uint64_t)k * W;
        bs[k] = b; es[k] = e;
        uint64_t zeros = (e - b) - ones_in(Bk, b, e);
        if ((c >> (l - 1 - k)) & 1u) b = b + zeros; else e = b + zeros;
    }
    if (j == 0 || j > e - b) return WTO_ENOTFOUND;
    uint64_t idx = j - 1;                    /* index inside the leaf */
    for (uint32_t kk = l; kk-- > 0;) {       /* bottom-up: back to the parent */
        const uint64_t *Bk = B + (uint64_t)kk * W;
        int bit = (int)((c >> (l - 1 - kk)) & 1u);
        uint64_t pos;
        if (select_in(Bk, bs[kk], es[kk], bit, idx + 1, &pos) != WTO_OK) return WTO_ENOTFOUND;
        idx = pos - bs[kk];
    }
    *out = idx;
    return WTO_OK;
}

/*
 * Forward decode: recover S from the bitmaps alone.  Node boundaries of each
 * level are derived top-down from the zeros of the parent node; then each
 * input position j is followed down the tree, taking at every level the next
 * unread slot of its node (stability makes the j-th symbol of a node sit at
 * the node start plus the number of earlier symbols of that node).
 */
int wto_decode(const uint64_t *B, uint64_t n, uint32_t sigma, uint32_t *out)
{
    uint32_t l = wto_levels(sigma);
    uint64_t W = wto_words_per_level(n);
    if (l == 0) { for (uint64_t j = 0; j < n; j++) out[j] = 0; return WTO_OK; }
    /* start[k] has 2^k + 1 entries; cnt[k] has 2^k entries */
    uint64_t total = (2ull << l);
    uint64_t *start = (uint64_t *)calloc(total + l + 1, sizeof(uint64_t));
    uint64_t *cnt = (uint64_t *)calloc(total, sizeof(uint64_t));
    if (!start || !cnt) { free(start); free(cnt); return WTO_ENOMEM; }
    uint64_t off[33];
    uint64_t o = 0;
    for (uint32_t k = 0; k <= l; k++) { off[k] = o; o += (1ull << k) + 1; }
    start[off[0]] = 0; start[off[0] + 1] = n;
    for (uint32_t k = 0; k < l; k++) {
        const uint64_t *Bk = B + (uint64_t)k * W;
        uint64_t nodes = 1ull << k;
        for (uint64_t v = 0; v < nodes; v++) {
            uint64_t b = start[off[k] + v], e = start[off[k] + v + 1];
            uint64_t zeros = (e - b) - ones_in(Bk, b, e);
            start[off[k + 1] + 2 * v] = b;
            start[off[k + 1] + 2 * v + 1] = b + zeros;
        }
        start[off[k + 1] + 2 * nodes] = n;
    }
    uint64_t coff = 0, cof[33];
    for (uint32_t k = 0; k < l; k++) { cof[k] = coff; coff += 1ull << k; }
    for (uint64_t j = 0; j < n; j++) {
        uint64_t v = 0;
        for (uint32_t k = 0; k < l; k++) {
            uint64_t pos = start[off[k] + v] + cnt[cof[k] + v]++;
            v = 2 * v + (uint64_t)get_bit(B + (uint64_t)k * W, pos);
        }
        out[j] = (uint32_t)v;
    }
    free(start);
    free(cnt);
    return WTO_OK;
}

/* ---------------------------------------------------- wavelet matrix ---- */
/*
 * The wavelet matrix, one of the variants the paper names as future work
 * (Section 5): the paper gives no construction for it, so this follows its
 * standard definition (Claude, Navarro and Ordonez, "The wavelet matrix",
 * Information Systems 2015).  A_0 = S; level i's bitmap is bit (l-1-i) of
 * A_i, position by position; A_{i+1} is A_i stably partitioned by that bit
 * over the whole level (all zeros first, in order, then all ones); z_i is
 * the number of zeros of level i.  Same word and rank-directory conventions
 * as the tree above.
 */
int wto_build_matrix(const void *S, uint64_t n, uint32_t sigma, uint32_t width,
                     uint64_t *B, uint64_t *R, uint64_t *Z)
{
    if (sigma == 0 || (width != 1 && width != 2 && width != 4)) return WTO_EINVAL;
    if (width < 4 && (uint64_t)sigma > (1ull << (8 * width))) return WTO_EINVAL;
    for (uint64_t j = 0; j < n; j++)
        if (sym_at(S, width, j) >= sigma) return WTO_ERANGE;

    uint32_t l = wto_levels(sigma);
    uint64_t W = wto_words_per_level(n);
    uint64_t K = wto_rank_entries(n), KS = wto_rank_stride(n);
    uint64_t *A = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    uint64_t *Anext = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    if (!A || !Anext) { free(A); free(Anext); return WTO_ENOMEM; }
    for (uint64_t j = 0; j < n; j++) A[j] = sym_at(S, width, j);

    for (uint32_t i = 0; i < l; i++) {
        uint32_t sh = l - 1 - i;
        uint64_t *Bi = B + (uint64_t)i * W;
        memset(Bi, 0, W * sizeof(uint64_t));
        uint64_t zeros = 0;
        for (uint64_t p = 0; p < n; p++) {
            uint64_t bit = (A[p] >> sh) & 1u;
            if (bit) Bi[p >> 6] |= 1ull << (p & 63);
            else zeros++;
        }
        if (Z) Z[i] = zeros;
        /* stable partition: zeros in order, then ones in order */
        uint64_t zp = 0, op = zeros;
        for (uint64_t p = 0; p < n; p++) {
            if ((A[p] >> sh) & 1u) Anext[op++] = A[p];
            else Anext[zp++] = A[p];
        }
        uint64_t *t = A; A = Anext; Anext = t;
        if (R) {
            uint64_t *Ri = R + (uint64_t)i * KS;
            memset(Ri, 0, KS * sizeof(uint64_t));
            uint64_t ones = 0;
            for (uint64_t p = 0; p < n; p++) {
                if ((p & 511) == 0) Ri[p >> 9] = ones;
                ones += (uint64_t)get_bit(Bi, p);
            }
            Ri[K - 1] = ones;
        }
    }
    free(A);
    free(Anext);
    return WTO_OK;
}

/*
 * Matrix queries (same definition): reading bit b at position p of level
 * i, the walk continues at rank0(B_i, p) when b = 0 and at
 * z_i + rank1(B_i, p) when b = 1.  Ranks are counted bit by bit.
 */
int wto_matrix_access(const uint64_t *B, const uint64_t *Z, uint64_t n, uint32_t sigma, uint64_t i,
                      uint32_t *sym)
{
    if (i >= n) return WTO_EINVAL;
    uint32_t l = wto_levels(sigma);
    uint64_t W = wto_words_per_level(n);
    uint64_t p = i;
    uint32_t s = 0;
    for (uint32_t k = 0; k < l; k++) {
        const uint64_t *Bk = B + (uint64_t)k * W;
        int bit = get_bit(Bk, p);
        uint64_t ones = ones_in(Bk, 0, p);
        p = bit ? Z[k] + ones : p - ones;
        s = (s << 1) | (uint32_t)bit;
    }
    *sym = s;
    return WTO_OK;
}

/* rank(c, i): the range [b, e) of the symbols before i narrows level by level. */
int wto_matrix_rank(const uint64_t *B, const uint64_t *Z, uint64_t n, uint32_t sigma, uint32_t c,
                    uint64_t i, uint64_t *out)
{
    if (c >= sigma || i > n) return WTO_EINVAL;
    uint32_t l = wto_levels(sigma);
    uint64_t W = wto_words_per_level(n);
    uint64_t b = 0, e = i;
    for (uint32_t k = 0; k < l; k++) {
        const uint64_t *Bk = B + (uint64_t)k * W;
        uint64_t ob = ones_in(Bk, 0, b), oe = ones_in(Bk, 0, e);
        if ((c >> (l - 1 - k)) & 1u) { b = Z[k] + ob; e = Z[k] + oe; }
        else                         { b = b - ob; e = e - oe; }
    }
    *out = e - b;
    return WTO_OK;
}

/* select(c, j): the j-th (1-based) c; WTO_ENOTFOUND when there is none. */
int wto_matrix_select(const uint64_t *B, const uint64_t *Z, uint64_t n, uint32_t sigma, uint32_t c,
                      uint64_t j, uint64_t *out)
{
    if (c >= sigma) return WTO_EINVAL;
    uint64_t occ;
    int rc = wto_matrix_rank(B, Z, n, sigma, c, n, &occ);
    if (rc != WTO_OK) return rc;
    if (j == 0 || j > occ) return WTO_ENOTFOUND;
    uint32_t l = wto_levels(sigma);
    uint64_t W = wto_words_per_level(n);
    /* start of c's block at the bottom: follow position 0 down */
    uint64_t b = 0;
    for (uint32_t k = 0; k < l; k++) {
        const uint64_t *Bk = B + (uint64_t)k * W;
        uint64_t ob = ones_in(Bk, 0, b);
        b = ((c >> (l - 1 - k)) & 1u) ? Z[k] + ob : b - ob;
    }
    uint64_t p = b + j - 1;
    /* back up: the position holding the (t+1)-th zero / one of level k */
    for (uint32_t k = l; k-- > 0;) {
        const uint64_t *Bk = B + (uint64_t)k * W;
        int want = (int)((c >> (l - 1 - k)) & 1u);
        uint64_t t = want ? p - Z[k] : p;   /* rank of the wanted bit */
        uint64_t seen = 0, q = 0;
        for (q = 0; q < n; q++) {
            if (get_bit(Bk, q) == want) {
                if (seen == t) break;
                seen++;
            }
        }
        p = q;
    }
    *out = p;
    return WTO_OK;
}

/* ------------------------------------------------------- 4-ary tree ---- */
/*
 * Multiary wavelet tree of fan-out 4 (Section 5 names multiary trees, where
 * a node has more than two children, as future work; this is the plain
 * generalisation of the one-pointer-per-level representation).  With
 * l = ceil(lg sigma), symbols are read as codes of L4 = ceil(l / 2) base-4
 * digits (one zero bit on top when l is odd).  Level i lists, node after
 * node in order, digit i of every symbol (bits 2(L4-1-i) + 1 .. 2(L4-1-i));
 * the node of s at level i is s >> 2(L4-i), and the symbols of a node keep
 * their input order.  The construction is the recursive definition of
 * Section 2.2 with four children per node, carried out level by level: each
 * node's digit sequence is its level's contribution, and its symbols go, in
 * order, to the child of their digit.
 *
 * Conventions (as for the binary tree, unpinned by the paper): digit p of a
 * level sits in 64-bit word p / 32 at bits 2 (p % 32) and 2 (p % 32) + 1;
 * each level owns round_up(ceil(n / 32), 8) words and every digit at a
 * position >= n is 0.  The directory of a level holds K = ceil(n/512) + 1
 * entries of four counts, entry k giving the number of digits 0, 1, 2, 3 in
 * positions [0, min(512k, n)), in a slot of round_up(K, 8) entries whose
 * padding entries are zero.
 */
uint32_t wto_levels4(uint32_t sigma) { return (wto_levels(sigma) + 1) / 2; }
uint64_t wto_words4(uint64_t n) { return round_up((n + 31) / 32, 8); }

static uint32_t get_digit(const uint64_t *D, uint64_t p) { return (uint32_t)((D[p >> 5] >> (2 * (p & 31))) & 3u); }

int wto_build4(const void *S, uint64_t n, uint32_t sigma, uint32_t width, uint64_t *D, uint64_t *R)
{
    if (sigma == 0 || (width != 1 && width != 2 && width != 4)) return WTO_EINVAL;
    if (width < 4 && (uint64_t)sigma > (1ull << (8 * width))) return WTO_EINVAL;
    for (uint64_t j = 0; j < n; j++)
        if (sym_at(S, width, j) >= sigma) return WTO_ERANGE;

    uint32_t L4 = wto_levels4(sigma);
    uint64_t W = wto_words4(n);
    uint64_t K = wto_rank_entries(n), KS = wto_rank_stride(n);
    uint64_t maxnodes = 1ull << (2 * L4);
    /* As for the binary tree: A is the level's node sequences concatenated,
     * len[v] the length of node v; each node hands its symbols, in order, to
     * its four children by digit. */
    uint32_t *A = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *Anext = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint64_t *len = (uint64_t *)malloc(maxnodes * sizeof(uint64_t));
    uint64_t *lennext = (uint64_t *)malloc(maxnodes * sizeof(uint64_t));
    if (!A || !Anext || !len || !lennext) {
        free(A); free(Anext); free(len); free(lennext);
        return WTO_ENOMEM;
    }
    for (uint64_t j = 0; j < n; j++) A[j] = (uint32_t)sym_at(S, width, j);
    len[0] = n;
    for (uint32_t i = 0; i < L4; i++) {
        uint64_t nodes = 1ull << (2 * i);
        uint32_t dsh = 2 * (L4 - 1 - i);   /* digit i of a padded code */
        uint64_t *Di = D + (uint64_t)i * W;
        memset(Di, 0, W * sizeof(uint64_t));
        uint64_t p = 0;
        for (uint64_t v = 0; v < nodes; v++) {
            uint64_t end = p + len[v];
            uint64_t cnt[4] = {0, 0, 0, 0};
            for (uint64_t k = p; k < end; k++) {
                uint64_t d = (A[k] >> dsh) & 3u;
                Di[k >> 5] |= d << (2 * (k & 31));
                cnt[d]++;
            }
            uint64_t at[4];
            at[0] = p;
            for (int d = 1; d < 4; d++) at[d] = at[d - 1] + cnt[d - 1];
            for (uint64_t k = p; k < end; k++) Anext[at[(A[k] >> dsh) & 3u]++] = A[k];
            for (int d = 0; d < 4; d++) lennext[4 * v + (uint64_t)d] = cnt[d];
            p = end;
        }
        if (R) {
            uint64_t *Ri = R + (uint64_t)i * KS * 4;
            memset(Ri, 0, KS * 4 * sizeof(uint64_t));
            uint64_t c4[4] = {0, 0, 0, 0};
            for (uint64_t q = 0; q < n; q++) {
                if ((q & 511) == 0)
                    for (int d = 0; d < 4; d++) Ri[(q >> 9) * 4 + d] = c4[d];
                c4[get_digit(Di, q)]++;
            }
            for (int d = 0; d < 4; d++) Ri[(K - 1) * 4 + d] = c4[d];
        }
        uint32_t *ta = A; A = Anext; Anext = ta;
        uint64_t *tl = len; len = lennext; lennext = tl;
    }
    free(A);
    free(Anext);
    free(len);
    free(lennext);
    return WTO_OK;
}

/* digits equal to d in positions [a, b) of one level, counted one by one */
static uint64_t digits_in(const uint64_t *Di, uint64_t a, uint64_t b, uint32_t d)
{
    uint64_t c = 0;
    for (uint64_t p = a; p < b; p++) c += get_digit(Di, p) == d;
    return c;
}

/*
 * Queries walk the levels: the current node is a range [b, e) of the level;
 * its child of digit d occupies, at the next level, the part of [b, e)
 * after the digits smaller than d of [b, e), as long as the digits equal to
 * d of [b, e).
 */
int wto_access4(const uint64_t *D, uint64_t n, uint32_t sigma, uint64_t i, uint32_t *sym)
{
    if (i >= n) return WTO_EINVAL;
    uint32_t L4 = wto_levels4(sigma);
    uint64_t W = wto_words4(n);
    uint64_t b = 0, e = n, p = i;
    uint32_t s = 0;
    for (uint32_t k = 0; k < L4; k++) {
        const uint64_t *Dk = D + (uint64_t)k * W;
        uint32_t d = get_digit(Dk, p);
        uint64_t below = 0;
        for (uint32_t x = 0; x < d; x++) below += digits_in(Dk, b, e, x);
        uint64_t nb = b + below;
        uint64_t ne = nb + digits_in(Dk, b, e, d);
        p = nb + digits_in(Dk, b, p, d);
        b = nb;
        e = ne;
        s = (s << 2) | d;
    }
    *sym = s;
    return WTO_OK;
}

int wto_rank4(const uint64_t *D, uint64_t n, uint32_t sigma, uint32_t c, uint64_t i, uint64_t *out)
{
    if (c >= sigma || i > n) return WTO_EINVAL;
    uint32_t L4 = wto_levels4(sigma);
    uint64_t W = wto_words4(n);
    uint64_t b = 0, e = n, p = i;
    for (uint32_t k = 0; k < L4; k++) {
        const uint64_t *Dk = D + (uint64_t)k * W;
        uint32_t d = (c >> (2 * (L4 - 1 - k))) & 3u;
        uint64_t below = 0;
        for (uint32_t x = 0; x < d; x++) below += digits_in(Dk, b, e, x);
        uint64_t nb = b + below;
        uint64_t ne = nb + digits_in(Dk, b, e, d);
        p = nb + digits_in(Dk, b, p, d);
        b = nb;
        e = ne;
    }
    *out = p - b;
    return WTO_OK;
}

int wto_select4(const uint64_t *D, uint64_t n, uint32_t sigma, uint32_t c, uint64_t j, uint64_t *out)
{
    if (c >= sigma) return WTO_EINVAL;
    uint32_t L4 = wto_levels4(sigma);
    uint64_t W = wto_words4(n);
    uint64_t bs[32];
    uint64_t b = 0, e = n;
    for (uint32_t k = 0; k < L4; k++) {
        const uint64_t *Dk = D + (uint64_t)k * W;
        uint32_t d = (c >> (2 * (L4 - 1 - k))) & 3u;
        bs[k] = b;
        uint64_t below = 0;
        for (uint32_t x = 0; x < d; x++) below += digits_in(Dk, b, e, x);
        uint64_t nb = b + below;
        e = nb + digits_in(Dk, b, e, d);
        b = nb;
    }
    if (j == 0 || j > e - b) return WTO_ENOTFOUND;
    uint64_t p = b + j - 1;   /* position inside the leaf range */
    uint64_t child = b;
    for (uint32_t k = L4; k-- > 0;) {
        const uint64_t *Dk = D + (uint64_t)k * W;
        uint32_t d = (c >> (2 * (L4 - 1 - k))) & 3u;
        uint64_t t = p - child;   /* the wanted digit's rank inside the node */
        uint64_t seen = 0, q;
        for (q = bs[k]; q < n; q++) {
            if (get_digit(Dk, q) == d) {
                if (seen == t) break;
                seen++;
            }
        }
        p = q;
        /* the node of level k starts at bs[k]; its parent node starts at bs[k-1] */
        child = bs[k];
    }
    *out = p;
    return WTO_OK;
}

/* ---------------------------------------------- Huffman-shaped tree ---- */
/*
 * Huffman-shaped wavelet tree, one of the compressed wavelet trees that
 * Section 5 names as future work (the paper gives no definition; this takes
 * the standard one): the tree's shape is the code tree of a Huffman code for
 * the symbol frequencies of S.  A symbol that occurs is a leaf at the depth
 * of its code length, reached by following its code bits (0 = left); every
 * internal node holds a bitmap listing, for the symbols of its subtree in
 * their input order, the next bit of their codes.  The pointerless layout
 * keeps one bitmap per depth d: the concatenation, from left to right, of
 * the bitmaps of the internal nodes at depth d.
 *
 * A Huffman code is not unique, so the construction fixes every choice
 * (readings listed in the design notes):
 *  - lengths: Huffman's merging of the two lightest items, done with two
 *    first-in first-out queues -- the symbols that occur, ordered by (count,
 *    symbol), and the merged items in the order they are made; the lighter
 *    front is taken, the symbol queue on equal weights; the code length of a
 *    symbol is the depth of its leaf.  One symbol alone has length 0 (a tree
 *    with no levels), as has every symbol when n = 0;
 *  - codes: canonical, from the lengths: symbols ordered by (length,
 *    symbol); the first gets 0, each next one the previous code plus one,
 *    shifted left by the increase in length.
 * Position p of depth d sits in word p/64 at bit p%64 of that depth's
 * round_up(ceil(n_d/64), 8) words (n_d = symbols whose code is longer than d),
 * every bit past n_d zero; its directory holds ceil(n_d/512) + 1 counts in a
 * slot of round_up(that, 8) entries, as for the balanced tree.
 */

static int cmp_count_sym(const void *a, const void *b, const uint64_t *counts)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    if (counts[x] != counts[y]) return counts[x] < counts[y] ? -1 : 1;
    return x < y ? -1 : (x > y);
}

/* merge sort of symbol indices by (count, symbol) */
static void sort_by_count(uint32_t *v, uint32_t *tmp, uint64_t k, const uint64_t *counts)
{
    if (k < 2) return;
    uint64_t h = k / 2;
    sort_by_count(v, tmp, h, counts);
    sort_by_count(v + h, tmp, k - h, counts);
    uint64_t a = 0, b = h, o = 0;
    while (a < h && b < k) tmp[o++] = (cmp_count_sym(&v[b], &v[a], counts) < 0) ? v[b++] : v[a++];
    while (a < h) tmp[o++] = v[a++];
    while (b < k) tmp[o++] = v[b++];
    memcpy(v, tmp, k * sizeof(uint32_t));
}

/* Code lengths of the sigma symbols (0 for a symbol that does not occur). */
int wto_huffman_lengths(const uint64_t *counts, uint32_t sigma, uint8_t *len, uint32_t *maxlen)
{
    if (sigma == 0) return WTO_EINVAL;
    memset(len, 0, sigma);
    *maxlen = 0;
    uint64_t k = 0;
    for (uint32_t c = 0; c < sigma; c++) k += counts[c] > 0;
    if (k < 2) return WTO_OK;
    uint32_t *leaf = (uint32_t *)malloc(k * sizeof(uint32_t));
    uint32_t *tmp = (uint32_t *)malloc(k * sizeof(uint32_t));
    uint64_t *iw = (uint64_t *)malloc(k * sizeof(uint64_t));      /* merged items' weights */
    uint64_t *parent = (uint64_t *)malloc((2 * k) * sizeof(uint64_t)); /* leaves 0..k-1, merged k.. */
    uint32_t *depth = (uint32_t *)malloc((2 * k) * sizeof(uint32_t));
    if (!leaf || !tmp || !iw || !parent || !depth) {
        free(leaf); free(tmp); free(iw); free(parent); free(depth);
        return WTO_ENOMEM;
    }
    uint64_t q = 0;
    for (uint32_t c = 0; c < sigma; c++)
        if (counts[c] > 0) leaf[q++] = c;
    sort_by_count(leaf, tmp, k, counts);
    uint64_t lf = 0, mf = 0, made = 0;  /* fronts of the two queues, merged items made */
    while (made < k - 1) {
        uint64_t pick[2];
        uint64_t w = 0;
        for (int t = 0; t < 2; t++) {
            int take_leaf = lf < k && (mf >= made || counts[leaf[lf]] <= iw[mf]);
            if (take_leaf) { pick[t] = lf; w += counts[leaf[lf]]; lf++; }
            else           { pick[t] = k + mf; w += iw[mf]; mf++; }
        }
        iw[made] = w;
        parent[pick[0]] = k + made;
        parent[pick[1]] = k + made;
        made++;
    }
    /* the last merged item is the root; parents are made after children */
    depth[k + made - 1] = 0;
    for (uint64_t m = made - 1; m-- > 0;) depth[k + m] = depth[parent[k + m]] + 1;
    for (uint64_t i = 0; i < k; i++) {
        uint32_t d = depth[parent[i]] + 1;
        if (d > 255) d = 255;
        len[leaf[i]] = (uint8_t)d;
        if (d > *maxlen) *maxlen = d;
    }
    free(leaf); free(tmp); free(iw); free(parent); free(depth);
    return WTO_OK;
}

/* Canonical codes from the lengths (code[c] right-aligned in len[c] bits). */
int wto_huffman_codes(const uint8_t *len, uint32_t sigma, uint32_t maxlen, uint32_t *code)
{
    if (maxlen > 32) return WTO_EINVAL;
    memset(code, 0, (uint64_t)sigma * sizeof(uint32_t));
    uint64_t c = 0;
    uint32_t prev = 0;
    int first = 1;
    for (uint32_t L = 1; L <= maxlen; L++) {
        for (uint32_t s = 0; s < sigma; s++) {
            if (len[s] != L) continue;
            if (first) { c = 0; first = 0; }
            else c = (c + 1) << (L - prev);
            prev = L;
            code[s] = (uint32_t)c;
        }
    }
    return WTO_OK;
}

/* bit d (from the top, d < len) of symbol s's code */
static uint32_t code_bit(const uint8_t *len, const uint32_t *code, uint32_t s, uint32_t d)
{
    return (code[s] >> (len[s] - 1 - d)) & 1u;
}

/* the first d bits of s's code (d <= len) */
static uint32_t code_prefix(const uint8_t *len, const uint32_t *code, uint32_t s, uint32_t d)
{
    return d == 0 ? 0u : (code[s] >> (len[s] - d));
}

/*
 * Build the maxlen depth bitmaps (and, when R != NULL, their directories).
 * Depth d's words start at B + bofs[d], its directory at R + rofs[d].
 * A holds the symbols of the current depth's internal nodes, node after node
 * from left to right, each node's symbols in input order; a node is a run
 * of equal code prefixes.  Each node's bitmap is the next code bit of its
 * symbols; the next depth splits every node into its 0-child and then its
 * 1-child (each in order), leaving out the symbols whose code ends here
 * (they are leaves).  Returns WTO_ERANGE if a symbol is >= sigma or has no
 * code (length 0 while the tree has levels).
 */
int wto_build_huffman(const void *S, uint64_t n, uint32_t sigma, uint32_t width, const uint8_t *len,
                      const uint32_t *code, uint32_t maxlen, const uint64_t *bofs, const uint64_t *rofs,
                      uint64_t *B, uint64_t *R)
{
    if (sigma == 0 || (width != 1 && width != 2 && width != 4)) return WTO_EINVAL;
    for (uint64_t j = 0; j < n; j++) {
        uint64_t s = sym_at(S, width, j);
        if (s >= sigma || (maxlen > 0 && len[s] == 0)) return WTO_ERANGE;
    }
    if (maxlen == 0) return WTO_OK;
    uint32_t *A = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t *Anext = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    if (!A || !Anext) { free(A); free(Anext); return WTO_ENOMEM; }
    uint64_t cur = n;
    for (uint64_t j = 0; j < n; j++) A[j] = (uint32_t)sym_at(S, width, j);
    for (uint32_t d = 0; d < maxlen; d++) {
        uint64_t *Bd = B + bofs[d];
        uint64_t W = wto_words_per_level(cur);
        memset(Bd, 0, W * sizeof(uint64_t));
        uint64_t nxt = 0;
        uint64_t p = 0;
        while (p < cur) {
            /* the node: the run of symbols sharing A[p]'s first d code bits */
            uint32_t pre = code_prefix(len, code, A[p], d);
            uint64_t e = p;
            while (e < cur && code_prefix(len, code, A[e], d) == pre) e++;
            for (uint64_t k = p; k < e; k++)
                if (code_bit(len, code, A[k], d)) Bd[k >> 6] |= 1ull << (k & 63);
            for (int b = 0; b < 2; b++)
                for (uint64_t k = p; k < e; k++)
                    if (code_bit(len, code, A[k], d) == (uint32_t)b && len[A[k]] > d + 1) Anext[nxt++] = A[k];
            p = e;
        }
        if (R) rank_directory(Bd, cur, R + rofs[d]);
        uint32_t *t = A; A = Anext; Anext = t;
        cur = nxt;
    }
    free(A);
    free(Anext);
    return WTO_OK;
}
