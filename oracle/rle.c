/*
 * Run-length static BWT format: encoder, decoder and rank by decoding,
 * written from the format's definition below. This is the bit-packed
 * static format of Sec. 2.2 (Fig. 2b): blocks that hold run-length coded
 * BWT with Elias-delta run lengths next to the block's marginal counts,
 * plus an index row for access by position.
 *
 * THIS IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg call it. The GPU library never links, loads or
 * calls anything here, and nothing here shares code with the GPU library.
 *
 * The format (the GPU library writes the same bytes from the same text):
 *   Segments  B[0, n) is cut into segments of 2^20 symbols (the last one may
 *             be shorter).
 *   Pieces    each segment is cut into its maximal runs of one symbol; such
 *             a run is a piece (length 1 .. 2^20).
 *   Code      a piece is written as its symbol in 3 bits, then its length L
 *             in the Elias delta code: with N the bit length of L and K the
 *             bit length of N, K - 1 zero bits, N in K bits, then the N - 1
 *             low bits of L. Every field is written most significant bit
 *             first.
 *   Blocks    128 bytes = 16 uint64 words. Words 0-1 are the header, words
 *             2-15 hold 896 stream bits: stream bit t is bit 63 - (t mod 64)
 *             of word 2 + t / 64. Unused bits are 0.
 *             word 0: bits 0-19 the block's first position minus its
 *             segment's first position (the block offset o); bits 20-39 and
 *             40-59 the occurrences of A and of C in the segment before the
 *             block; bits 60-63 the low 4 bits of the block's piece count.
 *             word 1: bits 0-19, 20-39, 40-59 the occurrences of G, T and N
 *             in the segment before the block; bits 60-63 the high 4 bits of
 *             the piece count. Those of $ are o minus the five counts.
 *   Packing   the pieces of a segment go into blocks in order, greedily: a
 *             block takes pieces while their codes fit in its 896 bits, and
 *             the first piece that does not fit starts the next block. Each
 *             segment starts a new block.
 *   Segments' table  nseg + 1 rows of 8 int64: the occurrences of $, A, C,
 *             G, T, N in B before the segment, the index of its first block,
 *             and 0. Row nseg holds the totals and the number of blocks.
 *   Index row with the row shift q (4 .. 20), entry j (0 <= j <= (n-1) >> q)
 *             is the index of the block holding position j << q, counted
 *             from its segment's first block (uint16).
 *   Rank      the occurrences of every symbol in B[0, i): i = n gives the
 *             totals; a segment start gives its table row; otherwise the
 *             table row, plus the header counts of the block the index row
 *             names, plus the pieces decoded from that block's offset up to
 *             i (continuing into the next block when i lies past it).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RLE_SEG_SHIFT 20
#define RLE_SEG ((int64_t)1 << RLE_SEG_SHIFT)
#define RLE_WORDS 16
#define RLE_BITS 896

/* bit length of v >= 1 */
static int orc_bitlen(uint64_t v)
{
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

/* Number of bits of the Elias delta code of L >= 1. */
int orc_delta_len(uint64_t L)
{
    int N = orc_bitlen(L), K = orc_bitlen((uint64_t)N);
    return (K - 1) + K + (N - 1);
}

/* The Elias delta code of L >= 1 as a string of '0'/'1' characters
 * (NUL-terminated), most significant bit first. Returns its length. */
int orc_delta_string(uint64_t L, char *out)
{
    int N = orc_bitlen(L), K = orc_bitlen((uint64_t)N), p = 0, i;
    for (i = 0; i < K - 1; ++i) out[p++] = '0';
    for (i = K - 1; i >= 0; --i) out[p++] = (char)('0' + ((N >> i) & 1));
    for (i = N - 2; i >= 0; --i) out[p++] = (char)('0' + ((L >> i) & 1));
    out[p] = 0;
    return p;
}

typedef struct {
    uint64_t *w; /* the block's 16 words */
    int bit;     /* next stream bit */
} orc_bw;

static void orc_put_bit(orc_bw *b, int v)
{
    if (v) b->w[2 + (b->bit >> 6)] |= 1ull << (63 - (b->bit & 63));
    ++b->bit;
}

static void orc_put_bits(orc_bw *b, uint64_t v, int nbits)
{
    int i;
    for (i = nbits - 1; i >= 0; --i) orc_put_bit(b, (int)((v >> i) & 1));
}

static void orc_put_piece(orc_bw *b, int sym, uint64_t L)
{
    int N = orc_bitlen(L), K = orc_bitlen((uint64_t)N), i;
    orc_put_bits(b, (uint64_t)sym, 3);
    for (i = 0; i < K - 1; ++i) orc_put_bit(b, 0);
    orc_put_bits(b, (uint64_t)N, K);
    orc_put_bits(b, L, N - 1); /* the low N - 1 bits */
}

static void orc_header(uint64_t *w, int64_t off, const int64_t cnt[6], int npieces)
{
    w[0] = (uint64_t)off | ((uint64_t)cnt[1] << 20) | ((uint64_t)cnt[2] << 40) |
           ((uint64_t)(npieces & 15) << 60);
    w[1] = (uint64_t)cnt[3] | ((uint64_t)cnt[4] << 20) | ((uint64_t)cnt[5] << 40) |
           ((uint64_t)(npieces >> 4) << 60);
}

/*
 * Encode B[0, n) (codes 0..5). Pass blocks = NULL to learn the sizes:
 * *nblocks_out gets the number of blocks. With buffers (blocks: nblocks * 16
 * words, seg: (nseg + 1) * 8, row: ((n - 1) >> q) + 1 entries; all zeroed by
 * the caller) the format is written. Returns 0, or -1 on a bad argument.
 */
int orc_rle_encode(const uint8_t *B, int64_t n, int q, uint64_t *blocks, int64_t *seg, uint16_t *row,
                   int64_t *nblocks_out)
{
    int64_t nseg = (n + RLE_SEG - 1) >> RLE_SEG_SHIFT, s, nb = 0;
    int64_t tot[6] = {0, 0, 0, 0, 0, 0};
    int c;
    if (n <= 0 || q < 4 || q > 20) return -1;
    for (s = 0; s < nseg; ++s) {
        int64_t s0 = s << RLE_SEG_SHIFT, s1 = s0 + RLE_SEG < n ? s0 + RLE_SEG : n;
        int64_t first = nb, cnt[6] = {0, 0, 0, 0, 0, 0}, i = s0;
        /* the open block */
        int64_t boff = 0, bcnt[6] = {0, 0, 0, 0, 0, 0};
        int used = 0, np = 0;
        orc_bw bw;
        uint64_t *cur = blocks ? blocks + nb * RLE_WORDS : NULL;
        if (seg) {
            for (c = 0; c < 6; ++c) seg[s * 8 + c] = tot[c];
            seg[s * 8 + 6] = first;
            seg[s * 8 + 7] = 0;
        }
        bw.w = cur;
        bw.bit = 0;
        while (i < s1) {
            int64_t j = i + 1, L;
            int sym = B[i], bits;
            while (j < s1 && B[j] == sym) ++j;
            L = j - i;
            bits = 3 + orc_delta_len((uint64_t)L);
            if (used + bits > RLE_BITS) {
                /* close the block; the piece opens the next one */
                if (cur) orc_header(cur, boff, bcnt, np);
                ++nb;
                cur = blocks ? blocks + nb * RLE_WORDS : NULL;
                bw.w = cur;
                bw.bit = 0;
                used = 0;
                np = 0;
                boff = i - s0;
                memcpy(bcnt, cnt, sizeof(bcnt));
            }
            if (cur) orc_put_piece(&bw, sym, (uint64_t)L);
            used += bits;
            ++np;
            cnt[sym] += L;
            i = j;
        }
        if (cur) orc_header(cur, boff, bcnt, np);
        ++nb;
        /* index row entries of this segment: the block holding j << q */
        if (row && blocks) {
            int64_t j0 = (s0 + ((int64_t)1 << q) - 1) >> q, j, b = first;
            for (j = j0; (j << q) < s1; ++j) {
                int64_t p = (j << q) - s0;
                while (b + 1 < nb && (int64_t)(blocks[(b + 1) * RLE_WORDS] & 0xFFFFF) <= p) ++b;
                row[j] = (uint16_t)(b - first);
            }
        }
        for (c = 0; c < 6; ++c) tot[c] += cnt[c];
    }
    if (seg) {
        for (c = 0; c < 6; ++c) seg[nseg * 8 + c] = tot[c];
        seg[nseg * 8 + 6] = nb;
        seg[nseg * 8 + 7] = 0;
    }
    *nblocks_out = nb;
    return 0;
}

/* ---- decoding ---- */

typedef struct {
    const uint64_t *w;
    int bit;
} orc_br;

static int orc_get_bit(orc_br *r)
{
    int v = (int)((r->w[2 + (r->bit >> 6)] >> (63 - (r->bit & 63))) & 1);
    ++r->bit;
    return v;
}

static uint64_t orc_get_bits(orc_br *r, int nbits)
{
    uint64_t v = 0;
    int i;
    for (i = 0; i < nbits; ++i) v = (v << 1) | (uint64_t)orc_get_bit(r);
    return v;
}

/* One piece; returns -1 on a malformed code. */
static int orc_get_piece(orc_br *r, int *sym, uint64_t *L)
{
    int K = 1, N;
    *sym = (int)orc_get_bits(r, 3);
    while (r->bit < RLE_BITS && orc_get_bit(r) == 0) ++K;
    if (K > 6) return -1;
    N = (int)((1ull << (K - 1)) | orc_get_bits(r, K - 1)); /* the leading 1 was read */
    if (N < 1 || N > 21) return -1;
    *L = (1ull << (N - 1)) | orc_get_bits(r, N - 1);
    return *sym > 5 ? -1 : 0;
}

static void orc_read_header(const uint64_t *w, int64_t *off, int64_t cnt[6], int *np)
{
    *off = (int64_t)(w[0] & 0xFFFFF);
    cnt[1] = (int64_t)((w[0] >> 20) & 0xFFFFF);
    cnt[2] = (int64_t)((w[0] >> 40) & 0xFFFFF);
    cnt[3] = (int64_t)(w[1] & 0xFFFFF);
    cnt[4] = (int64_t)((w[1] >> 20) & 0xFFFFF);
    cnt[5] = (int64_t)((w[1] >> 40) & 0xFFFFF);
    cnt[0] = *off - cnt[1] - cnt[2] - cnt[3] - cnt[4] - cnt[5];
    *np = (int)((w[0] >> 60) | ((w[1] >> 60) << 4));
}

/* The whole BWT back out of its blocks, block by block. Returns 0 or -1. */
int orc_rle_decode(const uint64_t *blocks, const int64_t *seg, int64_t n, uint8_t *B)
{
    int64_t nseg = (n + RLE_SEG - 1) >> RLE_SEG_SHIFT, s;
    for (s = 0; s < nseg; ++s) {
        int64_t s0 = s << RLE_SEG_SHIFT, s1 = s0 + RLE_SEG < n ? s0 + RLE_SEG : n, b;
        int64_t pos = s0;
        for (b = seg[s * 8 + 6]; b < seg[(s + 1) * 8 + 6]; ++b) {
            const uint64_t *w = blocks + b * RLE_WORDS;
            int64_t off, cnt[6];
            int np, t;
            orc_br r;
            orc_read_header(w, &off, cnt, &np);
            if (s0 + off != pos) return -1;
            r.w = w;
            r.bit = 0;
            for (t = 0; t < np; ++t) {
                int sym;
                uint64_t L;
                if (orc_get_piece(&r, &sym, &L) || pos + (int64_t)L > s1) return -1;
                memset(B + pos, sym, (size_t)L);
                pos += (int64_t)L;
            }
        }
        if (pos != s1) return -1;
    }
    return 0;
}

/* Occurrences of each symbol in B[0, i) for every i of pos[0..k), by the
 * format's rank rule. out: k rows of 6. Returns 0 or -1. */
int orc_rle_rank(const uint64_t *blocks, const int64_t *seg, const uint16_t *row, int64_t n, int q,
                 const int64_t *pos, int64_t k, int64_t *out)
{
    int64_t nseg = (n + RLE_SEG - 1) >> RLE_SEG_SHIFT, x;
    for (x = 0; x < k; ++x) {
        int64_t i = pos[x], *o = out + x * 6, s, off, b, p, hc[6];
        int c;
        if (i < 0 || i > n) return -1;
        if (i == n) {
            for (c = 0; c < 6; ++c) o[c] = seg[nseg * 8 + c];
            continue;
        }
        s = i >> RLE_SEG_SHIFT;
        off = i - (s << RLE_SEG_SHIFT);
        for (c = 0; c < 6; ++c) o[c] = seg[s * 8 + c];
        if (off == 0) continue;
        b = seg[s * 8 + 6] + row[i >> q];
        for (;;) {
            const uint64_t *w = blocks + b * RLE_WORDS;
            int np, t;
            orc_br r;
            orc_read_header(w, &p, hc, &np);
            r.w = w;
            r.bit = 0;
            for (t = 0; t < np && p < off; ++t) {
                int sym;
                uint64_t L;
                int64_t take;
                if (orc_get_piece(&r, &sym, &L)) return -1;
                take = (int64_t)L < off - p ? (int64_t)L : off - p;
                hc[sym] += take;
                p += take;
            }
            if (p >= off) {
                for (c = 0; c < 6; ++c) o[c] += hc[c];
                break;
            }
            ++b; /* i lies in a later block of the segment */
            if (b >= seg[(s + 1) * 8 + 6]) return -1;
        }
    }
    return 0;
}
