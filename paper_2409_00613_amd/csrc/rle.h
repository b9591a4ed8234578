// Run-length static BWT index on the device: its view and rank by decoding.
//
// The format is the bit-packed static one of Sec. 2.2 (Fig. 2b): blocks of
// run-length coded BWT whose run lengths are Elias delta codes, each block
// carrying the marginal counts before it, plus an index row that maps a
// position to its block.
//
//   Segments  B[0, n) is cut into segments of 2^20 symbols; each segment is
//             cut into its maximal runs of one symbol (pieces, 1 .. 2^20
//             long), so a piece never crosses a segment start.
//   Code      a piece is its symbol in 3 bits, then its length L in the
//             Elias delta code (K - 1 zeros, N in K bits, the N - 1 low bits
//             of L; N the bit length of L, K that of N), most significant bit
//             first: at most 3 + 29 = 32 bits.
//   Blocks    128 bytes (16 uint64 words, one L2 line): a 2-word header and
//             896 stream bits, stream bit t at bit 63 - t % 64 of word
//             2 + t / 64. Header word 0 = offset of the block's first symbol
//             in its segment (bits 0-19), occurrences of A and C in the
//             segment before the block (20-39, 40-59), low 4 bits of the
//             piece count (60-63); word 1 = occurrences of G, T, N (0-19,
//             20-39, 40-59), high 4 bits of the piece count. $ occurrences
//             are the offset minus the five counts.
//   Packing   a segment's pieces fill blocks in order, greedily; every
//             segment starts a new block.
//   Tables    per segment (and one row after the last): occurrences of the
//             six symbols before it, its first block, 0 (8 int64). Index row
//             entry j = block holding position j << q, counted from its
//             segment's first block (uint16; a segment has fewer than 2^16
//             blocks because a full block holds at least 27 pieces).
//
// Rank at i: i = n gives the totals; a segment start gives its table row;
// else the table row + the header of the block the index row names + the
// pieces decoded from that block's start up to i, moving on to the next
// block when i lies past the named one.
#pragma once

#include "rb3_internal.h"

namespace rb3 {

constexpr int RLE_SEG_SHIFT = 20;
constexpr int64_t RLE_SEG = (int64_t)1 << RLE_SEG_SHIFT;
constexpr int RLE_WORDS = 16;
constexpr int RLE_BITS = 896;
constexpr int RLE_MAX_PIECES = RLE_BITS / 4;  // one-symbol pieces cost 4 bits

struct RleView {
    const uint64_t *blk;  // nblk * 16 words
    const int64_t *seg;   // (nseg + 1) * 8
    const uint16_t *row;  // ((n - 1) >> q) + 1
    int64_t n, m, nseg, nblk;
    int64_t C[8];  // C[0..5]; C[6] = n
    int32_t q;
};

// Stream word k (0..14; 14 reads as 0) of a block held in registers, by a
// tree of selects on the bits of k (indexing a register array by a value
// known only at run time would put the array in scratch memory).
__device__ __forceinline__ uint64_t rle_word(const uint64_t w[14], uint32_t k) {
    const bool b0 = k & 1u, b1 = k & 2u, b2 = k & 4u, b3 = k & 8u;
    const uint64_t a0 = b0 ? w[1] : w[0], a1 = b0 ? w[3] : w[2], a2 = b0 ? w[5] : w[4], a3 = b0 ? w[7] : w[6];
    const uint64_t a4 = b0 ? w[9] : w[8], a5 = b0 ? w[11] : w[10], a6 = b0 ? w[13] : w[12];
    const uint64_t c0 = b1 ? a1 : a0, c1 = b1 ? a3 : a2, c2 = b1 ? a5 : a4, c3 = b1 ? 0ull : a6;
    const uint64_t d0 = b2 ? c1 : c0, d1 = b2 ? c3 : c2;
    return b3 ? d1 : d0;
}

// Occurrences of every symbol in B[0, i), 0 <= i <= n.
__device__ __forceinline__ void rle_occ_all(const RleView &v, int64_t i, int64_t out[6]) {
    const bool end = i >= v.n;
    const int64_t s = end ? v.nseg : (i >> RLE_SEG_SHIFT);
    const uint32_t off = end ? 0u : (uint32_t)(i & (RLE_SEG - 1));
    // the table row and the index-row entry are read together
    const int64_t *sr = v.seg + s * 8;
    const uint32_t rj = off ? (uint32_t)v.row[i >> v.q] : 0u;
#pragma unroll
    for (int c = 0; c < 6; ++c) out[c] = sr[c];
    if (off == 0) return;
    int64_t b = sr[6] + rj;
    for (;;) {
        const uint4 *p = (const uint4 *)(v.blk + b * RLE_WORDS);
        const uint4 q0 = p[0], q1 = p[1], q2 = p[2], q3 = p[3], q4 = p[4], q5 = p[5], q6 = p[6], q7 = p[7];
        const uint64_t h0 = u64_lo(q0), h1 = u64_hi(q0);
        const uint64_t w[14] = {u64_lo(q1), u64_hi(q1), u64_lo(q2), u64_hi(q2), u64_lo(q3), u64_hi(q3), u64_lo(q4),
                                u64_hi(q4), u64_lo(q5), u64_hi(q5), u64_lo(q6), u64_hi(q6), u64_lo(q7), u64_hi(q7)};
        uint32_t pos = (uint32_t)(h0 & 0xFFFFFu);
        const uint32_t np = (uint32_t)(h0 >> 60) | ((uint32_t)(h1 >> 60) << 4);
        // decoded occurrences, 21 bits a symbol: $ A C in one word, G T N
        // in the other (a block holds fewer than 2^20 symbols)
        uint64_t acc0 = 0, acc1 = 0;
        uint32_t bit = 0, k = 0;
        uint64_t cur = w[0], nxt = w[1];
        for (uint32_t t = 0; t < np && pos < off; ++t) {
            const uint32_t r = bit & 63u;
            uint64_t win = r ? (cur << r) | (nxt >> (64u - r)) : cur;
            const uint32_t sym = (uint32_t)(win >> 61);
            win <<= 3;
            const uint32_t z = (uint32_t)__clzll((long long)win);  // K - 1
            const uint32_t kb = 2u * z + 1u;                       // the zeros and N
            const uint32_t N = (uint32_t)(win >> (64u - kb));
            const uint64_t rest = win << kb;
            const uint32_t L = N > 1u ? ((1u << (N - 1u)) | (uint32_t)(rest >> (65u - N))) : 1u;
            const uint32_t take = L < off - pos ? L : off - pos;
            const uint64_t add = (uint64_t)take << (21u * (sym >= 3u ? sym - 3u : sym));
            if (sym < 3u)
                acc0 += add;
            else
                acc1 += add;
            pos += take;
            bit += 3u + kb + N - 1u;
            if ((bit >> 6) != k) {  // a piece crosses at most one word boundary
                ++k;
                cur = nxt;
                nxt = rle_word(w, k + 1u);
            }
        }
        if (pos >= off) {
            const int64_t hA = (int64_t)((h0 >> 20) & 0xFFFFFu), hC = (int64_t)((h0 >> 40) & 0xFFFFFu);
            const int64_t hG = (int64_t)(h1 & 0xFFFFFu), hT = (int64_t)((h1 >> 20) & 0xFFFFFu);
            const int64_t hN = (int64_t)((h1 >> 40) & 0xFFFFFu);
            const int64_t hS = (int64_t)(h0 & 0xFFFFFu) - hA - hC - hG - hT - hN;
            out[0] += hS + (int64_t)(acc0 & 0x1FFFFFu);
            out[1] += hA + (int64_t)((acc0 >> 21) & 0x1FFFFFu);
            out[2] += hC + (int64_t)((acc0 >> 42) & 0x1FFFFFu);
            out[3] += hG + (int64_t)(acc1 & 0x1FFFFFu);
            out[4] += hT + (int64_t)((acc1 >> 21) & 0x1FFFFFu);
            out[5] += hN + (int64_t)((acc1 >> 42) & 0x1FFFFFu);
            return;
        }
        // i lies past this block: the next block's header counts everything
        // before it
        if (++b >= v.nblk) return;  // only on a malformed index
    }
}

// rle.hip: the build from the device index (row shift q_req 0 = automatic:
// the largest q in [4, 16] with 2^q <= n / (4 * blocks)), the whole decode,
// and the checks of a loaded index (*d_bad set on a failed check).
struct RleBuild {
    DBuf blk, seg, row;
    int64_t n = 0, nseg = 0, nblk = 0, npieces = 0;
    int64_t tot[6] = {0, 0, 0, 0, 0, 0};
    int32_t q = 0;
};
int rle_build(Ctx &c, const DevIndex &ix, int32_t q_req, RleBuild &out);
int rle_decode_all(Ctx &c, const RleView &v, uint8_t *d_out);
int rle_check(Ctx &c, const RleView &v, int32_t *d_bad);
// query.hip: counts and SMEMs on the run-length index
int count_queries_rle(Ctx &c, const RleView &v, const uint8_t *d_q, const int64_t *d_qoff, int64_t nq,
                      int64_t *d_lo, int64_t *d_hi);
int smem_run_rle(Ctx &c, const RleView &v, const uint8_t *d_q, const int64_t *qlens, int64_t nq, int32_t min_len,
                 int64_t min_occ, int64_t out_cap, rb3_smem_t *d_out, int64_t *d_out_off, int64_t *h_kept,
                 int64_t *h_exts);

}  // namespace rb3
