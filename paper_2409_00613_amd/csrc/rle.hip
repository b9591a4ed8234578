// Building, checking and decoding the run-length static index (format in
// rle.h; Sec. 2.2, Fig. 2b).
//
// The build runs on the device from the 3-bit-plane index:
//   1. the BWT is unpacked to one byte a symbol;
//   2. piece starts (a symbol that differs from the one before it, or a
//      segment start) are counted per 4096-symbol tile, the counts scanned,
//      and the start positions written in order;
//   3. one thread per segment walks its pieces and packs them greedily into
//      blocks: a first pass counts the blocks and the symbols of each
//      segment, the host lays out the tables, and a second pass writes the
//      blocks and the index row.
// Pieces never cross a segment start, so segments pack independently.
#include "rle.h"

#include <vector>

namespace rb3 {

constexpr int RLE_TILE = 4096;            // symbols per tile of the start scan
constexpr int RLE_TILE_THREADS = 256;     // 16 symbols a thread
constexpr int RLE_TILES_PER_SEG = (int)(RLE_SEG / RLE_TILE);

__device__ __forceinline__ uint32_t bitlen32(uint32_t v) { return 32u - (uint32_t)__clz((int)v); }

// Start flags of the 16 symbols base .. base + 15 (bit k for base + k).
__device__ __forceinline__ uint32_t piece_starts16(const uint8_t *__restrict__ codes, int64_t n, int64_t base) {
    uint8_t s[16];
    if (base + 16 <= n) {
        const uint4 v = *(const uint4 *)(codes + base);
        const uint32_t x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) s[k] = (uint8_t)(x[k >> 2] >> (8 * (k & 3)));
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) s[k] = base + k < n ? codes[base + k] : 0;
    }
    const int prev = base > 0 ? (int)codes[base - 1] : -1;
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int64_t i = base + k;
        const int before = k ? (int)s[k - 1] : prev;
        const bool st = i < n && (before != (int)s[k] || (i & (RLE_SEG - 1)) == 0);
        m |= (uint32_t)st << k;
    }
    return m;
}

// Count mode (P == nullptr): cnt[tile] = starts in the tile, and their sum
// in 64 bits. Emit mode: the start positions at toff[tile] + their rank.
__global__ void __launch_bounds__(RLE_TILE_THREADS) k_rle_starts(const uint8_t *__restrict__ codes, int64_t n,
                                                                 uint32_t *__restrict__ cnt,
                                                                 unsigned long long *__restrict__ sum,
                                                                 const uint32_t *__restrict__ toff,
                                                                 int64_t *__restrict__ P) {
    __shared__ uint32_t wsum[RLE_TILE_THREADS / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * RLE_TILE + (int64_t)tid * 16;
    const uint32_t m = piece_starts16(codes, n, base);
    const uint32_t c = (uint32_t)__popc(m);
    uint32_t inc = c;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(inc, d);
        if (lane >= d) inc += t;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t pre = inc - c, tot = 0;
    for (int w = 0; w < RLE_TILE_THREADS / 64; ++w) {
        if (w < wave) pre += wsum[w];
        tot += wsum[w];
    }
    if (!P) {
        if (tid == 0) {
            cnt[blockIdx.x] = tot;
            atomicAdd(sum, (unsigned long long)tot);
        }
        return;
    }
    int64_t o = (int64_t)toff[blockIdx.x] + pre;
    uint32_t mm = m;
    while (mm) {
        const int k = __ffs((int)mm) - 1;
        P[o++] = base + k;
        mm &= mm - 1u;
    }
}

// First piece of each segment: a segment start is a piece start and the
// first symbol of its tile.
__global__ void k_rle_segp(const uint32_t *__restrict__ toff, int64_t nseg, uint32_t total,
                           uint32_t *__restrict__ segp) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s <= nseg;
         s += (int64_t)gridDim.x * blockDim.x)
        segp[s] = s < nseg ? toff[s * RLE_TILES_PER_SEG] : total;
}

// Sequential bit writer into global words, most significant bit first.
struct BitOut {
    uint64_t *w;  // next word
    uint64_t acc;
    uint32_t nb;
    __device__ void put(uint64_t v, uint32_t bits) {  // bits <= 32
        if (nb + bits <= 64u) {
            acc |= v << (64u - nb - bits);
            nb += bits;
            if (nb == 64u) {
                *w++ = acc;
                acc = 0;
                nb = 0;
            }
        } else {
            const uint32_t h = 64u - nb;
            acc |= v >> (bits - h);
            *w++ = acc;
            nb = bits - h;
            acc = v << (64u - nb);
        }
    }
    __device__ void flush() {
        if (nb) *w = acc;
    }
};

// One thread per segment. Pass 1 (WRITE false): blocks and symbol counts of
// the segment. Pass 2: the blocks and the segment's index-row entries.
template <bool WRITE>
__global__ void k_rle_pack(const uint8_t *__restrict__ codes, int64_t n, const int64_t *__restrict__ P,
                           const uint32_t *__restrict__ segp, int64_t nseg, uint32_t *__restrict__ nblocks,
                           int64_t *__restrict__ segcnt, const int64_t *__restrict__ seg,
                           uint64_t *__restrict__ blk, uint16_t *__restrict__ row, int32_t q) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    const int64_t s0 = s << RLE_SEG_SHIFT;
    const int64_t s1 = s0 + RLE_SEG < n ? s0 + RLE_SEG : n;
    const int64_t fb = WRITE ? seg[s * 8 + 6] : 0;
    int64_t b = fb;           // open block
    uint32_t used = 0, np = 0;
    uint32_t cnt[6] = {0, 0, 0, 0, 0, 0}, bc[6] = {0, 0, 0, 0, 0, 0};
    uint32_t boff = 0;
    BitOut out{WRITE ? blk + b * RLE_WORDS + 2 : nullptr, 0, 0};
    // closes block b, which covers segment offsets [boff, end)
    auto close = [&](uint32_t end) {
        if (!WRITE) return;
        out.flush();
        uint64_t *h = blk + b * RLE_WORDS;
        h[0] = (uint64_t)boff | ((uint64_t)bc[1] << 20) | ((uint64_t)bc[2] << 40) | ((uint64_t)(np & 15u) << 60);
        h[1] = (uint64_t)bc[3] | ((uint64_t)bc[4] << 20) | ((uint64_t)bc[5] << 40) | ((uint64_t)(np >> 4) << 60);
        const int64_t j0 = (s0 + boff + ((int64_t)1 << q) - 1) >> q;
        const int64_t j1 = (s0 + end + ((int64_t)1 << q) - 1) >> q;
        for (int64_t j = j0; j < j1; ++j) row[j] = (uint16_t)(b - fb);
    };
    const int64_t p1 = segp[s + 1];
    for (int64_t p = segp[s]; p < p1; ++p) {
        const int64_t st = P[p];
        const uint32_t L = (uint32_t)(P[p + 1] - st);
        const uint32_t sym = codes[st];
        const uint32_t N = bitlen32(L), K = bitlen32(N);
        const uint32_t dbits = 2u * K + N - 2u;
        const uint32_t bits = 3u + dbits;
        if (used + bits > (uint32_t)RLE_BITS) {
            close((uint32_t)(st - s0));
            ++b;
            used = 0;
            np = 0;
            boff = (uint32_t)(st - s0);
#pragma unroll
            for (int c = 0; c < 6; ++c) bc[c] = cnt[c];
            if (WRITE) out = BitOut{blk + b * RLE_WORDS + 2, 0, 0};
        }
        if (WRITE) {
            // the K - 1 zeros are the leading zeros of N in dbits - (N - 1) bits
            const uint64_t code = ((uint64_t)sym << dbits) | ((uint64_t)N << (N - 1u)) |
                                  (uint64_t)(L & ((1u << (N - 1u)) - 1u));
            out.put(code, bits);
        }
        used += bits;
        ++np;
#pragma unroll
        for (int c = 0; c < 6; ++c) cnt[c] += (uint32_t)c == sym ? L : 0u;
    }
    close((uint32_t)(s1 - s0));
    if (!WRITE) {
        nblocks[s] = (uint32_t)(b - fb + 1);
#pragma unroll
        for (int c = 0; c < 6; ++c) segcnt[s * 6 + c] = cnt[c];
    }
}

// Every symbol back out of the blocks: one thread per block.
__global__ void k_rle_decode(RleView v, uint8_t *__restrict__ out) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < v.nseg;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s0 = s << RLE_SEG_SHIFT;
        for (int64_t b = v.seg[s * 8 + 6]; b < v.seg[(s + 1) * 8 + 6]; ++b) {
            const uint64_t *w = v.blk + b * RLE_WORDS;
            int64_t pos = s0 + (int64_t)(w[0] & 0xFFFFFu);
            const uint32_t np = (uint32_t)(w[0] >> 60) | ((uint32_t)(w[1] >> 60) << 4);
            uint32_t bit = 0;
            for (uint32_t t = 0; t < np; ++t) {
                const uint32_t k = bit >> 6, r = bit & 63u;
                const uint64_t a = w[2 + k], c = k + 1 < 14 ? w[3 + k] : 0ull;
                uint64_t win = r ? (a << r) | (c >> (64u - r)) : a;
                const uint8_t sym = (uint8_t)(win >> 61);
                win <<= 3;
                const uint32_t z = (uint32_t)__clzll((long long)win), kb = 2u * z + 1u;
                const uint32_t N = (uint32_t)(win >> (64u - kb));
                const uint32_t L = N > 1u ? ((1u << (N - 1u)) | (uint32_t)((win << kb) >> (65u - N))) : 1u;
                for (uint32_t x = 0; x < L && pos + x < v.n; ++x) out[pos + x] = sym;
                pos += L;
                bit += 3u + kb + N - 1u;
            }
        }
    }
}

// Checks of a loaded index, one thread per segment: valid codes that fit
// their block, block offsets and header counts that chain from block to
// block and end at the segment's length and symbol counts, and index-row
// entries that name the block holding their position.
__global__ void k_rle_check(RleView v, int32_t *__restrict__ bad) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < v.nseg;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s0 = s << RLE_SEG_SHIFT;
        const int64_t len = (s0 + RLE_SEG < v.n ? s0 + RLE_SEG : v.n) - s0;
        const int64_t b0 = v.seg[s * 8 + 6], b1 = v.seg[(s + 1) * 8 + 6];
        int64_t cnt[6] = {0, 0, 0, 0, 0, 0};
        int64_t pos = 0;
        bool ok = b1 > b0 && b1 - b0 < 65536;
        for (int64_t b = b0; ok && b < b1; ++b) {
            const uint64_t *w = v.blk + b * RLE_WORDS;
            const int64_t h[6] = {0, (int64_t)((w[0] >> 20) & 0xFFFFFu), (int64_t)((w[0] >> 40) & 0xFFFFFu),
                                  (int64_t)(w[1] & 0xFFFFFu), (int64_t)((w[1] >> 20) & 0xFFFFFu),
                                  (int64_t)((w[1] >> 40) & 0xFFFFFu)};
            const int64_t off = (int64_t)(w[0] & 0xFFFFFu);
            const int64_t hs = off - h[1] - h[2] - h[3] - h[4] - h[5];
            ok = off == pos && hs == cnt[0];
            for (int c = 1; c < 6; ++c) ok = ok && h[c] == cnt[c];
            const uint32_t np = (uint32_t)(w[0] >> 60) | ((uint32_t)(w[1] >> 60) << 4);
            ok = ok && np >= 1 && np <= (uint32_t)RLE_MAX_PIECES;
            uint32_t bit = 0;
            for (uint32_t t = 0; ok && t < np; ++t) {
                if (bit + 4u > (uint32_t)RLE_BITS) {
                    ok = false;
                    break;
                }
                const uint32_t k = bit >> 6, r = bit & 63u;
                const uint64_t a = w[2 + k], c = k + 1 < 14 ? w[3 + k] : 0ull;
                uint64_t win = r ? (a << r) | (c >> (64u - r)) : a;
                const uint32_t sym = (uint32_t)(win >> 61);
                win <<= 3;
                const uint32_t z = (uint32_t)__clzll((long long)win);
                if (sym > 5u || z > 4u) {
                    ok = false;
                    break;
                }
                const uint32_t kb = 2u * z + 1u, N = (uint32_t)(win >> (64u - kb));
                if (N < 1u || N > 21u || bitlen32(N) != z + 1u) {
                    ok = false;
                    break;
                }
                const uint32_t L = N > 1u ? ((1u << (N - 1u)) | (uint32_t)((win << kb) >> (65u - N))) : 1u;
                bit += 3u + kb + N - 1u;
                ok = bit <= (uint32_t)RLE_BITS && pos + L <= len;
                cnt[sym] += L;
                pos += L;
            }
        }
        ok = ok && pos == len;
        for (int c = 0; c < 6; ++c) ok = ok && v.seg[(s + 1) * 8 + c] - v.seg[s * 8 + c] == cnt[c];
        // index row
        const int64_t qq = (int64_t)1 << v.q;
        int64_t b = b0;
        for (int64_t j = (s0 + qq - 1) >> v.q; ok && (j << v.q) < s0 + len; ++j) {
            const int64_t p = (j << v.q) - s0;
            while (b + 1 < b1 && (int64_t)(v.blk[(b + 1) * RLE_WORDS] & 0xFFFFFu) <= p) ++b;
            ok = (int64_t)v.row[j] == b - b0;
        }
        if (!ok) atomicOr(bad, 1);
    }
}

int rle_build(Ctx &c, const DevIndex &ix, int32_t q_req, RleBuild &out) {
    const int64_t n = ix.n;
    if (n <= 0) {
        set_error(RB3_EINVAL, "run-length index of an empty BWT");
        return RB3_EINVAL;
    }
    if (q_req != 0 && (q_req < 4 || q_req > 20)) {
        set_error(RB3_EINVAL, "row shift must be 0 (automatic) or 4..20");
        return RB3_EINVAL;
    }
    const int64_t nseg = (n + RLE_SEG - 1) >> RLE_SEG_SHIFT;
    const int64_t ntiles = (n + RLE_TILE - 1) / RLE_TILE;
    DBuf codes, cnt, toff, sum, P, segp, nbk, segcnt;
    RB3_ALLOC(codes, &c, n + 16);
    RB3_TRY(unpack_codes(c, ix, codes.as<uint8_t>()));
    RB3_ALLOC(cnt, &c, (ntiles + 1) * sizeof(uint32_t));
    RB3_ALLOC(toff, &c, (ntiles + 1) * sizeof(uint32_t));
    RB3_ALLOC(sum, &c, sizeof(unsigned long long));
    RB3_HIP(hipMemsetAsync(sum.p, 0, sizeof(unsigned long long), c.stream));
    RB3_LAUNCH("rle_starts", k_rle_starts, dim3((unsigned)ntiles), dim3(RLE_TILE_THREADS), 0, c.stream,
               codes.as<uint8_t>(), n, cnt.as<uint32_t>(), sum.as<unsigned long long>(), nullptr, nullptr);
    unsigned long long npieces = 0;
    RB3_HIP(hipMemcpyAsync(&npieces, sum.p, sizeof(npieces), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipStreamSynchronize(c.stream));
    if (npieces >= (unsigned long long)UINT32_MAX) {
        set_error(RB3_ELIMIT, "run-length index: 2^32 or more runs");
        return RB3_ELIMIT;
    }
    RB3_TRY(scan_u32(c, cnt.as<uint32_t>(), toff.as<uint32_t>(), ntiles, false, false, nullptr));
    RB3_ALLOC(P, &c, (npieces + 1) * sizeof(int64_t));
    RB3_LAUNCH("rle_starts", k_rle_starts, dim3((unsigned)ntiles), dim3(RLE_TILE_THREADS), 0, c.stream,
               codes.as<uint8_t>(), n, cnt.as<uint32_t>(), sum.as<unsigned long long>(), toff.as<uint32_t>(),
               P.as<int64_t>());
    RB3_HIP(hipMemcpyAsync(P.as<int64_t>() + npieces, &n, sizeof(int64_t), hipMemcpyHostToDevice, c.stream));
    RB3_ALLOC(segp, &c, (nseg + 1) * sizeof(uint32_t));
    RB3_LAUNCH("rle_segp", k_rle_segp, grid_for(nseg + 1, 256), dim3(256), 0, c.stream, toff.as<uint32_t>(), nseg,
               (uint32_t)npieces, segp.as<uint32_t>());
    RB3_ALLOC(nbk, &c, nseg * sizeof(uint32_t));
    RB3_ALLOC(segcnt, &c, nseg * 6 * sizeof(int64_t));
    const dim3 sg = grid_for(nseg, 64), sb(64);
    RB3_LAUNCH("rle_pack", k_rle_pack<false>, sg, sb, 0, c.stream, codes.as<uint8_t>(), n, P.as<int64_t>(),
               segp.as<uint32_t>(), nseg, nbk.as<uint32_t>(), segcnt.as<int64_t>(), nullptr, nullptr, nullptr, 0);
    std::vector<uint32_t> hnb(nseg);
    std::vector<int64_t> hcnt(nseg * 6);
    RB3_HIP(hipMemcpyAsync(hnb.data(), nbk.p, nseg * sizeof(uint32_t), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipMemcpyAsync(hcnt.data(), segcnt.p, nseg * 6 * sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipStreamSynchronize(c.stream));
    // the segment table
    std::vector<int64_t> hseg((nseg + 1) * 8, 0);
    int64_t nblk = 0;
    for (int64_t s = 0; s <= nseg; ++s) {
        hseg[s * 8 + 6] = nblk;
        if (s == nseg) break;
        for (int k = 0; k < 6; ++k) hseg[(s + 1) * 8 + k] = hseg[s * 8 + k] + hcnt[s * 6 + k];
        nblk += hnb[s];
    }
    // row shift: the largest q in [4, 16] with 2^q <= n / (4 * blocks), else 4
    int32_t q = q_req;
    if (q == 0) {
        q = 4;
        while (q < 16 && ((int64_t)1 << (q + 1)) <= n / (4 * nblk)) ++q;
    }
    const int64_t nrow = ((n - 1) >> q) + 1;
    RB3_ALLOC(out.blk, &c, nblk * RLE_WORDS * sizeof(uint64_t));
    RB3_ALLOC(out.seg, &c, (nseg + 1) * 8 * sizeof(int64_t));
    RB3_ALLOC(out.row, &c, nrow * sizeof(uint16_t));
    RB3_HIP(hipMemsetAsync(out.blk.p, 0, nblk * RLE_WORDS * sizeof(uint64_t), c.stream));
    RB3_HIP(hipMemcpyAsync(out.seg.p, hseg.data(), (nseg + 1) * 8 * sizeof(int64_t), hipMemcpyHostToDevice,
                           c.stream));
    RB3_LAUNCH("rle_pack", k_rle_pack<true>, sg, sb, 0, c.stream, codes.as<uint8_t>(), n, P.as<int64_t>(),
               segp.as<uint32_t>(), nseg, nullptr, nullptr, out.seg.as<int64_t>(), out.blk.as<uint64_t>(),
               out.row.as<uint16_t>(), q);
    RB3_HIP(hipStreamSynchronize(c.stream));
    out.n = n;
    out.nseg = nseg;
    out.nblk = nblk;
    out.npieces = (int64_t)npieces;
    out.q = q;
    for (int k = 0; k < 6; ++k) out.tot[k] = hseg[nseg * 8 + k];
    return RB3_OK;
}

int rle_decode_all(Ctx &c, const RleView &v, uint8_t *d_out) {
    RB3_LAUNCH("rle_decode", k_rle_decode, grid_for(v.nseg, 64), dim3(64), 0, c.stream, v, d_out);
    return RB3_OK;
}

int rle_check(Ctx &c, const RleView &v, int32_t *d_bad) {
    RB3_LAUNCH("rle_check", k_rle_check, grid_for(v.nseg, 64), dim3(64), 0, c.stream, v, d_bad);
    return RB3_OK;
}

}  // namespace rb3
