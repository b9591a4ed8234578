// Chain chunks cut at content-defined positions, and the lane order of the
// chain kernel.
//
// The LF chains of Algorithm 1 (Sec. 2.2) walk every new string right to
// left; the chain kernel cuts the strings into chunks so that many lanes run
// at once (merge.hip). On pangenome batches the strings are near-copies of
// one another and of the existing index: the suffixes of different new
// haplotypes at one locus sort next to each other, so walks that pass the
// same locus at the same step read the same index blocks. Chunks cut at
// fixed offsets never line up that way (indels shift every haplotype's
// offsets). Here the cut points are chosen by content:
//
//   * candidates: strand starts, and positions whose next CDC_K symbols hash
//     to 0 modulo CDC_D (about one position in CDC_D);
//   * anchors: candidates whose gap to the previous candidate is at least
//     4 CDC_D, or lmax / 2 if that is smaller (about one candidate in e^4 of
//     them, so the stretch between anchors is short enough for one thread to
//     cut, and still several chunks long); an anchor depends only
//     on the sequence around it, so the same locus gives the same anchor in
//     every haplotype that shares the sequence there;
//   * the stretch between two anchors is cut from its right end into pieces
//     of at most lmax symbols, each piece ending at the leftmost candidate
//     within reach (a fixed-length cut only when none is).
//
// The chain kernel then takes the chunks in the order of a key made of the
// CDC_TAIL symbols each chunk's walk reads first (and whether it starts at
// its strand's sentinel), so chunks of different haplotypes at one locus run
// in the same wave, step in lockstep and issue the same block addresses,
// which the memory pipeline serves with one line per wave instead of one
// per lane. The chunks themselves stay in string order (the fix-up needs
// each chunk's right neighbour at index + 1).
#include "rb3_internal.h"

namespace rb3 {

constexpr int CDC_K = 10;        // symbols hashed per candidate
constexpr uint32_t CDC_D = 256;  // one candidate in CDC_D positions
constexpr int CDC_TAIL = 16;     // symbols of a chunk's walk in its sort key
constexpr int64_t CDC_GAP = 4 * CDC_D;  // anchor gap (capped at lmax / 2)

__device__ __forceinline__ uint64_t cdc_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// One thread per 64 positions: bit j of word w marks position 64 w + j as a
// candidate; cnt[w] = candidates in the word. The thread reads the word's
// 64 symbols and the CDC_K - 1 after them (80 aligned bytes) and rolls the
// CDC_K-mer starting at each position across them. Q has at least 80
// readable bytes past the start of its last word (zero past its end), and
// every strand ends with its sentinel (0), so a k-mer that would cross a
// strand's end has a zero in it.
__device__ __forceinline__ uint32_t byte_of(const uint4 (&v)[5], int q) {
    const uint4 &x = v[q >> 4];
    const int w = (q >> 2) & 3;
    const uint32_t d = w == 0 ? x.x : (w == 1 ? x.y : (w == 2 ? x.z : x.w));
    return (d >> (8 * (q & 3))) & 0xFFu;
}

__global__ void k_cdc_mark(const uint8_t *__restrict__ Q, int64_t nw, uint64_t *__restrict__ bits,
                           uint32_t *__restrict__ cnt) {
    constexpr uint32_t KMASK = (1u << (3 * CDC_K)) - 1u;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nw; w += (int64_t)gridDim.x * blockDim.x) {
        const int64_t base = w << 6;
        const uint4 *src = (const uint4 *)(Q + base);
        uint4 v[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) v[i] = src[i];
        uint32_t prev = base > 0 ? Q[base - 1] : 0u;
        uint64_t word = 0;
        uint32_t packed = 0;
        int run = 0;  // symbols other than $ ending at q (capped at CDC_K)
#pragma unroll
        for (int q = 0; q < 64 + CDC_K - 1; ++q) {
            const uint32_t x = byte_of(v, q);
            if (q < 64 && x != 0 && prev == 0) word |= 1ull << q;  // a strand start
            prev = x;
            if (x != 0) {
                packed = ((packed << 3) | x) & KMASK;
                run = run < CDC_K ? run + 1 : CDC_K;
            } else {
                run = 0;
            }
            const int p = q - (CDC_K - 1);  // the k-mer Q[p .. q] starts at p
            if (p >= 0 && p < 64 && run == CDC_K && (cdc_mix(packed) & (CDC_D - 1)) == 0) word |= 1ull << p;
        }
        bits[w] = word;
        cnt[w] = (uint32_t)__popcll(word);
    }
}

// The candidates' positions, in order (off: exclusive scan of cnt).
__global__ void k_cdc_list(const uint64_t *__restrict__ bits, const uint32_t *__restrict__ off, int64_t nw,
                           uint32_t *__restrict__ pos) {
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nw; w += (int64_t)gridDim.x * blockDim.x) {
        uint64_t b = bits[w];
        uint32_t o = off[w];
        while (b) {
            const int j = __ffsll((unsigned long long)b) - 1;
            pos[o++] = (uint32_t)((w << 6) + j);
            b &= b - 1;
        }
    }
}

// Anchor flags: strand starts, and candidates at least gap after the
// previous candidate (which lies in the same strand: the strand's start is
// itself a candidate).
__global__ void k_cdc_anchor(const uint8_t *__restrict__ Q, const uint32_t *__restrict__ pos, int64_t ncand,
                             uint32_t gap, uint32_t *__restrict__ flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ncand;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = pos[i];
        const bool start = p == 0 || Q[p - 1] == 0;
        flag[i] = (i == 0 || start || p - pos[i - 1] >= gap) ? 1u : 0u;
    }
}

__global__ void k_cdc_alist(const uint32_t *__restrict__ flag, const uint32_t *__restrict__ off, int64_t ncand,
                            uint32_t *__restrict__ alist) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ncand;
         i += (int64_t)gridDim.x * blockDim.x)
        if (flag[i]) alist[off[i]] = (uint32_t)i;
}

// Pieces of the stretch that starts at anchor j, cut from its right end.
// Pass 1 (WRITE false) counts them into npc[j]; pass 2 writes them, in
// string order, at poff[j] .., with each chunk's sort key.
template <bool WRITE>
__global__ void k_cdc_pieces(const uint8_t *__restrict__ Q, int64_t n2, const uint32_t *__restrict__ pos,
                             int64_t ncand, const uint32_t *__restrict__ alist, int64_t nanch, int64_t lmax,
                             uint32_t *__restrict__ npc, const uint32_t *__restrict__ poff, Chunk *__restrict__ ch,
                             uint64_t *__restrict__ key) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nanch;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ia = alist[j];
        const int64_t ib = j + 1 < nanch ? (int64_t)alist[j + 1] : ncand;
        const int64_t S = pos[ia];
        const int64_t P2 = j + 1 < nanch ? (int64_t)pos[ib] : n2;
        // the stretch ends before the next anchor, or at its strand's sentinel
        const int64_t E = Q[P2 - 1] == 0 ? P2 - 1 : P2;
        int64_t R = E, hi = ib - 1;  // candidates (ia, hi] lie inside the stretch
        uint32_t t = 0;
        const int64_t top = WRITE ? (int64_t)poff[j + 1] - 1 : 0;
        for (;;) {
            int64_t cut;
            if (R - S <= lmax) {
                cut = S;
            } else {
                while (hi > ia && (int64_t)pos[hi] >= R) --hi;
                if (hi > ia && (int64_t)pos[hi] >= R - lmax) {
                    int64_t idx = hi;
                    while (idx - 1 > ia && (int64_t)pos[idx - 1] >= R - lmax) --idx;
                    cut = pos[idx];
                    hi = idx - 1;
                } else {
                    cut = R - lmax;
                }
            }
            if (WRITE) {
                const int64_t at = top - t;
                Chunk c;
                c.p0 = cut;
                c.len = (int32_t)(R - cut);
                c.last = Q[R] == 0 ? 1 : 0;
                c.first = (cut == 0 || Q[cut - 1] == 0) ? 1 : 0;
                c.pad = 0;
                ch[at] = c;
                // the symbols the walk reads first, then whether it starts
                // from a known value (at the sentinel)
                const int64_t a = R - CDC_TAIL > cut ? R - CDC_TAIL : cut;
                uint64_t packed = 0;
                for (int64_t q = a; q < R; ++q) packed = (packed << 3) | Q[q];
                key[at] = ((uint64_t)c.last << 24) | (cdc_mix(packed ^ ((uint64_t)(R - a) << 58)) & 0xFFFFFFull);
            }
            ++t;
            if (cut == S) break;
            R = cut;
        }
        if (!WRITE) npc[j] = t;
    }
}

int make_chunks(Ctx &c, const uint8_t *d_Q, int64_t n2, int64_t lmax, DBuf &chunks, int64_t *nch_out, DBuf &perm,
                int32_t *d_guard) {
    const int64_t nw = (n2 + 63) >> 6;
    DBuf bits, wcnt, cpos, aflag, aoff, alist, npc, tot;
    RB3_ALLOC(bits, &c, nw * sizeof(uint64_t));
    RB3_ALLOC(wcnt, &c, (nw + 1) * sizeof(uint32_t));
    RB3_ALLOC(tot, &c, 4 * sizeof(uint32_t));
    RB3_LAUNCH("cdc_mark", k_cdc_mark, grid_for(nw, 256, 1 << 16), dim3(256), 0, c.stream, d_Q, nw,
               bits.as<uint64_t>(), wcnt.as<uint32_t>());
    RB3_TRY(scan_u32(c, wcnt.as<uint32_t>(), wcnt.as<uint32_t>(), nw, false, false, tot.as<uint32_t>()));
    uint32_t h[2] = {0, 0};
    RB3_HIP(hipMemcpyAsync(&h[0], tot.p, sizeof(uint32_t), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipStreamSynchronize(c.stream));
    const int64_t ncand = h[0];
    if (ncand < 1) {
        set_error(RB3_EDEVICE, "chunking: no strand start found");
        return RB3_EDEVICE;
    }
    RB3_ALLOC(cpos, &c, ncand * sizeof(uint32_t));
    RB3_LAUNCH("cdc_list", k_cdc_list, grid_for(nw, 256, 1 << 16), dim3(256), 0, c.stream, bits.as<uint64_t>(),
               wcnt.as<uint32_t>(), nw, cpos.as<uint32_t>());
    bits.reset();
    RB3_ALLOC(aflag, &c, (ncand + 1) * sizeof(uint32_t));
    RB3_LAUNCH("cdc_anchor", k_cdc_anchor, grid_for(ncand, 256, 1 << 16), dim3(256), 0, c.stream, d_Q,
               cpos.as<uint32_t>(), ncand, (uint32_t)(lmax / 2 < CDC_GAP ? lmax / 2 : CDC_GAP),
               aflag.as<uint32_t>());
    RB3_ALLOC(aoff, &c, (ncand + 1) * sizeof(uint32_t));
    RB3_TRY(scan_u32(c, aflag.as<uint32_t>(), aoff.as<uint32_t>(), ncand, false, false, tot.as<uint32_t>()));
    RB3_HIP(hipMemcpyAsync(&h[0], tot.p, sizeof(uint32_t), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipStreamSynchronize(c.stream));
    const int64_t nanch = h[0];
    RB3_ALLOC(alist, &c, (nanch + 1) * sizeof(uint32_t));
    RB3_LAUNCH("cdc_alist", k_cdc_alist, grid_for(ncand, 256, 1 << 16), dim3(256), 0, c.stream,
               aflag.as<uint32_t>(), aoff.as<uint32_t>(), ncand, alist.as<uint32_t>());
    RB3_ALLOC(npc, &c, (nanch + 1) * sizeof(uint32_t));
    RB3_LAUNCH("cdc_count", k_cdc_pieces<false>, grid_for(nanch, 256, 1 << 16), dim3(256), 0, c.stream, d_Q, n2,
               cpos.as<uint32_t>(), ncand, alist.as<uint32_t>(), nanch, lmax, npc.as<uint32_t>(), nullptr,
               nullptr, nullptr);
    RB3_HIP(hipMemsetAsync(npc.as<uint32_t>() + nanch, 0, sizeof(uint32_t), c.stream));
    RB3_TRY(scan_u32(c, npc.as<uint32_t>(), npc.as<uint32_t>(), nanch + 1, false, false, tot.as<uint32_t>()));
    RB3_HIP(hipMemcpyAsync(&h[0], tot.p, sizeof(uint32_t), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipStreamSynchronize(c.stream));
    const int64_t nch = h[0];
    DBuf keys, ka, va, kb, vb;
    RB3_ALLOC(chunks, &c, nch * sizeof(Chunk));
    RB3_ALLOC(keys, &c, nch * sizeof(uint64_t));
    RB3_LAUNCH("cdc_pieces", k_cdc_pieces<true>, grid_for(nanch, 256, 1 << 16), dim3(256), 0, c.stream, d_Q, n2,
               cpos.as<uint32_t>(), ncand, alist.as<uint32_t>(), nanch, lmax, nullptr, npc.as<uint32_t>(),
               chunks.as<Chunk>(), keys.as<uint64_t>());
    RB3_ALLOC(ka, &c, nch * sizeof(uint64_t));
    RB3_ALLOC(kb, &c, nch * sizeof(uint64_t));
    RB3_ALLOC(va, &c, nch * sizeof(uint32_t));
    RB3_ALLOC(vb, &c, nch * sizeof(uint32_t));
    uint64_t *sk = nullptr;
    uint32_t *sv = nullptr;
    RB3_TRY(radix_sort(c, keys.as<uint64_t>(), nullptr, ka.as<uint64_t>(), va.as<uint32_t>(), kb.as<uint64_t>(),
                       vb.as<uint32_t>(), nch, 0, 25, true, &sk, &sv, d_guard, nullptr));
    // keep the buffer the sorted order landed in
    if (sv == va.as<uint32_t>()) {
        perm.reset();
        perm.ctx = &c;
        perm.p = va.release();
        perm.bytes = nch * sizeof(uint32_t);
    } else {
        perm.reset();
        perm.ctx = &c;
        perm.p = vb.release();
        perm.bytes = nch * sizeof(uint32_t);
    }
    *nch_out = nch;
    return RB3_OK;
}

}  // namespace rb3
