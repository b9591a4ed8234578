// Merging new strings into a device-resident BWT (Sec. 2.2, Algorithm 1).
//
// Algorithm 1 walks each new string right to left, keeping l = the number of
// suffixes of the existing BWT B1 that are smaller than the current suffix
// (l starts at m1 for the sentinel, then l <- pi_B1(a, l)), and adds the row
// of the suffix among the new suffixes, which it reads from the partial BWT
// B2 of the batch. Here:
//
//   1. LF chains (k_chain, k_fixup). The walk is cut into chunks so that
//      thousands of lanes run at once. A chunk whose right end is not the
//      sentinel starts from the closed range [m1, n1] of possible l values
//      and maps both ends through the monotone l -> pi(a, l); once they meet,
//      the value is exact whatever the true start was. The positions walked
//      before that are completed from the right neighbour's exact value by
//      a fix-up pass, from records the chain leaves (no index reads while
//      the interval spans at most 64 rows).
//   2. Order among the new suffixes without building B2. For new suffixes x,
//      y: l(x) < l(y) implies x < y, and when l(x) = l(y) the order is the
//      plain string order. So the new suffixes are radix-sorted by the key
//      (l, first w symbols). Inside a group of equal keys only members with
//      different BWT symbols need an order (the group's rows record only the
//      symbols): those groups are ordered by comparing the following
//      symbols, by kernels chosen by group size (k_tie_*), and only groups
//      of more than 8192 members fall back to prefix doubling on the key
//      sequence (k_gather, then k_rerank by direct counting within groups of
//      up to 2048 members, or a radix sort of the active records by (group,
//      key) when a group is larger). Sentinel suffixes are unique and sort
//      by strand index.
//   3. Interleave (k_interleave): the s-th new suffix in sorted order lands
//      on merged row l_s + s, its BWT symbol being the symbol before it; the
//      B1 rows fill the remaining rows in order. Checkpoints are rebuilt.
#include "rb3_internal.h"

#include <mutex>

namespace rb3 {

// Sort key of a new suffix at position p:
//   (l - m1) << lshift | packed(Q[p..p+w)) << 3 | emit
// where packed holds w codes, the first in the most significant place, with
// zeros after the strand's sentinel, and emit = Q[p-1] is the suffix's BWT
// symbol (0 = $ at a strand start). Bits 0..2 are carried but not sorted on.
// A key whose lowest packed code is 0 contains its sentinel: such suffixes
// are unique and ordered by position.
__device__ __forceinline__ uint64_t make_key(int64_t lrel, uint64_t packed, uint32_t emit, int lshift) {
    return ((uint64_t)lrel << lshift) | (packed << 3) | (uint64_t)emit;
}

__device__ __forceinline__ uint64_t pack_ahead(const uint8_t *__restrict__ Q, int64_t p, int w) {
    uint64_t packed = 0;
    for (int t = 0; t < w; ++t) {
        uint32_t c = Q[p + t];
        if (!c) break;
        packed |= (uint64_t)c << (3 * (w - 1 - t));
    }
    return packed;
}


// Rows lo .. lo + 63 of B1 holding symbol a, as a mask (bit j: row lo + j),
// from the block holding lo (BL) and, when two is set, the block after it
// (BH). Rows past the blocks read as 0: a caller only uses rows below the
// interval's high end, which lie in these blocks.
__device__ __forceinline__ uint64_t rows_with(const Block &BL, const Block &BH, bool two, int64_t lo, int a) {
    const uint64_t e0 = plane_match(u64_lo(BL.q0), u64_lo(BL.q1), u64_lo(BL.q2), a);
    const uint64_t e1 = plane_match(u64_hi(BL.q0), u64_hi(BL.q1), u64_hi(BL.q2), a);
    const uint64_t e2 = two ? plane_match(u64_lo(BH.q0), u64_lo(BH.q1), u64_lo(BH.q2), a) : 0ull;
    const int o = (int)(lo & (BLK_SYMS - 1));
    const uint64_t x = o < 64 ? e0 : e1, y = o < 64 ? e1 : e2;
    const int sh = o & 63;
    return sh ? (x >> sh) | (y << (64 - sh)) : x;
}

// Byte x of a 16-byte window held as two words (x in [0, 16)).
__device__ __forceinline__ uint32_t win_byte(uint64_t w0, uint64_t w1, int x) {
    return (uint32_t)((x < 8 ? (w0 >> (8 * x)) : (w1 >> (8 * (x - 8)))) & 0xFFu);
}

constexpr int CH_GROUP = 8;       // steps per group (keys written out per group)
// prefix-doubling rounds whose largest group is at most this large rank by
// direct counting; larger ones sort the active records
constexpr uint32_t TIE_RERANK_DIRECT = 2048;
constexpr int CH_WG = 256;        // threads per workgroup of the chain kernel
constexpr int CH_SB_LDS_MAX = 640;  // superblocks whose rows fit in LDS (5 int64 each)

// A wave's keys (or records) of one group, slot s of a lane holding position
// P - s, written out through LDS: lane L puts its 8 values in order of
// position, then in each store instruction eight consecutive lanes write
// one lane's run of 8 positions (64 bytes, each lane an aligned 8-byte
// word), so an instruction writes 8 whole runs instead of 64 values
// scattered over 64 runs. nvalid (per lane): the slots 0 .. nvalid - 1 hold
// values to write (the others are past the chunk's end, or not records).
// buf: this wave's 64 x 8 words of LDS.
__device__ __forceinline__ void wave_write_group(uint64_t *__restrict__ buf, const uint64_t (&v)[CH_GROUP],
                                                 int64_t P, int nvalid, uint64_t *__restrict__ dst) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int s = 0; s < CH_GROUP; ++s) buf[lane * CH_GROUP + (CH_GROUP - 1 - s)] = v[s];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int k = lane & (CH_GROUP - 1);  // run slot k holds position P_L - 7 + k
#pragma unroll
    for (int r = 0; r < 64 / CH_GROUP; ++r) {
        const int L = CH_GROUP * r + (lane >> 3);
        const int64_t PL = __shfl(P, L);
        const int nv = __shfl(nvalid, L);
        const uint64_t x = buf[L * CH_GROUP + k];
        if (k >= CH_GROUP - nv) dst[PL - (CH_GROUP - 1) + k] = x;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// One lane per chunk. The walk covers the chunk right to left. Until the
// interval [lo, hi] of possible values closes, each step records the
// interval's new low end pi(a, lo) (in K, where the position's key goes
// later) and, when the interval spans at most 64 rows, which of the rows
// lo .. lo + 63 hold the step's symbol a (in M; 0 for a wider interval).
// An exact value l in [lo, hi] then moves to
//   pi(a, l) = pi(a, lo) + #(rows lo .. l - 1 holding a),
// so the fix-up pass completes an unresolved end from the right
// neighbour's exact value with a popcount per position instead of a
// dependent read of the index.
//
// Lane t walks chunk perm[t] (chunk t when perm is null): neighbouring lanes
// get chunks whose walks begin with the same symbols (chunks.hip), so they
// read the same index blocks at the same step. The lanes of a wave step
// together in groups of CH_GROUP steps: a step's key and record go to
// registers (slot s of the group), and the wave writes the group's keys and
// records out together (wave_write_group) and fetches the symbols of its
// next group. Point lanes (value known) and interval lanes (value in
// [lo, hi]) share one step: the block of l or lo is read by every lane, the
// block of hi only by interval lanes. With SB_LDS the superblock rows (the
// int64 counts before each 2^24-symbol superblock) are read from LDS. Merges
// into a non-empty index only: keys hold one symbol (key_syms = 1).
template <bool SB_LDS>
__global__ void __launch_bounds__(CH_WG) k_chain(DevIndex ix, const uint8_t *__restrict__ Q,
                                                 const Chunk *__restrict__ ch, const uint32_t *__restrict__ perm,
                                                 int64_t nch, int64_t m1, uint64_t *__restrict__ K,
                                                 uint64_t *__restrict__ M, int32_t *__restrict__ unres,
                                                 int32_t *__restrict__ ulen, int32_t *__restrict__ nwu,
                                                 unsigned long long *__restrict__ stats) {
    extern __shared__ int64_t sb_lds[];  // SB_LDS: 5 per superblock (A .. N)
    __shared__ uint64_t stage[CH_WG / 64][64 * CH_GROUP];
    if (SB_LDS) {
        const int64_t nsb = num_superblocks(ix.n);
        for (int64_t e = threadIdx.x; e < nsb * 5; e += CH_WG)
            sb_lds[e] = ix.sb[(e / 5) * SB_STRIDE + 1 + (e % 5)];
        __syncthreads();
    }
    uint64_t *buf = stage[threadIdx.x >> 6];
    const int64_t lane = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool live = lane < nch;
    const int64_t i = !live ? 0 : (perm ? (int64_t)perm[lane] : lane);
    Chunk c;
    c.p0 = 0;
    c.len = 0;
    c.last = 1;
    if (live) c = ch[i];
    const int64_t p1 = c.p0 + c.len;
    const int32_t len = c.len;
    bool point = c.last != 0;
    int64_t l = m1, lo = m1, hi = ix.n;
    if (live && c.last) K[p1] = (uint64_t)Q[p1 - 1];  // sentinel suffix: l = m1, no symbols
    const uint64_t *Qw = (const uint64_t *)Q;
    int32_t unresolved = 0, nwide = 0;
    int64_t wide = 0;
    // Each step's block (and the symbol words of each group) is requested at
    // the end of the step before it, so the next group's first loads go out
    // before this group's keys are written: a wait for a load also waits for
    // every store issued before it (one counter covers both on this GPU).
    auto group_words = [&](int32_t t0, uint64_t &w0, uint64_t &w1, int64_t &wb) {
        const int64_t P = p1 - 1 - t0;
        wb = (t0 < len ? (P - CH_GROUP > 0 ? P - CH_GROUP : 0) : 0) >> 3;
        w0 = Qw[wb];
        w1 = Qw[wb + 1];
    };
    // (B1 keeps its old contents when only one block is read: the step
    // selects B0 then, and copying B0 would wait for its load)
    auto step_blocks = [&](bool act, Block &B0, Block &B1) {
        const int64_t x0 = act ? (point ? l : lo) : 0;
        B0 = load_block(ix.blk, x0 >> BLK_SHIFT);
        if (act && !point) B1 = load_block(ix.blk, hi >> BLK_SHIFT);
    };
    uint64_t nw0, nw1;
    int64_t nwb;
    Block NB0, NB1 = {};
    group_words(0, nw0, nw1, nwb);
    step_blocks(0 < len, NB0, NB1);
    for (int32_t t0 = 0; __ballot(t0 < len) != 0; t0 += CH_GROUP) {
        // positions P .. P - 7 of this group need the symbols Q[P - 8 .. P]
        const int64_t P = p1 - 1 - t0;
        const uint64_t w0 = nw0, w1 = nw1;
        const int64_t wb = nwb;
        uint64_t kslot[CH_GROUP], rslot[CH_GROUP];
        int nrec = 0;
#pragma clang loop unroll(full)
        for (int s = 0; s < CH_GROUP; ++s) {
            kslot[s] = 0;
            rslot[s] = 0;
            const bool act = t0 + s < len;
            const int64_t p = P - s;
            const int x = (int)(p - (wb << 3));
            const uint32_t a = act ? win_byte(w0, w1, x) : 1u;
            const uint32_t emit = (act && p > 0) ? win_byte(w0, w1, x - 1) : 0u;
            // the block of l (point) or lo (interval), and of hi (interval)
            const int64_t x0 = act ? (point ? l : lo) : 0;
            const bool two = act && !point;
            const int64_t x1 = two ? hi : x0;
            const int64_t b0 = x0 >> BLK_SHIFT, b1 = x1 >> BLK_SHIFT;
            const Block B0 = NB0;
            const Block B1 = two ? NB1 : NB0;
            int64_t s0, s1;
            if (SB_LDS) {
                s0 = sb_lds[(x0 >> SB_SHIFT) * 5 + (a - 1)];
                s1 = sb_lds[(x1 >> SB_SHIFT) * 5 + (a - 1)];
            } else {
                s0 = ix.sb[(x0 >> SB_SHIFT) * SB_STRIDE + a];
                s1 = two ? ix.sb[(x1 >> SB_SHIFT) * SB_STRIDE + a] : s0;
            }
            const int64_t n0 = s0 + (int64_t)ckpt_field(B0.q3, (int)a - 1) +
                               inblock_count(B0, (int)a, (int)(x0 & (BLK_SYMS - 1)));
            const int64_t n1 = two ? s1 + (int64_t)ckpt_field(B1.q3, (int)a - 1) +
                                         inblock_count(B1, (int)a, (int)(x1 & (BLK_SYMS - 1)))
                                   : n0;
            if (act) {
                if (point) {
                    l = n0;
                    kslot[s] = make_key(l - m1, a, emit, 6);
                } else {
                    if (b1 != b0) ++wide;
                    if (n0 == n1) {
                        point = true;
                        l = n0;
                        kslot[s] = make_key(l - m1, a, emit, 6);
                    } else {
                        ++unresolved;
                        kslot[s] = (uint64_t)n0;
                        const int64_t span = hi - lo;
                        if (span > 64) ++nwide;  // the widths only shrink: these come first
                        rslot[s] = span <= 64 ? rows_with(B0, B1, b1 != b0, lo, (int)a) & low_mask((int)span) : 0ull;
                        nrec = s + 1;  // a chunk's records are its first steps
                    }
                    lo = n0;
                    hi = n1;
                }
            }
            // the next step's loads
            if (s + 1 < CH_GROUP) {
                step_blocks(t0 + s + 1 < len, NB0, NB1);
            } else {
                group_words(t0 + CH_GROUP, nw0, nw1, nwb);
                step_blocks(t0 + CH_GROUP < len, NB0, NB1);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        const int nkey = len - t0 < 0 ? 0 : (len - t0 > CH_GROUP ? CH_GROUP : len - t0);
        wave_write_group(buf, kslot, P, nkey, K);
        if (__ballot(nrec > 0) != 0) wave_write_group(buf, rslot, P, nrec, M);
    }
    if (live) {
        unres[i] = unresolved;
        ulen[i] = unresolved;
        nwu[i] = nwide;
    }
    if (wide) atomicAdd(&stats[1], (unsigned long long)wide);
}

// Steps of a fix-up segment (see k_fix_compose).
constexpr int FIX_SEG = 256;

// After the chains: a chunk's first position is exact (ready) unless the
// whole chunk is unresolved; segn = number of fix-up segments of the chunk.
__global__ void k_chain_join(const Chunk *__restrict__ ch, int64_t nch, const int32_t *__restrict__ unres,
                             const int32_t *__restrict__ nwu, int32_t *__restrict__ ready,
                             uint32_t *__restrict__ segn, unsigned long long *__restrict__ stats) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nch) return;
    const int32_t u = unres[i], nw = nwu[i];
    ready[i] = u < ch[i].len ? 1 : 0;
    segn[i] = u > nw ? (uint32_t)((u - nw + FIX_SEG - 1) / FIX_SEG) : 0u;
    if (u) atomicAdd(&stats[0], (unsigned long long)u);
}

// The fix-up segments, one entry each: the chunk it belongs to.
__global__ void k_seg_list(const uint32_t *__restrict__ segoff, int64_t nch, uint32_t *__restrict__ owner) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nch) return;
    for (uint32_t sg = segoff[i]; sg < segoff[i + 1]; ++sg) owner[sg] = (uint32_t)i;
}

// The fix-up. In chunk i's unresolved end, number the steps t = 0, 1, ...
// from the chunk's right end (position p1 - 1 - t). Step t maps the exact
// value entering it, L_t in [lo_t, hi_t], to L_{t+1} = pi(a, L_t). The first
// nw[i] steps, whose interval spans more than 64 rows, read the index. For
// the others, with d_t = L_t - lo_t,
//   d_{t+1} = f_t(d_t) = popcount(M_t & low_mask(d_t)),
// a non-decreasing map of 0..64 that starts at 0 and rises by at most 1 per
// step of d. Such a map is its mask of rises, and the mask of f_t after g is
// the bits of M_t deposited on the set bits of g's mask. So the steps are cut
// into segments of FIX_SEG: k_fix_compose folds each segment's maps into one
// mask (all segments at once), k_fixup walks each run of chunks through the
// index steps and the segment masks only, recording every segment's entry
// value, and k_fix_keys replays every segment from its entry value, writing
// the keys (all segments at once).

// The r-th set bit of m (r below popcount(m)), as a one-bit mask.
__device__ __forceinline__ uint64_t nth_set_bit(uint64_t m, int r) {
    int pos = 0;
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) {
        const int cnt = __popcll(m & low_mask(sh));
        if (r >= cnt) {
            r -= cnt;
            m >>= sh;
            pos += sh;
        }
    }
    return 1ull << pos;
}

// Bits of src, lowest first, placed on the set bits of mask, lowest first:
// the set bits of mask whose rank r has bit r of src clear are dropped
// (usually none: every occurrence in the interval goes on with the step's
// symbol). Dropping the highest rank first leaves the lower ranks in place.
__device__ __forceinline__ uint64_t deposit_bits(uint64_t src, uint64_t mask) {
    uint64_t drop = ~src & low_mask(__popcll(mask));
    while (drop) {
        const int r = 63 - __clzll((long long)drop);
        mask &= ~nth_set_bit(mask, r);
        drop &= ~(1ull << r);
    }
    return mask;
}

// Word q of an 8-word line held as four 16-byte vectors.
__device__ __forceinline__ uint64_t line_word(const uint4 (&v)[4], int q) {
    const uint4 &x = v[q >> 1];
    return (q & 1) ? ((uint64_t)x.w << 32 | x.z) : ((uint64_t)x.y << 32 | x.x);
}

__device__ __forceinline__ void load_line(const uint64_t *__restrict__ a, int64_t base, uint4 (&v)[4]) {
    const uint4 *src = (const uint4 *)(a + base);
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = src[j];
}

// Segment s of the list folds the masks of its steps, walking the
// 8-position lines of M from the one holding the segment's first position
// down (the next line is requested while the current one is used). Lines
// are read whole: M is padded to a whole line past its end.
__global__ void k_fix_compose(const Chunk *__restrict__ ch, const uint32_t *__restrict__ owner,
                              const uint32_t *__restrict__ segoff, int64_t nseg, const uint64_t *__restrict__ M,
                              const int32_t *__restrict__ ulen, const int32_t *__restrict__ nwu,
                              uint64_t *__restrict__ HS) {
    const int64_t sg = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (sg >= nseg) return;
    const uint32_t i = owner[sg];
    const int64_t k = sg - (int64_t)segoff[i];
    const int32_t u = ulen[i];
    const int64_t t0 = (int64_t)nwu[i] + k * FIX_SEG;
    const int64_t t1 = t0 + FIX_SEG < u ? t0 + FIX_SEG : u;
    const Chunk c = ch[i];
    const int64_t top = c.p0 + c.len - 1;
    const int64_t ps = top - t0, pe = top - (t1 - 1);  // positions ps down to pe
    const int64_t bend = pe >> 3;
    uint4 cur[4], nxt[4];
    load_line(M, (ps >> 3) << 3, cur);
    uint64_t H = ~0ull;  // the identity map
    for (int64_t b = ps >> 3; b >= bend; --b) {
        if (b > bend) load_line(M, (b - 1) << 3, nxt);
        const int64_t base = b << 3;
#pragma unroll
        for (int q = 7; q >= 0; --q) {
            const int64_t p = base + q;
            if (p <= ps && p >= pe) H = p == ps ? line_word(cur, q) : deposit_bits(line_word(cur, q), H);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) cur[j] = nxt[j];
    }
    HS[sg] = H;
}

// Fix-up pass: a chunk with an unresolved end whose right neighbour's first
// position is exact walks its index steps (writing their keys), then the
// segment masks, recording each segment's entry value of d; the
// end of the walk is exact at the chunk's last unresolved position. A chunk
// that was unresolved throughout becomes exact at its first position (its
// key is written here too), so the same lane goes on into its left
// neighbour's unresolved end, and so on: a run of unresolved chunks is
// completed in one pass. (Only this lane writes the chunks of its run: their
// own lanes see a right neighbour that was not ready when the pass began,
// and a run ends at a chunk with an exact first position, so two runs never
// meet.) k_unres_count then counts what is left; the host repeats passes
// while anything is (one pass covers every run: a run's right neighbour is
// exact from the chains).
__global__ void k_fixup(DevIndex ix, const uint8_t *__restrict__ Q, const Chunk *__restrict__ ch,
                        int64_t nch, int64_t m1, int w, uint64_t *__restrict__ K,
                        int32_t *__restrict__ unres, const int32_t *__restrict__ nwu,
                        const uint32_t *__restrict__ segoff, const uint64_t *__restrict__ HS,
                        int32_t *__restrict__ SD, int64_t *__restrict__ EX, const int32_t *__restrict__ ready_in,
                        int32_t *__restrict__ ready_out,
                        unsigned long long *__restrict__ stats, int32_t *__restrict__ guard) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nch) return;
    int32_t u = unres[i];
    if (u == 0) return;
    // an unresolved chunk is never the last of its strand, so i+1 is its
    // right neighbour; its first position must already be exact
    if (!ready_in[i + 1]) return;
    Chunk c = ch[i];
    const int lshift = 3 + 3 * w, wsh = 3 * (w - 1);
    int64_t p1 = c.p0 + c.len;
    // the neighbour's first position: its key, or its value from an earlier pass
    const int64_t ex = EX[i + 1];
    int64_t l = ex >= 0 ? ex : (int64_t)(K[p1] >> lshift) + m1;
    int64_t j = i;
    unsigned long long run = 0;   // chunks completed by this lane
    unsigned long long slow = 0;  // steps that read the index
    bool bad = false;
    for (;;) {
        const int32_t nw = nwu[j];
        uint64_t packed = pack_ahead(Q, p1, w);
        int64_t lo = m1;
        for (int32_t t = 0; t < nw; ++t) {
            const int64_t p = p1 - 1 - t;
            const uint32_t a = Q[p];
            packed = ((uint64_t)a << wsh) | (packed >> 3);
            const int64_t nlo = (int64_t)K[p];
            l = pi_sym(ix, (int)a, l);
            lo = nlo;
            K[p] = make_key(l - m1, packed, p > 0 ? Q[p - 1] : 0u, lshift);
        }
        slow += (unsigned long long)nw;
        if (nw < u) {
            int64_t d = l - lo;
            if (d < 0 || d > 64) {
                bad = true;
                d = d < 0 ? 0 : 64;
            }
            int64_t seg = segoff[j];
            for (int64_t t0 = nw; t0 < u; t0 += FIX_SEG, ++seg) {
                SD[seg] = (int32_t)d;
                d = __popcll(HS[seg] & low_mask((int)d));
            }
            // exact at the last unresolved position p1 - u
            l = (int64_t)K[p1 - u] + d;
            if (l > ix.n) {  // never for consistent records: keeps reads in range
                l = ix.n;
                bad = true;
            }
        }
        unres[j] = 0;
        ++run;
        if (u < c.len) break;
        // chunk j was unresolved throughout: its first position is exact now
        // (its key is written by k_fix_keys; a later pass reads the value here)
        EX[j] = l;
        ready_out[j] = 1;
        if (c.first) break;
        // its left neighbour's end follows
        const int64_t nb = j - 1;
        const int32_t un = unres[nb];
        if (un == 0) break;
        j = nb;
        c = ch[nb];
        p1 = c.p0 + c.len;
        u = un;
    }
    if (bad) atomicOr(guard, GUARD_CHAIN);
    if (slow) atomicAdd(&stats[2], slow);
    atomicMax(&stats[3], run);
}

// Segment s of the list replays its steps from its entry value and writes
// their keys, a whole 8-position line of K at a time where the segment
// covers the line (the next line's records are requested while the current
// one is walked). K and M are padded to a whole line past their end.
__global__ void k_fix_keys(const uint8_t *__restrict__ Q, const Chunk *__restrict__ ch,
                           const uint32_t *__restrict__ owner, const uint32_t *__restrict__ segoff, int64_t nseg,
                           int64_t m1, int w, uint64_t *__restrict__ K, const uint64_t *__restrict__ M,
                           const int32_t *__restrict__ ulen, const int32_t *__restrict__ nwu,
                           const int32_t *__restrict__ SD, int32_t *__restrict__ guard) {
    const int64_t sg = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (sg >= nseg) return;
    const uint32_t i = owner[sg];
    const int64_t k = sg - (int64_t)segoff[i];
    const int32_t u = ulen[i];
    const int64_t t0 = (int64_t)nwu[i] + k * FIX_SEG;
    const int64_t t1 = t0 + FIX_SEG < u ? t0 + FIX_SEG : u;
    const Chunk c = ch[i];
    const int lshift = 3 + 3 * w, wsh = 3 * (w - 1);
    int d = SD[sg];
    if (d < 0 || d > 64) {  // no entry: the fix-up passes did not reach this chunk
        atomicOr(guard, GUARD_CHAIN);
        return;
    }
    const int64_t top = c.p0 + c.len - 1;
    const int64_t ps = top - t0, pe = top - (t1 - 1);  // positions ps down to pe
    const int64_t bend = pe >> 3;
    const uint64_t *Qw = (const uint64_t *)Q;
    uint64_t packed = pack_ahead(Q, ps + 1, w);
    uint4 ck[4], cm[4], nk[4], nm[4];
    load_line(K, (ps >> 3) << 3, ck);
    load_line(M, (ps >> 3) << 3, cm);
    bool bad = false;
    for (int64_t b = ps >> 3; b >= bend; --b) {
        if (b > bend) {
            load_line(K, (b - 1) << 3, nk);
            load_line(M, (b - 1) << 3, nm);
        }
        const int64_t base = b << 3;
        const uint64_t qw = Qw[b], qp = b > 0 ? Qw[b - 1] : 0ull;
        uint64_t kw[8];
#pragma unroll
        for (int q = 7; q >= 0; --q) {
            const int64_t p = base + q;
            kw[q] = 0;
            if (p <= ps && p >= pe) {
                const uint32_t a = (uint32_t)(qw >> (8 * q)) & 0xFFu;
                const uint32_t emit = q ? (uint32_t)(qw >> (8 * (q - 1))) & 0xFFu : (uint32_t)(qp >> 56);
                packed = ((uint64_t)a << wsh) | (packed >> 3);
                const uint64_t mq = line_word(cm, q);
                if (mq == 0ull) bad = true;  // a step of the narrow part always has a mask
                d = __popcll(mq & low_mask(d));
                kw[q] = make_key((int64_t)line_word(ck, q) + d - m1, packed, emit, lshift);
            }
        }
        if (base >= pe && base + 7 <= ps) {
            uint4 *dst = (uint4 *)(K + base);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                dst[j] = make_uint4((uint32_t)kw[2 * j], (uint32_t)(kw[2 * j] >> 32), (uint32_t)kw[2 * j + 1],
                                    (uint32_t)(kw[2 * j + 1] >> 32));
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (base + q <= ps && base + q >= pe) K[base + q] = kw[q];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            ck[j] = nk[j];
            cm[j] = nm[j];
        }
    }
    if (bad) atomicOr(guard, GUARD_CHAIN);
}

// Chunks still holding unresolved positions after a fix-up pass.
__global__ void k_unres_count(const int32_t *__restrict__ unres, int64_t nch, int32_t *__restrict__ left) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const uint64_t m = __ballot(i < nch && unres[i] > 0);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(left, (int32_t)__popcll(m));
}

// Keys for a merge into an empty index: every l is 0.
__global__ void k_build_keys(const uint8_t *__restrict__ Q, int64_t n2, int w, uint64_t *__restrict__ K) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n2;
         p += (int64_t)gridDim.x * blockDim.x) {
        uint64_t packed = pack_ahead(Q, p, w);
        uint32_t emit = p > 0 ? Q[p - 1] : 0u;
        K[p] = (packed << 3) | emit;
    }
}

// ---------------------------------------------------------------------------
// Tie resolution
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool starts_group(const uint64_t *__restrict__ SK, int64_t s) {
    if (s == 0) return true;
    uint64_t k = SK[s] >> 3;
    if ((k & 7) == 0) return true;  // contains its sentinel: unique
    return k != (SK[s - 1] >> 3);
}

__global__ void k_head_flags(const uint64_t *__restrict__ SK, int64_t n, uint32_t *__restrict__ hv) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x)
        hv[s] = starts_group(SK, s) ? (uint32_t)s : 0u;
}

// R[pos] = group head; tied[s] = 1 when the group has two or more members.
__global__ void k_rank_init(const uint64_t *__restrict__ SK, const uint32_t *__restrict__ SV,
                            const uint32_t *__restrict__ head, int64_t n, uint32_t *__restrict__ R,
                            uint32_t *__restrict__ tied) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        uint32_t h = head[s];
        R[SV[s]] = h;
        bool single = (h == (uint32_t)s) && (s + 1 == n || starts_group(SK, s + 1));
        tied[s] = single ? 0u : 1u;
    }
}

__global__ void k_active_init(const uint64_t *__restrict__ SK, const uint32_t *__restrict__ SV,
                              const uint32_t *__restrict__ head, const uint32_t *__restrict__ tied,
                              const uint32_t *__restrict__ idx, int64_t n, uint32_t *__restrict__ apos,
                              uint32_t *__restrict__ ahead, uint32_t *__restrict__ ags,
                              uint32_t *__restrict__ agsz, uint32_t *__restrict__ maxg) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        if (!tied[s]) continue;
        uint32_t i = idx[s], h = head[s];
        uint32_t gs = idx[h];
        apos[i] = SV[s];
        ahead[i] = h;
        ags[i] = gs;
        if (s + 1 == n || starts_group(SK, s + 1)) {
            uint32_t sz = (uint32_t)(s - h + 1);
            agsz[gs] = sz;
            atomicMax(maxg, sz);
        }
    }
}

__global__ void k_gather(const uint32_t *__restrict__ apos, int64_t A, const uint32_t *__restrict__ R,
                         int64_t h, int64_t n2, uint32_t *__restrict__ key2, int32_t *__restrict__ guard) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < A;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t q = (int64_t)apos[i] + h;
        if (q < n2) {
            key2[i] = R[q];
        } else {
            key2[i] = 0;
            atomicOr(guard, GUARD_GATHER);
        }
    }
}

// Refine each group by the rank h positions further on. Groups are
// contiguous in the active list and small, so every member counts the keys
// of its group directly.
__global__ void k_rerank(const uint32_t *__restrict__ apos, const uint32_t *__restrict__ ahead,
                         const uint32_t *__restrict__ ags, const uint32_t *__restrict__ agsz,
                         const uint32_t *__restrict__ key2, int64_t A, uint32_t *__restrict__ R,
                         uint32_t *__restrict__ tpos, uint32_t *__restrict__ thead,
                         uint32_t *__restrict__ tkeep, uint32_t *__restrict__ tsub,
                         uint32_t *__restrict__ teq, int32_t *__restrict__ guard) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < A;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t gs = ags[i];
        if ((int64_t)gs >= A) {
            atomicOr(guard, GUARD_RERANK);
            continue;
        }
        uint32_t sz = agsz[gs], mine = key2[i];
        if ((int64_t)gs + sz > A || (uint32_t)i < gs || (uint32_t)i >= gs + sz) {
            atomicOr(guard, GUARD_RERANK);
            continue;
        }
        uint32_t lt = 0, eq = 0, eqb = 0;
        for (uint32_t j = gs; j < gs + sz; ++j) {
            uint32_t kj = key2[j];
            lt += kj < mine;
            eq += kj == mine;
            eqb += (kj == mine) & (j < (uint32_t)i);
        }
        uint32_t nh = ahead[i] + lt;
        R[apos[i]] = nh;
        uint32_t sidx = gs + lt + eqb;
        tpos[sidx] = apos[i];
        thead[sidx] = nh;
        tkeep[sidx] = eq >= 2 ? 1u : 0u;
        tsub[sidx] = eqb;
        teq[sidx] = eq;
    }
}

// The same refinement for rounds with large groups, in linear work: the
// active records sorted stably by (group start, rank h further on) land
// exactly where k_rerank puts them (group start + smaller keys + equal keys
// before), so each sorted slot s reads its record from SV2[s] and its run of
// equal keys from the run's first slot (rstart, a max-scan of run heads).
__global__ void k_rr_keys(const uint32_t *__restrict__ ags, const uint32_t *__restrict__ key2, int64_t A, int kbits,
                          uint64_t *__restrict__ K2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < A; i += (int64_t)gridDim.x * blockDim.x)
        K2[i] = ((uint64_t)ags[i] << kbits) | (uint64_t)key2[i];
}

__global__ void k_rr_heads(const uint64_t *__restrict__ SK2, int64_t A, uint32_t *__restrict__ hs) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < A; s += (int64_t)gridDim.x * blockDim.x)
        hs[s] = (s == 0 || SK2[s] != SK2[s - 1]) ? (uint32_t)s : 0u;
}

__global__ void k_rr_apply(const uint64_t *__restrict__ SK2, const uint32_t *__restrict__ SV2,
                           const uint32_t *__restrict__ rstart, int64_t A, int kbits,
                           const uint32_t *__restrict__ apos, const uint32_t *__restrict__ ahead,
                           uint32_t *__restrict__ R, uint32_t *__restrict__ tpos, uint32_t *__restrict__ thead,
                           uint32_t *__restrict__ tkeep, uint32_t *__restrict__ tsub, uint32_t *__restrict__ teq,
                           int32_t *__restrict__ guard) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < A; s += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t i = SV2[s], r0 = rstart[s];
        const uint32_t gs = (uint32_t)(SK2[s] >> kbits);
        if ((int64_t)i >= A || r0 > (uint32_t)s || r0 < gs) {
            atomicOr(guard, GUARD_RERANK);
            continue;
        }
        const uint32_t nh = ahead[i] + (r0 - gs);
        R[apos[i]] = nh;
        tpos[s] = apos[i];
        thead[s] = nh;
        tsub[s] = (uint32_t)s - r0;
        const bool tail = s + 1 == A || SK2[s + 1] != SK2[s];
        tkeep[s] = ((uint32_t)s > r0 || !tail) ? 1u : 0u;
        if (tail) teq[r0] = (uint32_t)s - r0 + 1u;  // read at the run's first slot
    }
}

__global__ void k_compact(const uint32_t *__restrict__ tpos, const uint32_t *__restrict__ thead,
                          const uint32_t *__restrict__ tkeep, const uint32_t *__restrict__ tsub,
                          const uint32_t *__restrict__ teq, const uint32_t *__restrict__ nidx, int64_t A,
                          uint32_t *__restrict__ apos, uint32_t *__restrict__ ahead,
                          uint32_t *__restrict__ ags, uint32_t *__restrict__ agsz, uint32_t *__restrict__ maxg,
                          int32_t *__restrict__ guard) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < A;
         s += (int64_t)gridDim.x * blockDim.x) {
        if (!tkeep[s]) continue;
        uint32_t ni = nidx[s];
        if ((int64_t)ni >= A || tsub[s] > ni) {
            atomicOr(guard, GUARD_COMPACT);
            continue;
        }
        apos[ni] = tpos[s];
        ahead[ni] = thead[s];
        ags[ni] = ni - tsub[s];
        if (tsub[s] == 0) {
            agsz[ni] = teq[s];
            atomicMax(maxg, teq[s]);
        }
    }
}

// Move tied records to their final rows: SK[R[pos]] = K[pos].
__global__ void k_place(const uint32_t *__restrict__ SV, const uint32_t *__restrict__ R,
                        const uint64_t *__restrict__ K, int64_t n, uint64_t *__restrict__ SK,
                        uint32_t *__restrict__ PF, int32_t *__restrict__ guard) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        uint32_t p = SV[s];
        if ((int64_t)p >= n) {
            atomicOr(guard, GUARD_PLACE);
            continue;
        }
        uint32_t r = R[p];
        if ((int64_t)r >= n) {
            atomicOr(guard, GUARD_PLACE);
            continue;
        }
        if (r != (uint32_t)s) SK[r] = K[p];
        if (PF) PF[r] = p;
    }
}

// ---------------------------------------------------------------------------
// Tie resolution by symbol-aware refinement
// ---------------------------------------------------------------------------
//
// The suffixes of one tied group occupy consecutive rows of the merged BWT,
// and the rows only record each suffix's BWT symbol (bits 0..2 of its key).
// So the order inside a group matters only between members whose symbols
// differ. k_tie_groups lists the groups whose symbols are not all equal, by
// size; the k_tie_* kernels order each of them by comparing the symbols
// that follow the members, depth by depth (plain string order), and stop
// refining a subgroup as soon as its symbols agree.

// With suffix-array samples a new suffix is sampled when its position in the
// batch is a multiple of the sampling distance or it starts its strand (BWT
// symbol $). Tied suffixes with a sampled member need their exact order even
// when their BWT symbols agree, because the sample lands on its own row.
__device__ __forceinline__ bool sampled_pos(uint32_t p, uint32_t e, int32_t srate) {
    return srate > 0 && (p % (uint32_t)srate == 0u || e == 0u);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t t = __shfl_xor(v, o);
        v = t > v ? t : v;
    }
    return v;
}

// Tied groups, found with coalesced reads: each wave looks at 64 consecutive
// sorted keys (one per lane). Group starts come from a ballot; a group that
// starts and ends inside the window has its size from the next start and
// its mixed-symbol test from a ballot of members whose BWT symbol differs
// from their group leader's. Only the group reaching past the window's end
// is extended by the whole wave. Groups whose members carry different
// symbols are collected per workgroup in LDS, by size class, and flushed to
// one global list of (first sorted index, member count) per class with one
// atomic per class per flush; an entry that finds its LDS list full goes to
// the global list directly.
constexpr int TG_THREADS = 256;
constexpr int TG_CLASSES = 6;
constexpr int TG_WIN = 8;     // 64-key windows per wave per iteration, loaded together
constexpr int TG_LCAP = 256;  // LDS list capacity per class
// class upper bounds: 2 | 3..8 | 9..64 | 65..128 | 129..256 | 257..8192
constexpr uint32_t TG_BOUND[TG_CLASSES] = {2, 8, 64, 128, 256, 8192};

__device__ __forceinline__ int group_class(uint32_t k) {
    return k == 2 ? 0 : (k <= 8 ? 1 : (k <= 64 ? 2 : (k <= 128 ? 3 : (k <= 256 ? 4 : 5))));
}

struct TieLists {
    uint32_t *l[TG_CLASSES];
};

// Number of new suffixes landing in each 128-row output block (the
// interleave's input), counted while the sorted keys pass by: consecutive
// sorted entries land in non-decreasing blocks, so a wave adds one count per
// run of equal blocks in its 64-entry window instead of one per entry. The
// key bits (the rank in the existing index) are all it needs, so the count
// does not wait for the tie kernels, which only reorder equal keys.
__device__ __forceinline__ void count_out_blocks(uint64_t v, int64_t s, bool in, int lane, int64_t m1, int lshift,
                                                 int64_t nblk_out, uint32_t *__restrict__ cnt,
                                                 int32_t *__restrict__ guard) {
    const int64_t b = in ? (((int64_t)(v >> lshift) + m1 + s) >> BLK_SHIFT) : -1;
    const int64_t bprev = __shfl_up(b, 1);
    const bool head = in && (lane == 0 || b != bprev);
    const uint64_t heads = __ballot(head);
    const uint64_t vmask = __ballot(in);
    if (head) {
        const uint64_t above = heads & ~low_mask(lane + 1);
        const int next = above ? __ffsll((unsigned long long)above) - 1 : 64 - __clzll((long long)vmask);
        if (b >= 0 && b < nblk_out) atomicAdd(&cnt[b], (uint32_t)(next - lane));
        else atomicOr(guard, GUARD_INTERLEAVE);
    }
}

template <bool SMP>
__global__ void __launch_bounds__(TG_THREADS) k_tie_groups(const uint64_t *__restrict__ SK,
                                                           const uint32_t *__restrict__ SV, int32_t srate, int64_t n,
                                                           TieLists lists, uint32_t *__restrict__ gstat,
                                                           unsigned long long *__restrict__ tied,
                                                           uint32_t *__restrict__ ghist, int64_t m1, int lshift,
                                                           int64_t nblk_out, uint32_t *__restrict__ bcnt,
                                                           int32_t *__restrict__ guard) {
    const int32_t sr = SMP ? srate : 0;  // 0: the variant without samples
    __shared__ uint32_t lst[TG_CLASSES][TG_LCAP][2];
    __shared__ uint32_t hist[32];
    __shared__ uint32_t lcnt[TG_CLASSES];
    __shared__ uint32_t lbase[TG_CLASSES];
    __shared__ unsigned long long wt[TG_THREADS / 64];
    __shared__ uint32_t wm[TG_THREADS / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x < TG_CLASSES) lcnt[threadIdx.x] = 0;
    if (threadIdx.x < 32) hist[threadIdx.x] = 0;
    __syncthreads();
    uint64_t ntied = 0;
    uint32_t kmax = 0;
    constexpr int64_t TILE = (int64_t)TG_THREADS * TG_WIN;
    const int64_t ntiles = (n + TILE - 1) / TILE;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        // this wave's TG_WIN consecutive windows, all loads in flight at once
        const int64_t wbase = tile * TILE + (int64_t)wv * 64 * TG_WIN;
        // (vw[TG_WIN] is the window after the last one, for the extension test)
        uint64_t vw[TG_WIN + 1];
        uint32_t pw[TG_WIN + 1];  // positions, read only with samples
#pragma unroll
        for (int j = 0; j <= TG_WIN; ++j) {
            const int64_t sj = wbase + (int64_t)j * 64 + lane;
            vw[j] = sj < n ? SK[sj] : ~0ull;
            pw[j] = (sr > 0 && sj < n) ? SV[sj] : 1u;
        }
        uint64_t carry = (wbase > 0 && wbase < n) ? (SK[wbase - 1] >> 3) : ~0ull;  // key before the first window
#pragma unroll
        for (int j = 0; j < TG_WIN; ++j) {
            const int64_t w0 = wbase + (int64_t)j * 64;
            const int64_t s = w0 + lane;
            const bool in = s < n;
            const uint64_t v = vw[j];
            count_out_blocks(v, s, in, lane, m1, lshift, nblk_out, bcnt, guard);
            const uint64_t key = v >> 3;
            const uint32_t e = (uint32_t)(v & 7);
            uint64_t prevkey = __shfl_up(key, 1);
            if (lane == 0) prevkey = in ? carry : ~0ull;
            carry = __shfl(key, 63);
            // a key holding its sentinel is unique: always a group of its own
            const bool sent = (key & 7) == 0;
            const bool start = in && (s == 0 || sent || key != prevkey);
            const uint64_t smask = __ballot(start);
            const uint64_t inmask = __ballot(in);
            // leader of my group inside the window (lane of the last start at or below me)
            const uint64_t below = smask & low_mask(lane + 1);
            const int lead = below ? 63 - __clzll((long long)below) : -1;
            const uint32_t le = __shfl(e, lead < 0 ? 0 : lead);
            const bool mism = in && lead >= 0 && (e != le || sampled_pos(pw[j], e, sr));
            const uint64_t mmask = __ballot(mism);
            // the window's last group may run past its end: the whole wave
            // extends it with coalesced 64-key reads of the following windows
            const int last_in = inmask ? 63 - __clzll((long long)inmask) : -1;
            const int ls = smask ? 63 - __clzll((long long)smask) : -1;
            const uint64_t xkey = __shfl(key, ls < 0 ? 0 : ls);
            const uint32_t xe = __shfl(e, ls < 0 ? 0 : ls);
            int64_t ext = 0;
            bool xuni = true;
            if (ls >= 0 && last_in == 63 && (xkey & 7) != 0) {
                // the first following window is already in registers
                uint64_t uv = vw[j + 1];
                uint32_t up = pw[j + 1];
                for (int64_t t = w0 + 64; t < n;) {
                    const uint64_t mm = __ballot((uv >> 3) == xkey);
                    const int run = ~mm ? __ffsll((unsigned long long)~mm) - 1 : 64;
                    const uint32_t ue = (uint32_t)(uv & 7);
                    if (__ballot(lane < run && (ue != xe || sampled_pos(up, ue, sr)))) xuni = false;
                    ext += run;
                    if (run < 64) break;
                    t += 64;
                    uv = t + lane < n ? SK[t + lane] : ~0ull;
                    up = (sr > 0 && t + lane < n) ? SV[t + lane] : 1u;
                }
            }
            if (start && !sent) {
                const uint64_t above = smask & ~low_mask(lane + 1);
                const int ns = above ? __ffsll((unsigned long long)above) - 1 : last_in + 1;
                const int64_t k = (ns - lane) + (above ? 0 : ext);
                const bool uni = (mmask & low_mask(ns) & ~low_mask(lane)) == 0 && (above || xuni);
                if (k >= 2) {
                    ntied += (uint64_t)k;
                    if (!uni) {
                        uint32_t kk = (uint32_t)(k > 0xFFFFFFFFll ? 0xFFFFFFFFll : k);
                        int c = group_class(kk);
                        const uint32_t slot = atomicAdd(&lcnt[c], 1u);
                        if (slot < (uint32_t)TG_LCAP) {
                            lst[c][slot][0] = (uint32_t)s;
                            lst[c][slot][1] = kk;
                        } else {
                            const uint32_t g = atomicAdd(&gstat[c], 1u);
                            lists.l[c][2 * (int64_t)g] = (uint32_t)s;
                            lists.l[c][2 * (int64_t)g + 1] = kk;
                        }
                        atomicAdd(&hist[31 - __clz(kk)], 1u);
                        kmax = kk > kmax ? kk : kmax;
                    }
                }
            }
        }
        __syncthreads();
        // flush a class list once it is half full, and every list after the last tile
        const bool last_tile = tile + gridDim.x >= ntiles;
        for (int c = 0; c < TG_CLASSES; ++c) {
            uint32_t cnt = lcnt[c];
            if (cnt > (uint32_t)TG_LCAP) cnt = TG_LCAP;  // the rest went to the global list
            if (cnt == 0 || (!last_tile && cnt < (uint32_t)TG_LCAP / 2)) continue;
            if (threadIdx.x == 0) lbase[c] = atomicAdd(&gstat[c], cnt);
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < cnt; i += TG_THREADS) {
                lists.l[c][2 * (int64_t)(lbase[c] + i)] = lst[c][i][0];
                lists.l[c][2 * (int64_t)(lbase[c] + i) + 1] = lst[c][i][1];
            }
            __syncthreads();
            if (threadIdx.x == 0) lcnt[c] = 0;
            __syncthreads();
        }
    }
    const uint64_t t = wave_sum_u64(ntied);
    const uint32_t m = wave_max_u32(kmax);
    if (lane == 0) {
        wt[wv] = t;
        wm[wv] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tt = 0;
        uint32_t mm = 0;
        for (int w = 0; w < TG_THREADS / 64; ++w) {
            tt += wt[w];
            mm = wm[w] > mm ? wm[w] : mm;
        }
        if (tt) atomicAdd(tied, tt);
        if (mm) atomicMax(&gstat[TG_CLASSES], mm);
    }
    if (threadIdx.x < 32 && hist[threadIdx.x]) atomicAdd(&ghist[threadIdx.x], hist[threadIdx.x]);
}

// Sixteen symbols of the new strands starting at position q, from the
// batch packed 4 bits per symbol (k_pack_nibbles), the first in the most
// significant nibble, so that unsigned order is lexicographic order.
// Symbols after a sentinel (code 0) belong to the next strand and are
// cleared. QN holds a readable word past the one holding its last symbol.
__device__ __forceinline__ uint64_t load_chunk(const uint64_t *__restrict__ QN, int64_t q) {
    const int64_t j = q >> 4;
    const int sh = (int)(q & 15) * 4;
    uint64_t v = QN[j];
    if (sh) v = (v << sh) | (QN[j + 1] >> (64 - sh));
    // codes are below 8: a nibble is zero iff adding 7 leaves its top bit clear
    const uint64_t t = (v & 0x7777777777777777ull) + 0x7777777777777777ull;
    const uint64_t z = ~(t | v) & 0x8888888888888888ull;
    if (z) v &= ~0ull << (60 - (__clzll((long long)z) & ~3));
    return v;
}

// A chunk holds a sentinel iff it has a zero nibble (symbol codes are 1..5).
__device__ __forceinline__ bool chunk_has_sentinel(uint64_t v) {
    const uint64_t t = (v & 0x7777777777777777ull) + 0x7777777777777777ull;
    return (~(t | v) & 0x8888888888888888ull) != 0;
}

// The batch 4 bits per symbol, 16 symbols per word, the first in the most
// significant nibble; positions past n2 read as 0.
__global__ void k_pack_nibbles(const uint8_t *__restrict__ Q, int64_t n2, int64_t nw, uint64_t *__restrict__ QN) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nw;
         j += (int64_t)gridDim.x * blockDim.x) {
        uint64_t v = 0;
        if (16 * j < n2) {
            // Q is 8-byte aligned with 16 readable bytes past its last symbol
            const uint64_t *w = (const uint64_t *)Q + 2 * j;
            const uint64_t w0 = w[0], w1 = w[1];
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const uint64_t c = ((t < 8 ? w0 >> (8 * t) : w1 >> (8 * (t - 8))) & 0xFull);
                if (16 * j + t < n2) v |= c << (60 - 4 * t);
            }
        }
        QN[j] = v;
    }
}

// The tie kernels below compare suffixes that share their sort key, i.e.
// their insertion rank l and first symbol. Their order is then plain string
// order from the second symbol on, which they read sixteen symbols at a time
// (one chunk, CHUNK_SYMS). Two chunks that are equal and hold a sentinel belong to
// suffixes reaching their strands' ends together: strand order, which is
// position order in Q, decides.
constexpr int CHUNK_SYMS = 16;  // symbols per chunk
constexpr int WALK_DEPTHS = 4;  // chunks per member per load round


constexpr int SMALL_MAXK = 8;
constexpr int SMALL_DEPTHS = 4;
constexpr int LANES_WG = 256;
constexpr int LANES_MAX_DEPTH = 2048;  // symbols

// Groups of 2..8 members, one lane per group, persistent: a lane that has
// ordered its group takes the next one from a shared queue (one atomic per
// wave refill), so no lane idles while a neighbour walks a deep group. The
// queue is the pair list (entries 0..np) followed by the 3..8 list. Members
// are held in registers; every loop over them is unrolled.
template <bool SMP>
__global__ void __launch_bounds__(LANES_WG) k_tie_lanes(const uint64_t *__restrict__ Q, int64_t n2,
                                                        const uint32_t *__restrict__ SV,
                                                        const uint32_t *__restrict__ plist, int64_t np,
                                                        const uint32_t *__restrict__ slist, int64_t ns,
                                                        uint32_t *__restrict__ qhead,
                                                        uint32_t *__restrict__ dlist, uint32_t *__restrict__ dcount,
                                                        uint64_t *__restrict__ SK, uint32_t *__restrict__ PF,
                                                        int32_t srate, int32_t *__restrict__ guard,
                                                        unsigned long long *__restrict__ reads) {
    const int32_t sr = SMP ? srate : 0;  // 0: the variant without samples
    const int lane = threadIdx.x & 63;
    const int64_t total = np + ns;
    uint64_t steps = 0;
    uint32_t maxdepth = 0;
    bool busy = false, exhausted = false;
    uint32_t gs = 0;
    int k = 0;
    int64_t d0 = 1;
    uint32_t pos[SMALL_MAXK], e[SMALL_MAXK], o[SMALL_MAXK], sub[SMALL_MAXK];
    uint64_t gkey = 0;  // the group's common key bits (all but the symbol)
    bool act[SMALL_MAXK];
#pragma unroll
    for (int i = 0; i < SMALL_MAXK; ++i) {
        pos[i] = e[i] = o[i] = sub[i] = 0;
        act[i] = false;
    }
    for (;;) {
        uint64_t idle = __ballot(!busy);
        if (idle && !exhausted) {
            uint32_t nidle = (uint32_t)__popcll(idle);
            uint32_t base = 0;
            if (lane == __ffsll((unsigned long long)idle) - 1) base = atomicAdd(qhead, nidle);
            base = __shfl(base, __ffsll((unsigned long long)idle) - 1);
            if ((int64_t)base + nidle >= total) exhausted = true;
            if (!busy) {
                int64_t slot = (int64_t)base + __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                if (slot < total) {
                    const uint32_t *ent = slot < np ? plist + 2 * slot : slist + 2 * (slot - np);
                    gs = ent[0];
                    k = (int)ent[1];
                    if (k > SMALL_MAXK) {
                        atomicOr(guard, GUARD_RERANK);
                    } else {
                        busy = true;
                        d0 = 1;
#pragma unroll
                        for (int i = 0; i < SMALL_MAXK; ++i) {
                            pos[i] = i < k ? SV[gs + i] : 0u;
                            o[i] = (uint32_t)i;
                            sub[i] = 0;
                            act[i] = i < k;
                        }
#pragma unroll
                        for (int i = 0; i < SMALL_MAXK; ++i) e[i] = i < k ? (uint32_t)(SK[gs + i] & 7) : 0u;
                        gkey = SK[gs] & ~7ull;
                    }
                }
            }
        }
        if (__ballot(busy) == 0) break;
        if (!busy) continue;
        // one batch of depths for this lane's group
        uint64_t kv[SMALL_MAXK][SMALL_DEPTHS];
#pragma unroll
        for (int i = 0; i < SMALL_MAXK; ++i)
#pragma unroll
            for (int t = 0; t < SMALL_DEPTHS; ++t) {
                int64_t q = (int64_t)pos[i] + d0 + CHUNK_SYMS * t;
                kv[i][t] = (act[i] && q < n2) ? load_chunk(Q, q) : ~0ull;
            }
        bool any = true;
#pragma unroll
        for (int t = 0; t < SMALL_DEPTHS; ++t) {
            if (!any) break;
            uint64_t c[SMALL_MAXK];
            uint32_t tb[SMALL_MAXK];
#pragma unroll
            for (int i = 0; i < SMALL_MAXK; ++i) {
                c[i] = kv[i][t];
                tb[i] = 0;
                if (act[i]) {
                    ++steps;
                    if (kv[i][t] == ~0ull) {
                        atomicOr(guard, GUARD_RERANK);
                        act[i] = false;
                    } else if (chunk_has_sentinel(c[i])) {
                        tb[i] = pos[i];  // strand order
                    }
                }
            }
            bool split = false;
#pragma unroll
            for (int i = 0; i < SMALL_MAXK; ++i)
#pragma unroll
                for (int j = i + 1; j < SMALL_MAXK; ++j)
                    split |= act[i] && act[j] && sub[i] == sub[j] && (c[i] != c[j] || tb[i] != tb[j]);
            if (!split) continue;
            uint32_t no[SMALL_MAXK], nsb[SMALL_MAXK];
#pragma unroll
            for (int i = 0; i < SMALL_MAXK; ++i) {
                uint32_t less = 0, eqb = 0;
#pragma unroll
                for (int j = 0; j < SMALL_MAXK; ++j) {
                    bool same = act[i] && act[j] && sub[j] == sub[i];
                    bool lt_ = c[j] < c[i] || (c[j] == c[i] && tb[j] < tb[i]);
                    bool eq_ = c[j] == c[i] && tb[j] == tb[i];
                    less += (same && lt_) ? 1u : 0u;
                    eqb += (same && eq_ && o[j] < o[i]) ? 1u : 0u;
                }
                no[i] = act[i] ? sub[i] + less + eqb : o[i];
                nsb[i] = act[i] ? sub[i] + less : sub[i];
            }
            bool nact[SMALL_MAXK];
            any = false;
#pragma unroll
            for (int i = 0; i < SMALL_MAXK; ++i) {
                uint32_t cnt = 0;
                bool uni = true;
#pragma unroll
                for (int j = 0; j < SMALL_MAXK; ++j) {
                    bool same = act[j] && nsb[j] == nsb[i];
                    cnt += same ? 1u : 0u;
                    uni &= !same || (e[j] == e[i] && !sampled_pos(pos[j], e[j], sr));
                }
                nact[i] = act[i] && cnt >= 2 && !uni;
                any |= nact[i];
            }
#pragma unroll
            for (int i = 0; i < SMALL_MAXK; ++i) {
                o[i] = no[i];
                sub[i] = nsb[i];
                act[i] = nact[i];
            }
        }
        d0 += CHUNK_SYMS * SMALL_DEPTHS;
        if (!any) {
#pragma unroll
            for (int i = 0; i < SMALL_MAXK; ++i)
                if (i < k) {
                    SK[gs + o[i]] = gkey | e[i];
                    if (SMP && PF) PF[gs + o[i]] = pos[i];
                }
            busy = false;
            maxdepth = (uint32_t)d0 > maxdepth ? (uint32_t)d0 : maxdepth;
        }
        // a group still mixed after LANES_MAX_DEPTH goes to the deep walk
        bool evict = busy && d0 > LANES_MAX_DEPTH;
        uint64_t em = __ballot(evict);
        if (em) {
            int first = __ffsll((unsigned long long)em) - 1;
            uint32_t b = 0;
            if (lane == first) b = atomicAdd(dcount, (uint32_t)__popcll(em));
            b = __shfl(b, first);
            if (evict) {
                uint32_t slot = b + __builtin_amdgcn_mbcnt_hi((uint32_t)(em >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)em, 0u));
                dlist[2 * (int64_t)slot] = gs;
                dlist[2 * (int64_t)slot + 1] = (uint32_t)k;
                busy = false;
            }
        }
    }
    uint64_t tot = wave_sum_u64(steps);
    uint32_t md = wave_max_u32(maxdepth);
    if (lane == 0 && tot) atomicAdd(reads, (unsigned long long)tot);
    if (lane == 0 && md) atomicMax((unsigned long long *)reads + 1, (unsigned long long)md);
}


constexpr int DEEP_DPL = 4;  // depths per lane per window

// Groups of 2..8 members whose order needs deep comparisons, one wave each.
// Lane (m, t) = (lane / W, lane % W) loads depths d0 + 4t .. d0 + 4t + 3 of
// member m, W = 64 / (k rounded up to a power of two), so one round trip
// covers 4W depths. The wave finds the first depth where some subgroup
// splits, applies the same refinement as k_tie_lanes there (all lanes keep
// the same copy of the members' state), and goes on from the next depth.
template <bool SMP>
__global__ void __launch_bounds__(256, 4) k_tie_deep(const uint64_t *__restrict__ Q, int64_t n2,
                                                  const uint32_t *__restrict__ SV,
                                                  const uint32_t *__restrict__ dlist,
                                                  const uint32_t *__restrict__ dcount,
                                                  uint64_t *__restrict__ SK, uint32_t *__restrict__ PF,
                                                  int32_t srate, int32_t *__restrict__ guard,
                                                  unsigned long long *__restrict__ reads) {
    const int32_t sr = SMP ? srate : 0;  // 0: the variant without samples
    const int lane = threadIdx.x & 63;
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t nd = *dcount;
    uint64_t steps = 0;
    uint32_t maxdepth = 0;
    for (int64_t g = wave; g < nd; g += nwaves) {
        const uint32_t gs = dlist[2 * g];
        const int k = (int)dlist[2 * g + 1];
        if (k < 2 || k > SMALL_MAXK) {
            if (lane == 0) atomicOr(guard, GUARD_RERANK);
            continue;
        }
        const int kp = k <= 2 ? 2 : (k <= 4 ? 4 : 8);
        const int W = 64 / kp;
        const int mi = lane / W, ti = lane % W;
        uint32_t pos[SMALL_MAXK], e[SMALL_MAXK], o[SMALL_MAXK], sub[SMALL_MAXK], lead[SMALL_MAXK];
        bool act[SMALL_MAXK];
#pragma unroll
        for (int i = 0; i < SMALL_MAXK; ++i) {
            pos[i] = i < k ? SV[gs + i] : 0u;
            o[i] = (uint32_t)i;
            sub[i] = 0;
            lead[i] = 0;
            act[i] = i < k;
        }
#pragma unroll
        for (int i = 0; i < SMALL_MAXK; ++i) e[i] = i < k ? (uint32_t)(SK[gs + i] & 7) : 0u;
        const uint64_t gkey = SK[gs] & ~7ull;
        uint32_t mypos = 0;
        bool myact = false;
#pragma unroll
        for (int i = 0; i < SMALL_MAXK; ++i)
            if (i == mi) {
                mypos = pos[i];
                myact = act[i];
            }
        bool any = true;
        int64_t d0 = 1;
        const int WIN = W * DEEP_DPL;
        while (any) {
            uint64_t kv[DEEP_DPL];
#pragma unroll
            for (int j = 0; j < DEEP_DPL; ++j) {
                int64_t q = (int64_t)mypos + d0 + CHUNK_SYMS * (ti * DEEP_DPL + j);
                kv[j] = (mi < k && myact && q < n2) ? load_chunk(Q, q) : ~0ull;
            }
            int u0 = 0;  // first depth of the window not yet processed
            while (any && u0 < WIN) {
                // my member's leader, and the first depth >= u0 where I differ from it
                uint32_t my_lead = 0, my_sub = 0;
                bool my_act = false;
#pragma unroll
                for (int i = 0; i < SMALL_MAXK; ++i)
                    if (i == mi) {
                        my_lead = lead[i];
                        my_act = act[i];
                        my_sub = sub[i];
                    }
                (void)my_sub;
                int first = WIN;
#pragma unroll
                for (int j = 0; j < DEEP_DPL; ++j) {
                    uint64_t lk = __shfl(kv[j], (int)my_lead * W + ti);
                    int u = ti * DEEP_DPL + j;
                    uint64_t c = kv[j];
                    bool sent = chunk_has_sentinel(c);
                    bool differ = mi < k && my_act && u >= u0 &&
                                  (kv[j] == ~0ull || c != lk || (sent && (uint32_t)mi != my_lead));
                    if (differ && u < first) first = u;
                }
                for (int off = 32; off > 0; off >>= 1) {
                    int t = __shfl_xor(first, off);
                    first = t < first ? t : first;
                }
                if (first >= WIN) break;
                // refine at depth u = first using every member's key there
                const int u = first;
                const int src_t = u / DEEP_DPL, src_j = u % DEEP_DPL;
                uint64_t c[SMALL_MAXK];
                uint32_t tb[SMALL_MAXK];
#pragma unroll
                for (int i = 0; i < SMALL_MAXK; ++i) {
                    uint64_t v = 0;
#pragma unroll
                    for (int j = 0; j < DEEP_DPL; ++j) {
                        uint64_t x = __shfl(kv[j], (i < kp ? i : 0) * W + src_t);
                        if (j == src_j) v = x;
                    }
                    c[i] = v;
                    tb[i] = 0;
                    if (act[i]) {
                        if (v == ~0ull) {
                            if (lane == 0) atomicOr(guard, GUARD_RERANK);
                            act[i] = false;
                        } else if (chunk_has_sentinel(c[i])) {
                            tb[i] = pos[i];
                        }
                    }
                }
                uint32_t no[SMALL_MAXK], nsb[SMALL_MAXK];
#pragma unroll
                for (int i = 0; i < SMALL_MAXK; ++i) {
                    uint32_t less = 0, eqb = 0;
#pragma unroll
                    for (int j = 0; j < SMALL_MAXK; ++j) {
                        bool same = act[i] && act[j] && sub[j] == sub[i];
                        bool lt_ = c[j] < c[i] || (c[j] == c[i] && tb[j] < tb[i]);
                        bool eq_ = c[j] == c[i] && tb[j] == tb[i];
                        less += (same && lt_) ? 1u : 0u;
                        eqb += (same && eq_ && o[j] < o[i]) ? 1u : 0u;
                    }
                    no[i] = act[i] ? sub[i] + less + eqb : o[i];
                    nsb[i] = act[i] ? sub[i] + less : sub[i];
                }
                bool nact[SMALL_MAXK];
                uint32_t nlead[SMALL_MAXK];
                any = false;
#pragma unroll
                for (int i = 0; i < SMALL_MAXK; ++i) {
                    uint32_t cnt = 0, ld = lead[i];
                    bool uni = true;
#pragma unroll
                    for (int j = 0; j < SMALL_MAXK; ++j) {
                        bool same = act[j] && nsb[j] == nsb[i];
                        cnt += same ? 1u : 0u;
                        uni &= !same || (e[j] == e[i] && !sampled_pos(pos[j], e[j], sr));
                        if (same && no[j] == nsb[i]) ld = (uint32_t)j;
                    }
                    nact[i] = act[i] && cnt >= 2 && !uni;
                    nlead[i] = ld;
                    any |= nact[i];
                }
#pragma unroll
                for (int i = 0; i < SMALL_MAXK; ++i) {
                    o[i] = no[i];
                    sub[i] = nsb[i];
                    act[i] = nact[i];
                    lead[i] = nlead[i];
                }
                u0 = u + 1;
            }
            uint32_t na = 0;
#pragma unroll
            for (int i = 0; i < SMALL_MAXK; ++i) na += act[i] ? 1u : 0u;
            steps += (uint64_t)na * WIN;
#pragma unroll
            for (int i = 0; i < SMALL_MAXK; ++i)
                if (i == mi) myact = act[i];
            d0 += CHUNK_SYMS * WIN;
        }
        maxdepth = (uint32_t)d0 > maxdepth ? (uint32_t)d0 : maxdepth;
        if (lane < k) {
            uint32_t oo = 0, ee = 0, pp = 0;
#pragma unroll
            for (int i = 0; i < SMALL_MAXK; ++i)
                if (i == lane) {
                    oo = o[i];
                    ee = e[i];
                    pp = pos[i];
                }
            SK[gs + oo] = gkey | ee;
            if (SMP && PF) PF[gs + oo] = pp;
        }
    }
    if (lane == 0 && steps) atomicAdd(reads, (unsigned long long)steps);
    if (lane == 0 && maxdepth) atomicMax(reads + 1, (unsigned long long)maxdepth);
}

__device__ __forceinline__ uint32_t lane_read(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ uint64_t lane_read64(uint64_t v, int l) {
    return (uint64_t)lane_read((uint32_t)v, l) | ((uint64_t)lane_read((uint32_t)(v >> 32), l) << 32);
}

// One wave per listed group of up to 64 * MPL members; member i lives in
// lane i % 64, slot i / 64, for the whole walk, with its place o in the
// group's current order and the first place of its subgroup. At each depth
// the wave visits the classes of equal (subgroup, chunk) among the members
// of still-mixed subgroups, one class per step, with ballots and lane reads
// only (no LDS): a class that is its whole subgroup changes nothing; a
// class of a subgroup that splits takes consecutive places after the
// members of its subgroup with smaller chunks, and stays mixed if its
// members' symbols differ. The order inside a class is not kept (its
// members are still tied), so member order is used there.
//
// Members of a group share their sort key except for its symbol bits, so
// the symbols come from the group's run of sorted keys (coalesced). The next
// group's members are fetched while the current one is walked.
template <int MPL, bool SMP>
__global__ void __launch_bounds__(256) k_tie_walk(const uint64_t *__restrict__ Q, int64_t n2,
                                                  const uint32_t *__restrict__ SV,
                                                  const uint32_t *__restrict__ glist, int64_t ng,
                                                  uint64_t *__restrict__ SK, uint32_t *__restrict__ PF,
                                                  int32_t srate, int32_t *__restrict__ guard,
                                                  unsigned long long *__restrict__ reads) {
    const int32_t sr = SMP ? srate : 0;  // 0: the variant without samples
    constexpr uint32_t MAXK = 64 * MPL;
    const int lane = threadIdx.x & 63;
    const uint64_t below = low_mask(lane);
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    uint64_t steps = 0;
    uint32_t f_gs = 0, f_k = 0, f_p[MPL];
    uint64_t f_key[MPL];
    auto fetch = [&](int64_t g) {
        f_gs = glist[2 * g];
        f_k = glist[2 * g + 1];
        const bool ok = f_k >= 2 && f_k <= MAXK && (int64_t)f_gs + f_k <= n2;
#pragma unroll
        for (int s = 0; s < MPL; ++s) {
            const uint32_t i = (uint32_t)(s * 64 + lane);
            const bool m = ok && i < f_k;
            f_p[s] = m ? SV[f_gs + i] : 0u;
            f_key[s] = m ? SK[f_gs + i] : 0ull;
        }
    };
#pragma unroll
    for (int s = 0; s < MPL; ++s) {
        f_p[s] = 0;
        f_key[s] = 0;
    }
    if (wave < ng) fetch(wave);
    for (int64_t g = wave; g < ng; g += nwaves) {
        const uint32_t gs = f_gs, k = f_k;
        uint32_t p[MPL], e[MPL], o[MPL], sub[MPL];
        uint64_t key[MPL];
        bool act[MPL];
#pragma unroll
        for (int s = 0; s < MPL; ++s) {
            p[s] = f_p[s];
            key[s] = f_key[s];
        }
        if (g + nwaves < ng) fetch(g + nwaves);
        if (k < 2 || k > MAXK || (int64_t)gs + k > n2) {
            if (lane == 0) atomicOr(guard, GUARD_RERANK);
            continue;
        }
#pragma unroll
        for (int s = 0; s < MPL; ++s) {
            const uint32_t i = (uint32_t)(s * 64 + lane);
            e[s] = (uint32_t)(key[s] & 7);
            o[s] = i;
            sub[s] = 0;
            act[s] = i < k;
        }
        bool past = false;  // a member read past the batch (inconsistent keys): abandon the group
        for (int64_t d0 = 1;; d0 += CHUNK_SYMS * WALK_DEPTHS) {
            if (__ballot(past) != 0) break;
            bool any = false;
#pragma unroll
            for (int s = 0; s < MPL; ++s) any |= __ballot(act[s]) != 0;
            if (!any) break;
            uint64_t kv[MPL][WALK_DEPTHS];
#pragma unroll
            for (int s = 0; s < MPL; ++s)
#pragma unroll
                for (int t = 0; t < WALK_DEPTHS; ++t) {
                    const int64_t q = (int64_t)p[s] + d0 + CHUNK_SYMS * t;
                    kv[s][t] = (act[s] && q < n2) ? load_chunk(Q, q) : ~0ull;
                }
#pragma unroll
            for (int t = 0; t < WALK_DEPTHS; ++t) {
                uint64_t rem[MPL], kk[MPL];
                bool sent[MPL];
                bool left = false;
#pragma unroll
                for (int s = 0; s < MPL; ++s) {
                    kk[s] = act[s] ? kv[s][t] : 0ull;
                    if (act[s]) {
                        ++steps;
                        if (kk[s] == ~0ull) {
                            atomicOr(guard, GUARD_RERANK);
                            past = true;
                        }
                    }
                    sent[s] = act[s] && chunk_has_sentinel(kk[s]);
                    rem[s] = __ballot(act[s]);
                    left |= rem[s] != 0;
                }
                if (!left) break;
                uint32_t no[MPL], nsub[MPL];
                bool nact[MPL];
#pragma unroll
                for (int s = 0; s < MPL; ++s) {
                    no[s] = o[s];
                    nsub[s] = sub[s];
                    nact[s] = act[s];
                }
                for (;;) {
                    int sl = -1;
#pragma unroll
                    for (int s = MPL - 1; s >= 0; --s)
                        if (rem[s]) sl = s;
                    if (sl < 0) break;
                    uint64_t remL = rem[0];
                    uint32_t subR = sub[0], sentR = sent[0] ? 1u : 0u;
                    uint64_t kR = kk[0];
#pragma unroll
                    for (int s = 1; s < MPL; ++s)
                        if (sl == s) {
                            remL = rem[s];
                            subR = sub[s];
                            sentR = sent[s] ? 1u : 0u;
                            kR = kk[s];
                        }
                    const int L = __ffsll((unsigned long long)remL) - 1;
                    const uint32_t subL = lane_read(subR, L);
                    const uint64_t kL = lane_read64(kR, L);
                    const bool sL = lane_read(sentR, L) != 0;
                    uint64_t m[MPL], ins[MPL];
                    bool whole = true;
#pragma unroll
                    for (int s = 0; s < MPL; ++s) {
                        const bool same = act[s] && sub[s] == subL;
                        ins[s] = __ballot(same);
                        m[s] = sL ? ((s == sl) ? (1ull << L) : 0ull) : __ballot(same && !sent[s] && kk[s] == kL);
                        whole &= m[s] == ins[s];
                    }
                    if (!whole) {
                        // the subgroup splits here: place this class
                        uint32_t pR = p[0], eR = e[0];
#pragma unroll
                        for (int s = 1; s < MPL; ++s)
                            if (sl == s) {
                                pR = p[s];
                                eR = e[s];
                            }
                        const uint32_t pL = lane_read(pR, L), eL = lane_read(eR, L);
                        uint32_t less = 0, cnt = 0;
                        bool uni = true;
#pragma unroll
                        for (int s = 0; s < MPL; ++s) {
                            const bool same = act[s] && sub[s] == subL;
                            less += (uint32_t)__popcll(
                                __ballot(same && (kk[s] < kL || (kk[s] == kL && sent[s] && p[s] < pL))));
                            cnt += (uint32_t)__popcll(m[s]);
                            uni &= (__ballot(e[s] == eL && !sampled_pos(p[s], e[s], sr)) & m[s]) == m[s];
                        }
                        const uint32_t base = subL + less;
                        uint32_t pre = 0;
#pragma unroll
                        for (int s = 0; s < MPL; ++s) {
                            if ((m[s] >> lane) & 1ull) {
                                no[s] = base + pre + (uint32_t)__popcll(m[s] & below);
                                nsub[s] = base;
                                nact[s] = cnt >= 2 && !uni;
                            }
                            pre += (uint32_t)__popcll(m[s]);
                        }
                    }
#pragma unroll
                    for (int s = 0; s < MPL; ++s) rem[s] &= ~m[s];
                }
#pragma unroll
                for (int s = 0; s < MPL; ++s) {
                    o[s] = no[s];
                    sub[s] = nsub[s];
                    act[s] = nact[s];
                }
            }
        }
#pragma unroll
        for (int s = 0; s < MPL; ++s)
            if ((uint32_t)(s * 64 + lane) < k) {
                SK[gs + o[s]] = key[s];
                if (SMP && PF) PF[gs + o[s]] = p[s];
            }
    }
    const uint64_t tot = wave_sum_u64(steps);
    if (lane == 0 && tot) atomicAdd(reads, (unsigned long long)tot);
}

// Groups of more than 64 members (up to T * MPT), one workgroup each. The
// members' state lives in LDS, indexed by each member's place in the
// group's current order; a subgroup is a run of places [S, S + size) whose
// members are known equal so far. Every round loads DEPTHS chunks of each
// member of a still-mixed subgroup; at each depth the workgroup checks whether
// some subgroup splits, and if so ranks every member inside its subgroup
// (stable, by chunk, sentinel chunks by strand order), moves the members to
// their new places, measures the new subgroups and keeps only those whose
// members carry different symbols. A split moves members, so the round ends
// there and the next one loads from the following depth.
//
// Ranking inside subgroups. Near-identical members split a few at a time:
// when at most TB_MINOR members hold a chunk other than their subgroup
// head's, each member counts only those (the head's chunk holds no
// sentinel, so its members keep their place order). Otherwise, while every
// mixed subgroup has at most TB_SORT_MIN members, each member counts the
// members of its subgroup that go before it; a larger one (which would
// cost the square of its size) makes the workgroup sort all places by
// (subgroup, chunk, strand position for sentinel chunks or else place)
// with a bitonic network over an index array, and a member's new subgroup
// starts at the first place holding its chunk, found by binary search.
constexpr int TB_SORT_MIN = 256;
constexpr int TB_MINOR = 256;

template <int T, int MPT, int DEPTHS, bool SMP>
__global__ void __launch_bounds__(T) k_tie_block(const uint64_t *__restrict__ Q, int64_t n2, const uint32_t *__restrict__ SV,
                                                 const uint32_t *__restrict__ glist, int64_t ng,
                                                 uint64_t *__restrict__ SK, uint32_t *__restrict__ PF,
                                                 int32_t srate, int32_t *__restrict__ guard,
                                                 unsigned long long *__restrict__ stat) {
    const int32_t sr = SMP ? srate : 0;  // 0: the variant without samples
    constexpr int MAXK = T * MPT;
    static_assert(MAXK <= 65535, "places must fit 16 bits");
    __shared__ uint64_t sc[MAXK];   // chunk at the current depth
    __shared__ uint32_t spos[MAXK]; // position of the member in Q
    __shared__ uint16_t ssub[MAXK]; // first place of the member's subgroup
    __shared__ uint16_t ssz[MAXK];  // subgroup size, kept at its first place
    __shared__ uint8_t se[MAXK];    // the member's BWT symbol
    __shared__ uint8_t sact[MAXK];  // the member's subgroup still mixes symbols
    __shared__ uint8_t snew[MAXK];  // per new subgroup: still mixed
    __shared__ int smx, snm, shs;   // largest mixed subgroup, minority count, a head's chunk ends a strand
    __shared__ uint16_t sminor[TB_MINOR];  // places of the minority
    uint16_t *const perm = ssz;     // the sort's index array (sizes are remeasured after it)
    const int tid = threadIdx.x;
    uint64_t reads = 0;
    int64_t maxd = 0;
    for (int64_t g = blockIdx.x; g < ng; g += gridDim.x) {
        const uint32_t gs = glist[2 * g];
        const int k = (int)glist[2 * g + 1];
        if (k < 2 || k > MAXK || (int64_t)gs + k > n2) {
            if (tid == 0) atomicOr(guard, GUARD_RERANK);
            continue;
        }
        const uint64_t gkey = SK[gs] & ~7ull;
        for (int o = tid; o < k; o += T) {
            spos[o] = SV[gs + o];
            se[o] = (uint8_t)(SK[gs + o] & 7);
            ssub[o] = 0;
            sact[o] = 1;
        }
        if (tid == 0) ssz[0] = (uint16_t)k;
        __syncthreads();
        int64_t d0 = 1;
        int past = 0;  // a member read past the batch (inconsistent keys): abandon the group
        for (;;) {
            if (__syncthreads_or(past)) break;
            uint64_t kv[MPT][DEPTHS];
#pragma unroll
            for (int j = 0; j < MPT; ++j) {
                const int o = tid + j * T;
                const bool a = o < k && sact[o];
                const int64_t p = o < k ? (int64_t)spos[o] : 0;
#pragma unroll
                for (int t = 0; t < DEPTHS; ++t) {
                    const int64_t q = p + d0 + CHUNK_SYMS * t;
                    kv[j][t] = a ? (q < n2 ? load_chunk(Q, q) : ~0ull) : 0ull;
                    reads += a ? 1u : 0u;
                }
            }
            int used = DEPTHS;
            bool any = true;
            for (int t = 0; t < DEPTHS; ++t) {
#pragma unroll
                for (int j = 0; j < MPT; ++j) {
                    const int o = tid + j * T;
                    if (o < k && sact[o]) {
                        if (kv[j][t] == ~0ull) {
                            atomicOr(guard, GUARD_RERANK);
                            past = 1;
                        }
                        sc[o] = kv[j][t];
                    }
                }
                __syncthreads();
                int sp = 0;
#pragma unroll
                for (int j = 0; j < MPT; ++j) {
                    const int o = tid + j * T;
                    if (o < k && sact[o]) {
                        const int S = ssub[o];
                        const uint64_t v = sc[o];
                        sp |= (v != sc[S] || (o != S && chunk_has_sentinel(v))) ? 1 : 0;
                    }
                }
                if (!__syncthreads_or(sp)) continue;
                // rank every member of a mixed subgroup inside it: list the
                // members whose chunk differs from their subgroup head's
                // (the minority) and find the largest mixed subgroup
                if (tid == 0) {
                    smx = 0;
                    snm = 0;
                    shs = 0;
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < MPT; ++j) {
                    const int o = tid + j * T;
                    if (o < k && sact[o]) {
                        const int S = ssub[o];
                        if (sc[o] != sc[S]) {
                            const int d = atomicAdd(&snm, 1);
                            if (d < TB_MINOR) sminor[d] = (uint16_t)o;
                        }
                        if (o == S) {
                            atomicMax(&smx, (int)ssz[o]);
                            if (chunk_has_sentinel(sc[o])) shs = 1;
                        }
                    }
                }
                __syncthreads();
                const int nminor = snm;
                const bool byminor = nminor <= TB_MINOR && !shs;
                const bool bysort = !byminor && smx > TB_SORT_MIN;
                uint32_t r_no[MPT], r_sub[MPT], r_pos[MPT];
                uint8_t r_e[MPT], r_a[MPT];
                if (byminor) {
                    // a member's rank: minority members of its subgroup
                    // below it, plus, for a minority member above its
                    // head's chunk, the head's (majority) members; equal
                    // non-sentinel chunks keep their place order
#pragma unroll
                    for (int j = 0; j < MPT; ++j) {
                        const int o = tid + j * T;
                        r_no[j] = r_sub[j] = r_pos[j] = 0;
                        r_e[j] = r_a[j] = 0;
                        if (o < k) {
                            r_pos[j] = spos[o];
                            r_e[j] = se[o];
                            r_a[j] = sact[o];
                            const int S = ssub[o];
                            r_no[j] = (uint32_t)o;
                            r_sub[j] = (uint32_t)S;
                            if (r_a[j]) {
                                const uint64_t v = sc[o], H = sc[S];
                                const bool sv = chunk_has_sentinel(v);
                                uint32_t less = 0, eqb = 0, nm = 0, nmb = 0;
                                for (int q = 0; q < nminor; ++q) {
                                    const int x = sminor[q];
                                    if (ssub[x] != S) continue;
                                    const uint64_t w = sc[x];
                                    ++nm;
                                    nmb += x < o ? 1u : 0u;
                                    less += (w < v || (w == v && sv && spos[x] < r_pos[j])) ? 1u : 0u;
                                    eqb += (w == v && !sv && x < o) ? 1u : 0u;
                                }
                                if (v == H) {
                                    // majority: the minority below it, then the
                                    // majority members at earlier places
                                    eqb = (uint32_t)(o - S) - nmb;
                                } else if (H < v) {
                                    less += (uint32_t)ssz[S] - nm;
                                }
                                r_no[j] = (uint32_t)S + less + eqb;
                                r_sub[j] = (uint32_t)S + less;
                            }
                        }
                    }
                } else if (bysort) {
                    int P = 1;
                    while (P < k) P <<= 1;
                    __syncthreads();  // every thread has read smx and ssz before perm overwrites them
                    for (int i = tid; i < P; i += T) perm[i] = (uint16_t)i;
                    __syncthreads();
                    // key of place a: (subgroup, chunk, strand position of a
                    // sentinel chunk or else the place); places past k last
                    auto gt = [&](int a, int b) -> bool {
                        if (a >= k) return b < k || a > b;
                        if (b >= k) return false;
                        const int sa = ssub[a], sb = ssub[b];
                        if (sa != sb) return sa > sb;
                        const bool act = sact[a];
                        const uint64_t va = act ? sc[a] : 0ull, vb = act ? sc[b] : 0ull;
                        if (va != vb) return va > vb;
                        const bool sent = act && chunk_has_sentinel(va);
                        const uint32_t ta = sent ? spos[a] : (uint32_t)a, tb = sent ? spos[b] : (uint32_t)b;
                        return ta > tb;
                    };
                    for (int size = 2; size <= P; size <<= 1) {
                        for (int stride = size >> 1; stride > 0; stride >>= 1) {
                            for (int i = tid; i < (P >> 1); i += T) {
                                const int lo = (i / stride) * 2 * stride + (i % stride), hi = lo + stride;
                                const int a = perm[lo], b = perm[hi];
                                if (gt(a, b) == ((lo & size) == 0)) {
                                    perm[lo] = (uint16_t)b;
                                    perm[hi] = (uint16_t)a;
                                }
                            }
                            __syncthreads();
                        }
                    }
#pragma unroll
                    for (int j = 0; j < MPT; ++j) {
                        const int i = tid + j * T;  // the new place
                        r_no[j] = r_sub[j] = r_pos[j] = 0;
                        r_e[j] = r_a[j] = 0;
                        if (i < k) {
                            const int o = perm[i];
                            const int S = ssub[o];
                            r_no[j] = (uint32_t)i;
                            r_pos[j] = spos[o];
                            r_e[j] = se[o];
                            r_a[j] = sact[o];
                            r_sub[j] = (uint32_t)S;
                            if (r_a[j]) {
                                const uint64_t v = sc[o];
                                if (chunk_has_sentinel(v)) {
                                    r_sub[j] = (uint32_t)i;
                                } else {
                                    // the first place of the subgroup holding v
                                    int lo = S, hi = i;
                                    while (lo < hi) {
                                        const int mid = (lo + hi) >> 1;
                                        if (sc[perm[mid]] < v)
                                            lo = mid + 1;
                                        else
                                            hi = mid;
                                    }
                                    r_sub[j] = (uint32_t)lo;
                                }
                            }
                        }
                    }
                } else {
#pragma unroll
                for (int j = 0; j < MPT; ++j) {
                    const int o = tid + j * T;
                    r_no[j] = r_sub[j] = r_pos[j] = 0;
                    r_e[j] = r_a[j] = 0;
                    if (o < k) {
                        r_pos[j] = spos[o];
                        r_e[j] = se[o];
                        r_a[j] = sact[o];
                        const int S = ssub[o];
                        if (r_a[j]) {
                            const int size = ssz[S];
                            const uint64_t v = sc[o];
                            const bool sv = chunk_has_sentinel(v);
                            uint32_t less = 0, eqb = 0;
                            for (int x = S; x < S + size; ++x) {
                                const uint64_t w = sc[x];
                                less += (w < v || (w == v && sv && spos[x] < r_pos[j])) ? 1u : 0u;
                                eqb += (w == v && !sv && x < o) ? 1u : 0u;
                            }
                            r_no[j] = (uint32_t)S + less + eqb;
                            r_sub[j] = (uint32_t)S + less;
                        } else {
                            r_no[j] = (uint32_t)o;
                            r_sub[j] = (uint32_t)S;
                        }
                    }
                }
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < MPT; ++j) {
                    const int o = tid + j * T;
                    if (o < k) {
                        const uint32_t no = r_no[j];
                        spos[no] = r_pos[j];
                        se[no] = r_e[j];
                        ssub[no] = (uint16_t)r_sub[j];
                        sact[no] = r_a[j];
                    }
                }
                __syncthreads();
                // measure the new subgroups: each member raises its
                // subgroup's last place and clears its uniform flag when its
                // symbol differs from the first member's or it is sampled
                // (the chunks are reloaded before the next comparison, so
                // their array holds the two counters meanwhile)
                uint32_t *const mlast = reinterpret_cast<uint32_t *>(sc);
                uint32_t *const muni = mlast + MAXK;
#pragma unroll
                for (int j = 0; j < MPT; ++j) {
                    const int o = tid + j * T;
                    if (o < k && sact[o] && ssub[o] == o) {
                        mlast[o] = (uint32_t)o;
                        muni[o] = 1u;
                    }
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < MPT; ++j) {
                    const int o = tid + j * T;
                    if (o < k && sact[o]) {
                        const int S = ssub[o];
                        if (o != S) atomicMax(&mlast[S], (uint32_t)o);
                        if (se[o] != se[S] || sampled_pos(spos[o], se[o], sr)) atomicAnd(&muni[S], 0u);
                    }
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < MPT; ++j) {
                    const int o = tid + j * T;
                    if (o < k && sact[o] && ssub[o] == o) {
                        const uint32_t size = mlast[o] - (uint32_t)o + 1u;
                        ssz[o] = (uint16_t)size;
                        snew[o] = (size >= 2 && !muni[o]) ? 1 : 0;
                    }
                }
                __syncthreads();
                int anyact = 0;
#pragma unroll
                for (int j = 0; j < MPT; ++j) {
                    const int o = tid + j * T;
                    if (o < k && sact[o]) {
                        const uint8_t a = snew[ssub[o]];
                        sact[o] = a;
                        anyact |= a;
                    }
                }
                any = __syncthreads_or(anyact) != 0;
                used = t + 1;
                break;
            }
            if (!any) break;
            d0 += CHUNK_SYMS * used;
        }
        maxd = d0 > maxd ? d0 : maxd;
        // every thread read gkey before the first barrier of this group
        for (int o = tid; o < k; o += T) {
            SK[gs + o] = gkey | se[o];
            if (SMP && PF) PF[gs + o] = spos[o];
        }
        __syncthreads();
    }
    const uint64_t tot = wave_sum_u64(reads);
    if ((tid & 63) == 0 && tot) atomicAdd(&stat[0], (unsigned long long)tot);
    if (tid == 0 && maxd) atomicMax(&stat[1], (unsigned long long)maxd);
}

// ---------------------------------------------------------------------------
// Interleave
// ---------------------------------------------------------------------------

// One wave per 128-row output block. The old rows of a block are a run of
// consecutive B1 rows, held by at most two B1 blocks: their plane words are
// loaded together with the block's sorted entries (and the next block's
// offsets are loaded a block ahead), so one memory latency is paid per block
// instead of three dependent ones; lanes then take their old symbols from
// the loaded words by lane shuffles.
//
// With suffix-array samples (srate > 0) the wave also writes the block's
// sample bits and count: an old row keeps its bit from the existing index
// (lanes 12..15 hold the old blocks' sample words), a new row is sampled
// when its position in the batch is a multiple of srate or starts a strand
// (its BWT symbol is $).
template <bool SMP>
__global__ void __launch_bounds__(256) k_interleave(const uint64_t *__restrict__ b1words, int64_t nblk1,
                                                    const uint64_t *__restrict__ SK,
                                                    const uint32_t *__restrict__ bs, int64_t nout,
                                                    int64_t nblk_out, int64_t n1, int64_t m1, int lshift,
                                                    uint4 *__restrict__ out, int32_t *__restrict__ guard,
                                                    int32_t srate, const uint64_t *__restrict__ orec,
                                                    const uint32_t *__restrict__ PF,
                                                    uint64_t *__restrict__ nbits, uint32_t *__restrict__ ncnt) {
    const int32_t sr = SMP ? srate : 0;  // 0: the variant without samples
    __shared__ uint8_t slot[4][128];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    uint32_t s0n = 0, s1n = 0;
    if (wave < nblk_out) {
        s0n = bs[wave];
        s1n = bs[wave + 1];
    }
    for (int64_t b = wave; b < nblk_out; b += nwaves) {
        const uint32_t s0 = s0n, s1 = s1n;
        if (b + nwaves < nblk_out) {
            s0n = bs[b + nwaves];
            s1n = bs[b + nwaves + 1];
        }
        const int64_t P0 = b << BLK_SHIFT;
        const int64_t i0 = P0 - (int64_t)s0;  // first old row of the block
        const int64_t rows = nout - P0 < 128 ? nout - P0 : 128;
        const int64_t nnew = (int64_t)s1 - (int64_t)s0;
        const int64_t nold = rows - nnew;
        const int64_t ib0 = i0 >> BLK_SHIFT;
        // lane j < 12 holds plane word j % 6 of old block ib0 + j / 6; with
        // samples, lane 12 + j (j < 4) holds sample word j % 2 of old block
        // ib0 + j / 2
        uint64_t wd = 0;
        if (nold > 0 && i0 >= 0 && i0 < n1) {
            if (lane < 12) {
                const int64_t ib = ib0 + lane / 6;
                if (ib <= ((i0 + nold - 1) >> BLK_SHIFT) && ib < nblk1) wd = b1words[ib * 8 + lane % 6];
            } else if (sr > 0 && lane < 16) {
                const int64_t ib = ib0 + ((lane - 12) >> 1);
                if (ib <= ((i0 + nold - 1) >> BLK_SHIFT) && ib < nblk1) wd = orec[ib * SMP_REC + (lane & 1)];
            }
        }
        const uint32_t ka = s0 + (uint32_t)lane, kb = ka + 64u;
        const uint64_t keya = ka < s1 ? SK[ka] : 0ull;
        const uint64_t keyb = kb < s1 ? SK[kb] : 0ull;
        const uint32_t pa = (sr > 0 && ka < s1) ? PF[ka] : 1u;
        const uint32_t pb = (sr > 0 && kb < s1) ? PF[kb] : 1u;
        slot[wv][lane] = 0;
        slot[wv][lane + 64] = 0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (ka < s1) {
            const int64_t M = (int64_t)(keya >> lshift) + m1 + ka;
            const uint32_t ea = (uint32_t)(keya & 7);
            const uint32_t sa = (sr > 0 && (pa % (uint32_t)sr == 0u || ea == 0u)) ? 0x40u : 0u;
            if (M >= P0 && M < P0 + 128) slot[wv][M - P0] = (uint8_t)(0x80u | sa | ea);
            else atomicOr(guard, GUARD_INTERLEAVE);
        }
        if (kb < s1) {
            const int64_t M = (int64_t)(keyb >> lshift) + m1 + kb;
            const uint32_t eb = (uint32_t)(keyb & 7);
            const uint32_t sb = (sr > 0 && (pb % (uint32_t)sr == 0u || eb == 0u)) ? 0x40u : 0u;
            if (M >= P0 && M < P0 + 128) slot[wv][M - P0] = (uint8_t)(0x80u | sb | eb);
            else atomicOr(guard, GUARD_INTERLEAVE);
        }
        if (nnew > 128 && lane == 0) atomicOr(guard, GUARD_INTERLEAVE);  // more entries than rows
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const uint32_t e0 = slot[wv][lane], e1 = slot[wv][lane + 64];
        const uint64_t nm0 = __ballot(e0 & 0x80u), nm1 = __ballot(e1 & 0x80u);
        // old row of each of my two output rows, and where its bits are
        const int64_t ia = i0 + lane - __popcll(nm0 & low_mask(lane));
        const int64_t ib = i0 + 64 + lane - __popcll(nm0) - __popcll(nm1 & low_mask(lane));
        const bool olda = P0 + lane < nout && !(e0 & 0x80u);
        const bool oldb = P0 + 64 + lane < nout && !(e1 & 0x80u);
        const int sela = (int)((ia >> BLK_SHIFT) - ib0), selb = (int)((ib >> BLK_SHIFT) - ib0);
        const bool oka = olda && ia >= 0 && ia < n1 && (sela == 0 || sela == 1);
        const bool okb = oldb && ib >= 0 && ib < n1 && (selb == 0 || selb == 1);
        if ((olda && !oka) || (oldb && !okb)) atomicOr(guard, GUARD_INTERLEAVE);
        const int la = (oka ? sela : 0) * 6 + (int)((ia >> 6) & 1), lb = (okb ? selb : 0) * 6 + (int)((ib >> 6) & 1);
        // shuffles run with every lane active
        const uint64_t a0w = __shfl(wd, la), a1w = __shfl(wd, la + 2), a2w = __shfl(wd, la + 4);
        const uint64_t b0w = __shfl(wd, lb), b1w = __shfl(wd, lb + 2), b2w = __shfl(wd, lb + 4);
        const int ba = (int)(ia & 63), bb = (int)(ib & 63);
        uint32_t c0 = 7, c1 = 7;
        if (P0 + lane < nout) {
            if (e0 & 0x80u) c0 = e0 & 7u;
            else if (oka)
                c0 = (uint32_t)((a0w >> ba) & 1u) | (uint32_t)(((a1w >> ba) & 1u) << 1) |
                     (uint32_t)(((a2w >> ba) & 1u) << 2);
        }
        if (P0 + 64 + lane < nout) {
            if (e1 & 0x80u) c1 = e1 & 7u;
            else if (okb)
                c1 = (uint32_t)((b0w >> bb) & 1u) | (uint32_t)(((b1w >> bb) & 1u) << 1) |
                     (uint32_t)(((b2w >> bb) & 1u) << 2);
        }
        if (sr > 0) {
            // old rows' sample bits, with every lane active for the shuffles
            const uint64_t swa = __shfl(wd, 12 + 2 * (oka ? sela : 0) + (int)((ia >> 6) & 1));
            const uint64_t swb = __shfl(wd, 12 + 2 * (okb ? selb : 0) + (int)((ib >> 6) & 1));
            const bool sma = P0 + lane < nout &&
                             ((e0 & 0x80u) ? (e0 & 0x40u) != 0u : (oka && ((swa >> (ia & 63)) & 1ull)));
            const bool smb = P0 + 64 + lane < nout &&
                             ((e1 & 0x80u) ? (e1 & 0x40u) != 0u : (okb && ((swb >> (ib & 63)) & 1ull)));
            const uint64_t q0 = __ballot(sma), q1 = __ballot(smb);
            if (lane == 0) {
                nbits[2 * b] = q0;
                nbits[2 * b + 1] = q1;
                ncnt[b] = (uint32_t)(__popcll(q0) + __popcll(q1));
            }
        }
        uint64_t a0 = __ballot(c0 & 1), a1 = __ballot(c0 & 2), a2 = __ballot(c0 & 4);
        uint64_t d0 = __ballot(c1 & 1), d1 = __ballot(c1 & 2), d2 = __ballot(c1 & 4);
        uint32_t cnt = 0;
        if (lane < 6)
            cnt = __popcll(plane_match(a0, a1, a2, lane)) + __popcll(plane_match(d0, d1, d2, lane));
        uint32_t lo = 0, hi = 0;
        for (int s = 0; s < 6; ++s) {
            uint32_t v = __shfl(cnt, s);
            if (s < 4) lo |= v << (8 * s);
            else hi |= v << (8 * (s - 4));
        }
        uint4 *dst = out + (b << 2);
        if (lane == 0) dst[0] = make_uint4((uint32_t)a0, (uint32_t)(a0 >> 32), (uint32_t)d0, (uint32_t)(d0 >> 32));
        if (lane == 1) dst[1] = make_uint4((uint32_t)a1, (uint32_t)(a1 >> 32), (uint32_t)d1, (uint32_t)(d1 >> 32));
        if (lane == 2) dst[2] = make_uint4((uint32_t)a2, (uint32_t)(a2 >> 32), (uint32_t)d2, (uint32_t)(d2 >> 32));
        if (lane == 3) dst[3] = make_uint4(lo, hi, 0u, 0u);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// Sample values of the merged index, one wave per 128-row output block with
// a sampled row: the block's new rows are found again from its sorted
// entries; a sampled new row gets (strand, offset) of its position in the
// batch (strands numbered on from sid0; sstart holds the m2 + 1 strand
// starts in the batch), a sampled old row brings the existing index's value
// along. The k-th sampled row of the block goes to nval[nbase[b] + k].
__global__ void __launch_bounds__(256) k_smp_values(const uint64_t *__restrict__ SK, const uint32_t *__restrict__ PF,
                                                    const uint32_t *__restrict__ bs, int64_t nout, int64_t nblk_out,
                                                    int64_t n1, int64_t m1, int lshift,
                                                    const uint64_t *__restrict__ nbits,
                                                    const uint32_t *__restrict__ nbase, int64_t nsmp,
                                                    const uint64_t *__restrict__ orec,
                                                    const uint64_t *__restrict__ oval, int64_t onsmp, int64_t nblk1,
                                                    const int64_t *__restrict__ sstart, int64_t m2, int64_t sid0,
                                                    uint64_t *__restrict__ nval, int32_t *__restrict__ guard) {
    __shared__ uint8_t slot[4][128];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const uint64_t below = low_mask(lane);
    for (int64_t b = wave; b < nblk_out; b += nwaves) {
        const uint64_t w0 = nbits[2 * b], w1 = nbits[2 * b + 1];
        if ((w0 | w1) == 0ull) continue;
        const uint32_t s0 = bs[b], s1 = bs[b + 1];
        const int64_t P0 = b << BLK_SHIFT;
        const int64_t i0 = P0 - (int64_t)s0;
        slot[wv][lane] = 0;
        slot[wv][lane + 64] = 0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (uint32_t k = s0 + (uint32_t)lane; k < s1 && k < s0 + 128u; k += 64u) {
            const int64_t M = (int64_t)(SK[k] >> lshift) + m1 + k;
            if (M >= P0 && M < P0 + 128) slot[wv][M - P0] = (uint8_t)(k - s0 + 1u);
            else atomicOr(guard, GUARD_SAMPLE);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const uint32_t ea = slot[wv][lane], eb = slot[wv][lane + 64];
        const uint64_t na = __ballot(ea != 0u), nb = __ballot(eb != 0u);
        const uint32_t base = nbase[b];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint64_t w = h ? w1 : w0;
            if (!((w >> lane) & 1ull)) continue;
            const int64_t r = P0 + 64 * h + lane;
            const int64_t outi = (int64_t)base + (h ? __popcll(w0) + __popcll(w1 & below) : __popcll(w0 & below));
            const uint32_t e = h ? eb : ea;
            uint64_t v = 0;
            bool ok = outi < nsmp && r < nout;
            if (e) {
                const uint32_t p = PF[s0 + e - 1u];
                int64_t lo = 0, hi = m2;  // sstart[lo] <= p < sstart[hi]
                while (hi - lo > 1) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (sstart[mid] <= (int64_t)p) lo = mid;
                    else hi = mid;
                }
                const int64_t off = (int64_t)p - sstart[lo];
                ok = ok && off >= 0 && (uint64_t)off <= SMP_OFF_MASK;
                v = ((uint64_t)(sid0 + lo) << SMP_ID_SHIFT) | (uint64_t)off;
            } else {
                const int64_t before = h ? __popcll(na) + __popcll(nb & below) : __popcll(na & below);
                const int64_t i = i0 + 64 * h + lane - before;  // old row
                ok = ok && i >= 0 && i < n1 && (i >> BLK_SHIFT) < nblk1;
                if (ok) {
                    int64_t idx = 0;
                    smp_rank_rec(orec, i, &idx);
                    ok = idx < onsmp;
                    if (ok) v = oval[idx];
                }
            }
            if (ok) nval[outi] = v;
            else atomicOr(guard, GUARD_SAMPLE);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// The merged index's sample records: each block's two bit words and the
// number of samples before it.
__global__ void k_smp_pack(const uint64_t *__restrict__ nbits, const uint32_t *__restrict__ nbase, int64_t nblk,
                           uint64_t *__restrict__ rec) {
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nblk;
         b += (int64_t)gridDim.x * blockDim.x) {
        rec[b * SMP_REC] = nbits[2 * b];
        rec[b * SMP_REC + 1] = nbits[2 * b + 1];
        rec[b * SMP_REC + 2] = nbase[b];
        rec[b * SMP_REC + 3] = 0;
    }
}

// Side streams for the tie kernels. The size classes order disjoint groups
// (each kernel reads and writes only its own groups' rows), so their kernels
// may run at the same time: a class of few large groups then fills the CUs
// that a class of many small groups leaves idle in its tail. Two streams per
// device, default priority, created on first use and kept for the process.
constexpr int TIE_SIDE = 2;
static std::mutex g_side_mu;
static hipStream_t g_side[64][TIE_SIDE];

struct TieStreams {
    hipStream_t main;
    hipStream_t s[TIE_SIDE + 1];
    hipEvent_t ev[TIE_SIDE + 1] = {};
    bool joined = true;

    explicit TieStreams(hipStream_t m) : main(m) {
        for (int k = 0; k <= TIE_SIDE; ++k) s[k] = m;
    }
    // Work queued on main so far happens before any work on the side streams.
    int fork(int dev) {
        if (dev < 0 || dev >= 64) return RB3_OK;  // stays on main
        {
            std::lock_guard<std::mutex> g(g_side_mu);
            for (int k = 0; k < TIE_SIDE; ++k)
                if (!g_side[dev][k]) RB3_HIP(hipStreamCreateWithFlags(&g_side[dev][k], hipStreamNonBlocking));
        }
        for (int k = 0; k <= TIE_SIDE; ++k) RB3_HIP(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming));
        RB3_HIP(hipEventRecord(ev[0], main));
        for (int k = 0; k < TIE_SIDE; ++k) {
            RB3_HIP(hipStreamWaitEvent(g_side[dev][k], ev[0], 0));
            s[k + 1] = g_side[dev][k];
        }
        joined = false;
        return RB3_OK;
    }
    // Later work on main waits for everything queued on the side streams.
    int join() {
        if (joined) return RB3_OK;
        joined = true;
        for (int k = 1; k <= TIE_SIDE; ++k) {
            RB3_HIP(hipEventRecord(ev[k], s[k]));
            RB3_HIP(hipStreamWaitEvent(main, ev[k], 0));
        }
        return RB3_OK;
    }
    ~TieStreams() {
        // on an early return the side streams drain before the caller's
        // deferred frees can release their buffers
        if (!joined && join() == RB3_OK) (void)hipStreamSynchronize(main);
        for (int k = 0; k <= TIE_SIDE; ++k)
            if (ev[k]) (void)hipEventDestroy(ev[k]);
    }
};

static int bits_for(int64_t v) {  // bits to hold values 0..v
    int b = 0;
    while (b < 63 && (v >> b) != 0) ++b;
    return b;
}

int merge_into(Ctx &c, IndexData &ix, const uint8_t *d_Q, const int64_t *strand_lens, int64_t m2,
               int64_t n2, uint4 **new_blk, int64_t **new_sb, int64_t new_C[6], MergeStats &st,
               SmpOut *smp) {
    const DevIndex b1 = ix.dev();
    const int64_t n1 = ix.n, m1 = ix.m;
    const int w = n1 == 0 ? 20 : 1;
    const int lbits = n1 == 0 ? 0 : bits_for(n1 - m1);
    const int lshift = 3 + 3 * w;
    const int hi_bit = lshift + lbits;
    st = MergeStats();
    st.n1 = n1;
    st.m1 = m1;
    st.n2 = n2;
    st.m2 = m2;
    st.key_syms = w;
    st.sort_bits = hi_bit - 3;
    if (hi_bit > 64) {
        set_error(RB3_ELIMIT, "index too large for the merge key");
        return RB3_ELIMIT;
    }
    if (ix.ctx.ssa > 0) {
        // at most one sample per multiple of the distance plus one per strand
        if (ix.nsmp + n2 / ix.ctx.ssa + m2 + 1 >= (int64_t)UINT32_MAX) {
            set_error(RB3_ELIMIT, "too many suffix-array samples (raise the sampling distance)");
            return RB3_ELIMIT;
        }
        if (m1 + m2 > SMP_MAX_STRANDS) {
            set_error(RB3_ELIMIT, "too many strands for suffix-array samples");
            return RB3_ELIMIT;
        }
    }

    DBuf K, stats, guardb;
    RB3_ALLOC(K, &c, (n2 + 8) * sizeof(uint64_t));  // (a whole line past the end: the fix-up reads lines)
    RB3_ALLOC(guardb, &c, sizeof(int32_t));
    RB3_HIP(hipMemsetAsync(guardb.p, 0, sizeof(int32_t), c.stream));
    int32_t *guard = guardb.as<int32_t>();
    RB3_ALLOC(stats, &c, 4 * sizeof(unsigned long long));
    RB3_HIP(hipMemsetAsync(stats.p, 0, 4 * sizeof(unsigned long long), c.stream));

    // ---- 1. insertion ranks ----
    if (n1 > 0) {
        // default: at most 2048 positions, doubled while the batch would make
        // more than 2^17 chunks (past that many lanes, random block reads stop
        // gaining throughput, while the unresolved share of each chunk still
        // grows)
        int64_t CL = c.chunk_len;
        if (CL <= 0) CL = tuned_chunk_len(c.device, n1, n2, m2);
        if (CL <= 0) {
            CL = 2048;
            while (CL < (1 << 20) && n2 / CL > (1 << 17)) CL *= 2;
        }
        if (CL > (1 << 30)) CL = 1 << 30;
        if (CL < 16) CL = 16;
        DBuf d_ch, d_perm;
        int64_t nch = 0;
        RB3_TRY(make_chunks(c, d_Q, n2, CL, d_ch, &nch, d_perm, guard));
        st.chunks = nch;
        st.chunk_len = CL;
        st.chain_steps = n2 - m2;
        DBuf unres, ulen, nwu, segn, recm, readyA, readyB, pend;
        RB3_ALLOC(unres, &c, nch * sizeof(int32_t));
        RB3_ALLOC(ulen, &c, nch * sizeof(int32_t));
        RB3_ALLOC(nwu, &c, nch * sizeof(int32_t));
        RB3_ALLOC(segn, &c, (nch + 1) * sizeof(uint32_t));
        RB3_HIP(hipMemsetAsync(segn.p, 0, (nch + 1) * sizeof(uint32_t), c.stream));
        // the chains' records for unresolved positions (with K, which holds
        // their interval low ends until the fix-up writes their keys), padded
        // to a whole line past the end
        RB3_ALLOC(recm, &c, (n2 + 8) * sizeof(uint64_t));
        RB3_ALLOC(readyA, &c, (nch + 1) * sizeof(int32_t));
        RB3_ALLOC(readyB, &c, (nch + 1) * sizeof(int32_t));
        RB3_ALLOC(pend, &c, sizeof(int32_t));
        RB3_HIP(hipMemsetAsync(readyA.p, 0, (nch + 1) * sizeof(int32_t), c.stream));
        // superblock rows in LDS when the table is small enough
        const int64_t nsb1 = num_superblocks(n1);
        const bool sb_lds = nsb1 <= CH_SB_LDS_MAX;
        const size_t sb_bytes = sb_lds ? (size_t)nsb1 * 5 * sizeof(int64_t) : 0;
        if (c.launch_per_string) {
            // the plain form: each new string's chunks (in string order) in a
            // launch of their own
            std::vector<Chunk> hch(nch);
            RB3_HIP(hipMemcpyAsync(hch.data(), d_ch.p, nch * sizeof(Chunk), hipMemcpyDeviceToHost, c.stream));
            RB3_HIP(hipStreamSynchronize(c.stream));
            std::vector<int64_t> first_chunk;
            for (int64_t i = 0; i < nch; ++i)
                if (hch[i].first) first_chunk.push_back(i);
            first_chunk.push_back(nch);
            for (size_t s = 0; s + 1 < first_chunk.size(); ++s) {
                const int64_t f = first_chunk[s], k = first_chunk[s + 1] - f;
                if (sb_lds)
                    RB3_LAUNCH("chain", k_chain<true>, grid_for(k, CH_WG, 1 << 30), dim3(CH_WG), sb_bytes, c.stream,
                               b1, d_Q, d_ch.as<Chunk>() + f, (const uint32_t *)nullptr, k, m1, K.as<uint64_t>(),
                               recm.as<uint64_t>(), unres.as<int32_t>() + f, ulen.as<int32_t>() + f,
                               nwu.as<int32_t>() + f, stats.as<unsigned long long>());
                else
                    RB3_LAUNCH("chain", k_chain<false>, grid_for(k, CH_WG, 1 << 30), dim3(CH_WG), 0, c.stream, b1,
                               d_Q, d_ch.as<Chunk>() + f, (const uint32_t *)nullptr, k, m1, K.as<uint64_t>(),
                               recm.as<uint64_t>(), unres.as<int32_t>() + f, ulen.as<int32_t>() + f,
                               nwu.as<int32_t>() + f, stats.as<unsigned long long>());
            }
        } else {
            if (sb_lds)
                RB3_LAUNCH("chain", k_chain<true>, grid_for(nch, CH_WG, 1 << 30), dim3(CH_WG), sb_bytes, c.stream, b1,
                           d_Q, d_ch.as<Chunk>(), d_perm.as<uint32_t>(), nch, m1, K.as<uint64_t>(),
                           recm.as<uint64_t>(), unres.as<int32_t>(), ulen.as<int32_t>(), nwu.as<int32_t>(),
                           stats.as<unsigned long long>());
            else
                RB3_LAUNCH("chain", k_chain<false>, grid_for(nch, CH_WG, 1 << 30), dim3(CH_WG), 0, c.stream, b1,
                           d_Q, d_ch.as<Chunk>(), d_perm.as<uint32_t>(), nch, m1, K.as<uint64_t>(),
                           recm.as<uint64_t>(), unres.as<int32_t>(), ulen.as<int32_t>(), nwu.as<int32_t>(),
                           stats.as<unsigned long long>());
        }
        RB3_LAUNCH("chain_join", k_chain_join, grid_for(nch, 256, 1 << 30), dim3(256), 0, c.stream,
                   d_ch.as<Chunk>(), nch, unres.as<int32_t>(), nwu.as<int32_t>(), readyA.as<int32_t>(),
                   segn.as<uint32_t>(), stats.as<unsigned long long>());
        // fix-up segments: offsets per chunk (exclusive scan), total at nch
        RB3_TRY(scan_u32(c, segn.as<uint32_t>(), segn.as<uint32_t>(), nch + 1, false, false, nullptr));
        unsigned long long hs[4];
        uint32_t nseg_h = 0;
        RB3_HIP(hipMemcpyAsync(hs, stats.p, sizeof(hs), hipMemcpyDeviceToHost, c.stream));
        RB3_HIP(hipMemcpyAsync(&nseg_h, segn.as<uint32_t>() + nch, sizeof(uint32_t), hipMemcpyDeviceToHost,
                               c.stream));
        RB3_HIP(hipStreamSynchronize(c.stream));
        const int64_t nseg = nseg_h;
        st.fixup_segments = nseg;
        st.fixup_steps = (int64_t)hs[0];
        st.chain_steps += (int64_t)hs[1];
        int32_t *rin = readyA.as<int32_t>(), *rout = readyB.as<int32_t>();
        int64_t passes = 0;
        if (hs[0] > 0) {
            DBuf HS, SD, EX, owner;
            const int64_t ns1 = nseg > 0 ? nseg : 1;
            RB3_ALLOC(HS, &c, ns1 * sizeof(uint64_t));
            RB3_ALLOC(SD, &c, ns1 * sizeof(int32_t));
            RB3_ALLOC(owner, &c, ns1 * sizeof(uint32_t));
            RB3_ALLOC(EX, &c, (nch + 1) * sizeof(int64_t));
            RB3_HIP(hipMemsetAsync(SD.p, 0xFF, ns1 * sizeof(int32_t), c.stream));
            RB3_HIP(hipMemsetAsync(EX.p, 0xFF, (nch + 1) * sizeof(int64_t), c.stream));
            if (nseg > 0) {
                RB3_LAUNCH("fix_list", k_seg_list, grid_for(nch, 256, 1 << 30), dim3(256), 0, c.stream,
                           segn.as<uint32_t>(), nch, owner.as<uint32_t>());
                RB3_LAUNCH("fix_compose", k_fix_compose, grid_for(nseg, 256, 1 << 30), dim3(256), 0, c.stream,
                           d_ch.as<Chunk>(), owner.as<uint32_t>(), segn.as<uint32_t>(), nseg, recm.as<uint64_t>(),
                           ulen.as<int32_t>(), nwu.as<int32_t>(), HS.as<uint64_t>());
            }
            for (;;) {
                RB3_HIP(hipMemcpyAsync(rout, rin, (nch + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                       c.stream));
                RB3_HIP(hipMemsetAsync(pend.p, 0, sizeof(int32_t), c.stream));
                RB3_LAUNCH("chain_fixup", k_fixup, grid_for(nch, 256, 1 << 30), dim3(256), 0, c.stream,
                           b1, d_Q, d_ch.as<Chunk>(), nch, m1, w, K.as<uint64_t>(), unres.as<int32_t>(),
                           nwu.as<int32_t>(), segn.as<uint32_t>(), HS.as<uint64_t>(), SD.as<int32_t>(),
                           EX.as<int64_t>(), rin, rout, stats.as<unsigned long long>(), guard);
                RB3_LAUNCH("chain_left", k_unres_count, grid_for(nch, 256, 1 << 30), dim3(256), 0, c.stream,
                           unres.as<int32_t>(), nch, pend.as<int32_t>());
                int32_t hp = 0;
                RB3_HIP(hipMemcpyAsync(&hp, pend.p, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
                RB3_HIP(hipStreamSynchronize(c.stream));
                ++passes;
                std::swap(rin, rout);
                if (hp == 0) break;
                if (passes > nch + 1) {
                    set_error(RB3_EDEVICE, "chain fix-up did not converge");
                    return RB3_EDEVICE;
                }
            }
            if (nseg > 0)
                RB3_LAUNCH("fix_keys", k_fix_keys, grid_for(nseg, 256, 1 << 30), dim3(256), 0, c.stream, d_Q,
                           d_ch.as<Chunk>(), owner.as<uint32_t>(), segn.as<uint32_t>(), nseg, m1, w,
                           K.as<uint64_t>(), recm.as<uint64_t>(), ulen.as<int32_t>(), nwu.as<int32_t>(),
                           SD.as<int32_t>(), guard);
            RB3_HIP(hipMemcpyAsync(hs, stats.p, sizeof(hs), hipMemcpyDeviceToHost, c.stream));
            RB3_HIP(hipStreamSynchronize(c.stream));
            st.fixup_index_steps = (int64_t)hs[2];
            st.fixup_run_max = (int64_t)hs[3];
        }
        st.fixup_passes = passes;
        // the stream has drained: the records go back to the allocator now
        c.free_now(recm.release());
    } else {
        RB3_LAUNCH("build_keys", k_build_keys, grid_for(n2, 256 * 4), dim3(256), 0, c.stream, d_Q, n2, w,
                   K.as<uint64_t>());
    }

    RB3_TRY(fault_point(1));

    // ---- 2. order of the new suffixes ----
    DBuf ka, va, kb, vb;
    RB3_ALLOC(ka, &c, n2 * sizeof(uint64_t));
    RB3_ALLOC(kb, &c, n2 * sizeof(uint64_t));
    RB3_ALLOC(va, &c, n2 * sizeof(uint32_t));
    RB3_ALLOC(vb, &c, n2 * sizeof(uint32_t));
    uint64_t *SK = nullptr;
    uint32_t *SV = nullptr;
    int packed_sort = 0, sort_passes = 0;
    RB3_TRY(radix_sort(c, K.as<uint64_t>(), nullptr, ka.as<uint64_t>(), va.as<uint32_t>(), kb.as<uint64_t>(),
                       vb.as<uint32_t>(), n2, 3, hi_bit, true, &SK, &SV, guard, &packed_sort, &sort_passes));
    st.sort_packed = packed_sort;
    st.sort_passes = sort_passes;
    RB3_TRY(fault_point(2));
    // free the other buffer pair early
    if (SK == ka.as<uint64_t>()) {
        kb.reset();
        vb.reset();
    } else {
        ka.reset();
        va.reset();
    }
    // With suffix-array samples the interleave needs every new suffix's
    // position in its final order: PF starts as the sorted positions, and
    // the tie kernels write their groups' final order into it.
    const bool samples = ix.ctx.ssa > 0;
    const int32_t srate = samples ? ix.ctx.ssa : 0;
    DBuf pfb;
    uint32_t *PF = nullptr;
    if (samples) {
        RB3_ALLOC(pfb, &c, n2 * sizeof(uint32_t));
        PF = pfb.as<uint32_t>();
        RB3_HIP(hipMemcpyAsync(PF, SV, n2 * sizeof(uint32_t), hipMemcpyDeviceToDevice, c.stream));
    }

    const int64_t nout = n1 + n2;
    const int64_t nblk_out = num_blocks(nout);
    DBuf bcnt;
    RB3_ALLOC(bcnt, &c, (nblk_out + 1) * sizeof(uint32_t));
    RB3_HIP(hipMemsetAsync(bcnt.p, 0, (nblk_out + 1) * sizeof(uint32_t), c.stream));
    bool bcnt_scanned = false;

    // Groups whose members carry different BWT symbols need an order; the
    // tie kernels handle groups of up to 8192 members by size class, prefix
    // doubling (which orders every tie) handles larger ones.
    bool need_doubling = false;
    {
        DBuf lists[TG_CLASSES], gstat, gtied, ghist, gdeep, gblk;
        TieLists tl;
        for (int q = 0; q < TG_CLASSES; ++q) {
            // a class-q group has more than TG_BOUND[q-1] members
            const int64_t minsz = q == 0 ? 2 : (int64_t)TG_BOUND[q - 1] + 1;
            RB3_ALLOC(lists[q], &c, (n2 / minsz + 1) * 2 * sizeof(uint32_t));
            tl.l[q] = lists[q].as<uint32_t>();
        }
        RB3_ALLOC(ghist, &c, 32 * sizeof(uint32_t));
        RB3_ALLOC(gstat, &c, 8 * sizeof(uint32_t));
        RB3_ALLOC(gtied, &c, 4 * sizeof(unsigned long long));
        RB3_ALLOC(gdeep, &c, 2 * sizeof(unsigned long long));
        RB3_ALLOC(gblk, &c, 2 * sizeof(unsigned long long));
        RB3_HIP(hipMemsetAsync(ghist.p, 0, 32 * sizeof(uint32_t), c.stream));
        RB3_HIP(hipMemsetAsync(gstat.p, 0, 8 * sizeof(uint32_t), c.stream));
        RB3_HIP(hipMemsetAsync(gtied.p, 0, 4 * sizeof(unsigned long long), c.stream));
        RB3_HIP(hipMemsetAsync(gdeep.p, 0, 2 * sizeof(unsigned long long), c.stream));
        RB3_HIP(hipMemsetAsync(gblk.p, 0, 2 * sizeof(unsigned long long), c.stream));
        // (the pass over the sorted keys also counts each output block's new rows)
        if (samples)
            RB3_LAUNCH("tie_groups", k_tie_groups<true>, grid_for(n2, TG_THREADS * TG_WIN * 16, 2048), dim3(TG_THREADS), 0,
                       c.stream, SK, SV, srate, n2, tl, gstat.as<uint32_t>(), gtied.as<unsigned long long>(), ghist.as<uint32_t>(),
                       m1, lshift, nblk_out, bcnt.as<uint32_t>(), guard);
        else
            RB3_LAUNCH("tie_groups", k_tie_groups<false>, grid_for(n2, TG_THREADS * TG_WIN * 16, 2048), dim3(TG_THREADS), 0,
                       c.stream, SK, SV, srate, n2, tl, gstat.as<uint32_t>(), gtied.as<unsigned long long>(), ghist.as<uint32_t>(),
                       m1, lshift, nblk_out, bcnt.as<uint32_t>(), guard);
        uint32_t hs2[8];
        unsigned long long ht[4];
        RB3_HIP(hipMemcpyAsync(st.group_hist, ghist.p, sizeof(st.group_hist), hipMemcpyDeviceToHost, c.stream));
        RB3_HIP(hipMemcpyAsync(hs2, gstat.p, sizeof(hs2), hipMemcpyDeviceToHost, c.stream));
        RB3_HIP(hipMemcpyAsync(ht, gtied.p, sizeof(ht), hipMemcpyDeviceToHost, c.stream));
        RB3_HIP(hipStreamSynchronize(c.stream));
        st.tied_records = (int64_t)ht[0];
        st.tie_pairs = hs2[0];
        st.tie_groups = 0;
        for (int q = 0; q < TG_CLASSES; ++q) st.tie_groups += hs2[q];
        st.max_group = hs2[TG_CLASSES];
        if (hs2[TG_CLASSES] > TG_BOUND[TG_CLASSES - 1]) {
            need_doubling = true;
        } else if (st.tie_groups > 0) {
            // the batch 4 bits per symbol for the comparisons (a word past the
            // one holding the last symbol stays readable)
            DBuf qn;
            const int64_t nqw = (n2 >> 4) + 3;
            RB3_ALLOC(qn, &c, nqw * sizeof(uint64_t));
            RB3_LAUNCH("tie_pack", k_pack_nibbles, grid_for(nqw, 256, 1 << 16), dim3(256), 0, c.stream, d_Q, n2, nqw,
                       qn.as<uint64_t>());
            const uint64_t *Qc = qn.as<uint64_t>();
            DBuf qh, dl;
            const int64_t nq = (int64_t)hs2[0] + hs2[1];
            if (nq > 0) {
                RB3_ALLOC(qh, &c, 2 * sizeof(uint32_t));
                RB3_ALLOC(dl, &c, nq * 2 * sizeof(uint32_t));
                RB3_HIP(hipMemsetAsync(qh.p, 0, 2 * sizeof(uint32_t), c.stream));
            }
            // main: 9..64 members; side 1: up to 8 (and their deep part),
            // then 129..256, then 65..128; side 2: 257..8192 (one workgroup
            // a group, the longest-running class on batches with long
            // repeats, so it runs alone)
            TieStreams ts(c.stream);
            RB3_TRY(ts.fork(c.device));
            // the block counts' scan runs beside the side streams' first kernels
            RB3_TRY(scan_u32(c, bcnt.as<uint32_t>(), bcnt.as<uint32_t>(), nblk_out + 1, false, false, nullptr));
            bcnt_scanned = true;
            if (hs2[5] > 0) {
                if (samples)
                    RB3_LAUNCH("tie_block8k", (k_tie_block<1024, 8, 1, true>), grid_for(hs2[5], 1, 256), dim3(1024), 0,
                               ts.s[2], Qc, n2, SV, tl.l[5], (int64_t)hs2[5], SK, PF, srate, guard,
                               gblk.as<unsigned long long>());
                else
                    RB3_LAUNCH("tie_block8k", (k_tie_block<1024, 8, 1, false>), grid_for(hs2[5], 1, 256), dim3(1024), 0,
                               ts.s[2], Qc, n2, SV, tl.l[5], (int64_t)hs2[5], SK, PF, srate, guard,
                               gblk.as<unsigned long long>());
            }
            if (nq > 0) {
                // persistent: enough waves to fill the chip, no more than the work
                int64_t wgs = (nq + LANES_WG - 1) / LANES_WG;
                if (wgs > 2048) wgs = 2048;
                if (samples)
                    RB3_LAUNCH("tie_lanes", k_tie_lanes<true>, dim3((unsigned)wgs), dim3(LANES_WG), 0, ts.s[1],
                               Qc, n2, SV, tl.l[0], (int64_t)hs2[0], tl.l[1], (int64_t)hs2[1],
                               qh.as<uint32_t>(), dl.as<uint32_t>(), qh.as<uint32_t>() + 1, SK, PF, srate, guard,
                               gtied.as<unsigned long long>() + 1);
                else
                    RB3_LAUNCH("tie_lanes", k_tie_lanes<false>, dim3((unsigned)wgs), dim3(LANES_WG), 0, ts.s[1],
                               Qc, n2, SV, tl.l[0], (int64_t)hs2[0], tl.l[1], (int64_t)hs2[1],
                               qh.as<uint32_t>(), dl.as<uint32_t>(), qh.as<uint32_t>() + 1, SK, PF, srate, guard,
                               gtied.as<unsigned long long>() + 1);
            }
            if (hs2[2] > 0) {
                if (samples)
                    RB3_LAUNCH("tie_walk", (k_tie_walk<1, true>), grid_for(hs2[2], 4 * 8, 1 << 20), dim3(256), 0, ts.s[0],
                               Qc, n2, SV, tl.l[2], (int64_t)hs2[2], SK, PF, srate, guard,
                               gtied.as<unsigned long long>() + 3);
                else
                    RB3_LAUNCH("tie_walk", (k_tie_walk<1, false>), grid_for(hs2[2], 4 * 8, 1 << 20), dim3(256), 0, ts.s[0],
                               Qc, n2, SV, tl.l[2], (int64_t)hs2[2], SK, PF, srate, guard,
                               gtied.as<unsigned long long>() + 3);
            }
            if (nq > 0) {
                // the deep list's length stays on the device: a fixed grid loops over it
                if (samples)
                    RB3_LAUNCH("tie_deep", k_tie_deep<true>, dim3(1024), dim3(256), 0, ts.s[1], Qc, n2, SV,
                               dl.as<uint32_t>(), qh.as<uint32_t>() + 1, SK, PF, srate, guard,
                               gdeep.as<unsigned long long>());
                else
                    RB3_LAUNCH("tie_deep", k_tie_deep<false>, dim3(1024), dim3(256), 0, ts.s[1], Qc, n2, SV,
                               dl.as<uint32_t>(), qh.as<uint32_t>() + 1, SK, PF, srate, guard,
                               gdeep.as<unsigned long long>());
            }
            if (hs2[4] > 0) {
                if (samples)
                    RB3_LAUNCH("tie_walk256", (k_tie_walk<4, true>), grid_for(hs2[4], 4 * 8, 1 << 20), dim3(256), 0,
                               ts.s[1], Qc, n2, SV, tl.l[4], (int64_t)hs2[4], SK, PF, srate, guard,
                               gtied.as<unsigned long long>() + 3);
                else
                    RB3_LAUNCH("tie_walk256", (k_tie_walk<4, false>), grid_for(hs2[4], 4 * 8, 1 << 20), dim3(256), 0,
                               ts.s[1], Qc, n2, SV, tl.l[4], (int64_t)hs2[4], SK, PF, srate, guard,
                               gtied.as<unsigned long long>() + 3);
            }
            if (hs2[3] > 0) {
                if (samples)
                    RB3_LAUNCH("tie_walk128", (k_tie_walk<2, true>), grid_for(hs2[3], 4 * 8, 1 << 20), dim3(256), 0,
                               ts.s[1], Qc, n2, SV, tl.l[3], (int64_t)hs2[3], SK, PF, srate, guard,
                               gtied.as<unsigned long long>() + 3);
                else
                    RB3_LAUNCH("tie_walk128", (k_tie_walk<2, false>), grid_for(hs2[3], 4 * 8, 1 << 20), dim3(256), 0,
                               ts.s[1], Qc, n2, SV, tl.l[3], (int64_t)hs2[3], SK, PF, srate, guard,
                               gtied.as<unsigned long long>() + 3);
            }
            RB3_TRY(ts.join());
            unsigned long long hd[2], hb[2];
            RB3_HIP(hipMemcpyAsync(ht, gtied.p, sizeof(ht), hipMemcpyDeviceToHost, c.stream));
            RB3_HIP(hipMemcpyAsync(hd, gdeep.p, sizeof(hd), hipMemcpyDeviceToHost, c.stream));
            RB3_HIP(hipMemcpyAsync(hb, gblk.p, sizeof(hb), hipMemcpyDeviceToHost, c.stream));
            RB3_HIP(hipStreamSynchronize(c.stream));
            st.tie_small_reads = (int64_t)ht[1];
            unsigned long long md = ht[2] > hd[1] ? ht[2] : hd[1];
            md = md > hb[1] ? md : hb[1];
            st.tie_max_depth = (int64_t)md;
            st.tie_deep_reads = (int64_t)hd[0];
            st.tie_work = (int64_t)ht[3];
            st.tie_block_reads = (int64_t)hb[0];
        }
    }
    if (need_doubling) {
        DBuf head, tied, idx, R, cnt;
        RB3_ALLOC(head, &c, n2 * sizeof(uint32_t));
        RB3_ALLOC(tied, &c, n2 * sizeof(uint32_t));
        RB3_ALLOC(idx, &c, n2 * sizeof(uint32_t));
        RB3_ALLOC(R, &c, n2 * sizeof(uint32_t));
        RB3_ALLOC(cnt, &c, 4 * sizeof(uint32_t));
        RB3_HIP(hipMemsetAsync(cnt.p, 0, 4 * sizeof(uint32_t), c.stream));
        dim3 g = grid_for(n2, 256 * 8);
        RB3_LAUNCH("tie_flags", k_head_flags, g, dim3(256), 0, c.stream, SK, n2, head.as<uint32_t>());
        RB3_TRY(scan_u32(c, head.as<uint32_t>(), head.as<uint32_t>(), n2, true, true, nullptr));
        RB3_LAUNCH("tie_rank_init", k_rank_init, g, dim3(256), 0, c.stream, SK, SV, head.as<uint32_t>(), n2,
                   R.as<uint32_t>(), tied.as<uint32_t>());
        uint32_t *d_tot = cnt.as<uint32_t>();
        RB3_TRY(scan_u32(c, tied.as<uint32_t>(), idx.as<uint32_t>(), n2, false, false, d_tot));
        uint32_t h_cnt[4];
        RB3_HIP(hipMemcpyAsync(h_cnt, cnt.p, sizeof(h_cnt), hipMemcpyDeviceToHost, c.stream));
        RB3_HIP(hipStreamSynchronize(c.stream));
        int64_t A = h_cnt[0];
        st.tie_doubling = 1;
        st.tie_work = 0;
        if (A > 0) {
            DBuf apos[2], ahead[2], ags[2], agsz[2], key2, tpos, thead, tkeep, tsub, teq, nidx;
            for (int q = 0; q < 2; ++q) {
                RB3_ALLOC(apos[q], &c, A * sizeof(uint32_t));
                RB3_ALLOC(ahead[q], &c, A * sizeof(uint32_t));
                RB3_ALLOC(ags[q], &c, A * sizeof(uint32_t));
                RB3_ALLOC(agsz[q], &c, A * sizeof(uint32_t));
            }
            RB3_ALLOC(key2, &c, A * sizeof(uint32_t));
            RB3_ALLOC(tpos, &c, A * sizeof(uint32_t));
            RB3_ALLOC(thead, &c, A * sizeof(uint32_t));
            RB3_ALLOC(tkeep, &c, A * sizeof(uint32_t));
            RB3_ALLOC(tsub, &c, A * sizeof(uint32_t));
            RB3_ALLOC(teq, &c, A * sizeof(uint32_t));
            RB3_ALLOC(nidx, &c, A * sizeof(uint32_t));
            RB3_LAUNCH("tie_active_init", k_active_init, g, dim3(256), 0, c.stream, SK, SV, head.as<uint32_t>(),
                       tied.as<uint32_t>(), idx.as<uint32_t>(), n2, apos[0].as<uint32_t>(),
                       ahead[0].as<uint32_t>(), ags[0].as<uint32_t>(), agsz[0].as<uint32_t>(), d_tot + 1);
            RB3_HIP(hipMemcpyAsync(h_cnt, cnt.p, sizeof(h_cnt), hipMemcpyDeviceToHost, c.stream));
            RB3_HIP(hipStreamSynchronize(c.stream));
            uint32_t maxg = h_cnt[1];
            head.reset();
            tied.reset();
            idx.reset();
            int cur = 0;
            int64_t h = w;
            int rounds = 0;
            // rank bits of the keys h further on (ranks are below n2)
            int kbits = 1;
            while (kbits < 32 && ((int64_t)1 << kbits) < n2) ++kbits;
            while (A > 0) {
                dim3 ga = grid_for(A, 256 * 4);
                RB3_LAUNCH("tie_gather", k_gather, ga, dim3(256), 0, c.stream, apos[cur].as<uint32_t>(), A,
                           R.as<uint32_t>(), h, n2, key2.as<uint32_t>(), guard);
                if (maxg <= TIE_RERANK_DIRECT) {
                    // every member counts the keys of its group: work A * group size
                    RB3_LAUNCH("tie_rerank", k_rerank, ga, dim3(256), 0, c.stream, apos[cur].as<uint32_t>(),
                               ahead[cur].as<uint32_t>(), ags[cur].as<uint32_t>(), agsz[cur].as<uint32_t>(),
                               key2.as<uint32_t>(), A, R.as<uint32_t>(), tpos.as<uint32_t>(), thead.as<uint32_t>(),
                               tkeep.as<uint32_t>(), tsub.as<uint32_t>(), teq.as<uint32_t>(), guard);
                } else {
                    // large groups (long runs of one symbol, many identical
                    // strings): sort the active records by (group start, key)
                    int abits = 1;
                    while (abits < 32 && ((int64_t)1 << abits) < A) ++abits;
                    DBuf k2, ka2, kb2, va2, vb2, hs;
                    RB3_ALLOC(k2, &c, A * sizeof(uint64_t));
                    RB3_ALLOC(ka2, &c, A * sizeof(uint64_t));
                    RB3_ALLOC(kb2, &c, A * sizeof(uint64_t));
                    RB3_ALLOC(va2, &c, A * sizeof(uint32_t));
                    RB3_ALLOC(vb2, &c, A * sizeof(uint32_t));
                    RB3_ALLOC(hs, &c, A * sizeof(uint32_t));
                    RB3_LAUNCH("tie_rr_keys", k_rr_keys, ga, dim3(256), 0, c.stream, ags[cur].as<uint32_t>(),
                               key2.as<uint32_t>(), A, kbits, k2.as<uint64_t>());
                    uint64_t *SK2 = nullptr;
                    uint32_t *SV2 = nullptr;
                    RB3_TRY(radix_sort(c, k2.as<uint64_t>(), nullptr, ka2.as<uint64_t>(), va2.as<uint32_t>(),
                                       kb2.as<uint64_t>(), vb2.as<uint32_t>(), A, 0, kbits + abits, true, &SK2, &SV2,
                                       guard, nullptr));
                    RB3_LAUNCH("tie_rr_heads", k_rr_heads, ga, dim3(256), 0, c.stream, SK2, A, hs.as<uint32_t>());
                    RB3_TRY(scan_u32(c, hs.as<uint32_t>(), hs.as<uint32_t>(), A, true, true, nullptr));
                    RB3_LAUNCH("tie_rr_apply", k_rr_apply, ga, dim3(256), 0, c.stream, SK2, SV2, hs.as<uint32_t>(), A,
                               kbits, apos[cur].as<uint32_t>(), ahead[cur].as<uint32_t>(), R.as<uint32_t>(),
                               tpos.as<uint32_t>(), thead.as<uint32_t>(), tkeep.as<uint32_t>(), tsub.as<uint32_t>(),
                               teq.as<uint32_t>(), guard);
                }
                RB3_TRY(scan_u32(c, tkeep.as<uint32_t>(), nidx.as<uint32_t>(), A, false, false, d_tot));
                int nx = cur ^ 1;
                RB3_HIP(hipMemsetAsync(d_tot + 1, 0, sizeof(uint32_t), c.stream));
                RB3_LAUNCH("tie_compact", k_compact, ga, dim3(256), 0, c.stream, tpos.as<uint32_t>(),
                           thead.as<uint32_t>(), tkeep.as<uint32_t>(), tsub.as<uint32_t>(), teq.as<uint32_t>(),
                           nidx.as<uint32_t>(), A, apos[nx].as<uint32_t>(), ahead[nx].as<uint32_t>(),
                           ags[nx].as<uint32_t>(), agsz[nx].as<uint32_t>(), d_tot + 1, guard);
                RB3_HIP(hipMemcpyAsync(h_cnt, cnt.p, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, c.stream));
                RB3_HIP(hipStreamSynchronize(c.stream));
                st.tie_work += A;
                A = h_cnt[0];
                maxg = h_cnt[1];
                cur = nx;
                h *= 2;
                ++rounds;
                if (rounds > 48) {
                    set_error(RB3_EDEVICE, "tie resolution did not terminate");
                    return RB3_EDEVICE;
                }
            }
            st.tie_rounds = rounds;
            RB3_LAUNCH("tie_place", k_place, g, dim3(256), 0, c.stream, SV, R.as<uint32_t>(), K.as<uint64_t>(),
                       n2, SK, PF, guard);
        }
    }

    RB3_TRY(fault_point(3));

    // ---- 3. interleave into the merged BWT ----
    if (!bcnt_scanned)
        RB3_TRY(scan_u32(c, bcnt.as<uint32_t>(), bcnt.as<uint32_t>(), nblk_out + 1, false, false, nullptr));
    DBuf out_blk, out_sb;
    RB3_ALLOC(out_blk, &c, nblk_out * 64);
    RB3_ALLOC(out_sb, &c, num_superblocks(nout) * SB_STRIDE * sizeof(int64_t));
    DBuf sbits, scnt, sval, sst, srec;
    if (samples) {
        RB3_ALLOC(sbits, &c, nblk_out * 2 * sizeof(uint64_t));
        RB3_ALLOC(scnt, &c, (nblk_out + 1) * sizeof(uint32_t));
        RB3_HIP(hipMemsetAsync(sbits.p, 0, nblk_out * 2 * sizeof(uint64_t), c.stream));
        RB3_HIP(hipMemsetAsync(scnt.p, 0, (nblk_out + 1) * sizeof(uint32_t), c.stream));
    }
    if (samples)
        RB3_LAUNCH("interleave", k_interleave<true>, grid_for(nblk_out, 4, 1 << 18), dim3(256), 0, c.stream,
                   (const uint64_t *)b1.blk, num_blocks(n1), SK, bcnt.as<uint32_t>(), nout, nblk_out, n1, m1, lshift,
                   out_blk.as<uint4>(), guard, srate, (const uint64_t *)ix.smp_rec, PF,
                   samples ? sbits.as<uint64_t>() : nullptr, samples ? scnt.as<uint32_t>() : nullptr);
    else
        RB3_LAUNCH("interleave", k_interleave<false>, grid_for(nblk_out, 4, 1 << 18), dim3(256), 0, c.stream,
                   (const uint64_t *)b1.blk, num_blocks(n1), SK, bcnt.as<uint32_t>(), nout, nblk_out, n1, m1, lshift,
                   out_blk.as<uint4>(), guard, srate, (const uint64_t *)ix.smp_rec, PF,
                   samples ? sbits.as<uint64_t>() : nullptr, samples ? scnt.as<uint32_t>() : nullptr);
    RB3_TRY(fault_point(4));
    int64_t nsmp_new = 0;
    if (samples) {
        RB3_TRY(scan_u32(c, scnt.as<uint32_t>(), scnt.as<uint32_t>(), nblk_out + 1, false, false, nullptr));
        uint32_t tot = 0;
        RB3_HIP(hipMemcpyAsync(&tot, scnt.as<uint32_t>() + nblk_out, sizeof(uint32_t), hipMemcpyDeviceToHost,
                               c.stream));
        RB3_HIP(hipStreamSynchronize(c.stream));
        nsmp_new = tot;
        std::vector<int64_t> hst(m2 + 1);
        hst[0] = 0;
        for (int64_t j = 0; j < m2; ++j) hst[j + 1] = hst[j] + strand_lens[j] + 1;
        RB3_ALLOC(sst, &c, (m2 + 1) * sizeof(int64_t));
        RB3_HIP(hipMemcpyAsync(sst.p, hst.data(), (m2 + 1) * sizeof(int64_t), hipMemcpyHostToDevice, c.stream));
        RB3_ALLOC(sval, &c, (nsmp_new > 0 ? nsmp_new : 1) * sizeof(uint64_t));
        RB3_LAUNCH("smp_values", k_smp_values, grid_for(nblk_out, 4, 1 << 18), dim3(256), 0, c.stream, SK, PF,
                   bcnt.as<uint32_t>(), nout, nblk_out, n1, m1, lshift, sbits.as<uint64_t>(), scnt.as<uint32_t>(),
                   nsmp_new, (const uint64_t *)ix.smp_rec,
                   (const uint64_t *)ix.smp_val, ix.nsmp, num_blocks(n1), sst.as<int64_t>(), m2, m1,
                   sval.as<uint64_t>(), guard);
        RB3_ALLOC(srec, &c, nblk_out * SMP_REC * sizeof(uint64_t));
        RB3_LAUNCH("smp_pack", k_smp_pack, grid_for(nblk_out, 256), dim3(256), 0, c.stream, sbits.as<uint64_t>(),
                   scnt.as<uint32_t>(), nblk_out, srec.as<uint64_t>());
    }
    int64_t counts[6];
    RB3_TRY(build_checkpoints(c, out_blk.as<uint4>(), nout, out_sb.as<int64_t>(), new_C, counts));
    RB3_TRY(fault_point(5));
    int32_t hg = 0;
    RB3_HIP(hipMemcpyAsync(&hg, guard, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipStreamSynchronize(c.stream));
    if (hg) {
        set_error(RB3_EDEVICE, "merge: internal consistency guard tripped (mask " + std::to_string(hg) + ")");
        return RB3_EDEVICE;
    }
    if (counts[0] != m1 + m2) {
        set_error(RB3_EDEVICE, "merged BWT has the wrong number of sentinels");
        return RB3_EDEVICE;
    }
    if (samples && smp) {
        smp->rec = srec.as<uint64_t>();
        smp->val = sval.as<uint64_t>();
        smp->nsmp = nsmp_new;
        srec.release();
        sval.release();
    }
    *new_blk = (uint4 *)out_blk.release();
    *new_sb = (int64_t *)out_sb.release();
    return RB3_OK;
}

}  // namespace rb3
