// Local haplotype enumeration (Sec. 2.8): semi-global alignment of each
// query to the prefix DAWG of the index by the revised BWA-SW recurrences
// (Sec. 2.7, Algorithm 5), then the bi-interval redundancy filter.
//
// G_P is the path graph of the query taken from its end; a node of G_T is a
// bi-interval (k, k', s), its children the non-empty backward extensions by
// A, C, G, T (one rank-all pair gives all four). The start cell (query end,
// root [0, n)) has H = 0; every other cell is kept only while H > 0. At each
// query position: match/mismatch and insertion from the previous position's
// cells, then deletion repeated until no cell improves, then the cells with
// H <= 0 are dropped and, with a band W > 0, only the W cells of largest H
// stay (ties: smaller k, then smaller s). The cells left at the query's
// start, by decreasing H (same ties), are the result, except those whose
// interval or reverse-complement interval lies inside the corresponding
// interval of a cell kept before them.
//
// Two kernels. k_hapl_wave gives each query half or all of a wavefront and
// keeps its cells in LDS (below). k_hapl, one thread per query, keeps them
// in device memory, for the queries that outgrow the LDS tables (or all
// queries, on request): the previous and the current position's cells (40
// bytes each) and an open-addressing hash of the current ones keyed by (k,
// s), whose entries carry the position's generation so that it never needs
// clearing between positions.
#include "views.h"

#include <algorithm>
#include <type_traits>
#include <vector>

namespace rb3 {

constexpr int32_t HP_NEG = -1000000000;

// A cell's score H (best alignment), E (ending in an insertion) and F
// (ending in a deletion) each come with a representative: a node holds
// every string with its SA interval (X and XZ when each occurrence of X is
// followed by Z), and their reverse complements start at different rows.
// A score's representative is, among the node's strings whose alignment
// attains it, the one whose reverse complement's interval starts first; a
// match or deletion passes on the representative of the score it extends
// with b prepended, an insertion passes it on unchanged. Backward extension
// keeps the order of those starts among a node's strings, so keeping the
// best (score, start) offer per score gives that string.
//
// A score and its representative's reverse-complement start travel as one
// word: the score in the high bits, the start's complement in the low
// HAPL_KRC_BITS bits, so that an unsigned maximum keeps the higher score
// and, at equal scores, the smaller start. Only positive scores are packed;
// 0 means none.
constexpr uint64_t HP_KMASK = ((uint64_t)1 << HAPL_KRC_BITS) - 1u;

__device__ __forceinline__ uint64_t hp_pack(int32_t v, int64_t kr) {
    return ((uint64_t)(uint32_t)v << HAPL_KRC_BITS) | (HP_KMASK - (uint64_t)kr);
}
__device__ __forceinline__ int32_t hp_val(uint64_t w) { return (int32_t)(w >> HAPL_KRC_BITS); }
__device__ __forceinline__ int64_t hp_rep(uint64_t w) { return (int64_t)(HP_KMASK - (w & HP_KMASK)); }

struct HpCell {
    int64_t k, s;
    uint64_t hw, ew, fw;  // packed H, E, F
    int32_t dirty;
};

struct HpParams {
    int32_t match, mismatch, gap_open, gap_ext, band, cap, hcap;
};

// What a gap passes on from a cell with packed H hw (positive) and packed
// gap score gw (E or F): max(H - open, G) - ext, with the representative of
// the higher term (the smaller start at a tie); 0 when not positive.
__device__ __forceinline__ uint64_t hp_gap(uint64_t hw, uint64_t gw, const HpParams &p) {
    const int32_t a = hp_val(hw) - p.gap_open;
    const int32_t b = gw ? hp_val(gw) : HP_NEG;
    const int32_t v = (a > b ? a : b) - p.gap_ext;
    if (v <= 0) return 0;
    const int64_t ra = hp_rep(hw), rb = gw ? hp_rep(gw) : ra;
    return hp_pack(v, a > b ? ra : (b > a ? rb : (ra < rb ? ra : rb)));
}

__device__ __forceinline__ int32_t hp_max(int32_t a, int32_t b) { return a > b ? a : b; }

__device__ __forceinline__ bool hp_before(const HpCell &a, const HpCell &b) {
    if (hp_val(a.hw) != hp_val(b.hw)) return hp_val(a.hw) > hp_val(b.hw);
    if (a.k != b.k) return a.k < b.k;
    return a.s < b.s;
}

// The four children (b = A, C, G, T) of bi-interval (k, kr, s): Algorithm
// 3's backward extension, all symbols from one rank-all pair.
template <class V>
__device__ __forceinline__ void hp_children(const V &ix, int64_t k, int64_t kr, int64_t s, int64_t ck[4],
                                            int64_t ckr[4], int64_t cs[4]) {
    int64_t p0[6], p1[6];
    ix.pi2(k, k + s, p0, p1);
    int64_t occ[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) occ[c] = p1[c] - p0[c];
    // reverse-complement starts: kr + occurrences of the complements below
    // comp(b) in the order $ < A < C < G < T < N; comp(A) = T, comp(C) = G,
    // comp(G) = C, comp(T) = A, so for b = A the sum runs over $, A, C, G of
    // the complements ($, T, G, C), and so on
    const int64_t oS = occ[0], oA = occ[1], oC = occ[2], oG = occ[3], oT = occ[4];
    ck[0] = p0[1], cs[0] = oA, ckr[0] = kr + oS + oT + oG + oC;  // A: comp T (4): b' < 4
    ck[1] = p0[2], cs[1] = oC, ckr[1] = kr + oS + oT + oG;       // C: comp G (3)
    ck[2] = p0[3], cs[2] = oG, ckr[2] = kr + oS + oT;            // G: comp C (2)
    ck[3] = p0[4], cs[3] = oT, ckr[3] = kr + oS;                 // T: comp A (1)
}

// v[b] as a sum of masked terms, so that a loop over b needs no indexed
// register array (which the compiler would place in scratch memory)
__device__ __forceinline__ int64_t hp_pick(const int64_t v[4], int b) {
    int64_t r = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) r += v[c] & -(int64_t)(b == c);
    return r;
}

__device__ __forceinline__ uint32_t hp_hash(int64_t k, int64_t s, uint32_t mask) {
    uint64_t z = (uint64_t)k * 0x9E3779B97F4A7C15ull ^ ((uint64_t)s + 0x632BE59BD9B4E019ull) * 0xC2B2AE3D27D4EB4Full;
    z ^= z >> 29;
    return (uint32_t)z & mask;
}

// Index of the current position's cell for (k, s), created when absent;
// -1 when the table is full.
__device__ __forceinline__ int32_t hp_upsert(HpCell *T, int32_t &nT, uint32_t *hash, const HpParams &p, uint32_t gen,
                                             int64_t k, int64_t s) {
    const uint32_t mask = (uint32_t)p.hcap - 1u;
    uint32_t h = hp_hash(k, s, mask);
    for (;;) {
        const uint32_t e = hash[h];
        if ((e >> 16) == gen) {
            const int32_t j = (int32_t)(e & 0xFFFFu);
            if (T[j].k == k && T[j].s == s) return j;
            h = (h + 1u) & mask;
            continue;
        }
        if (nT >= p.cap) return -1;
        const int32_t j = nT++;
        HpCell c;
        c.k = k;
        c.s = s;
        c.hw = c.ew = c.fw = 0;
        c.dirty = 1;
        T[j] = c;
        hash[h] = (gen << 16) | (uint32_t)j;
        return j;
    }
}

// The w-th largest score among the positive cells of B[0, n), or 1 when
// fewer than w cells are positive; *above = positive cells scoring higher.
// The positive scores are copied to hv (n entries) and the w-th largest is
// found there by selection (Hoare partitions around a median of three).
__device__ int32_t hp_kth(const HpCell *B, int32_t n, int32_t w, int32_t *hv, int32_t *above) {
    int32_t m = 0;
    for (int32_t x = 0; x < n; ++x) {
        const int32_t h = hp_val(B[x].hw);
        if (h > 0) hv[m++] = h;
    }
    if (m < w) {
        *above = m;
        return 1;
    }
    // w-th largest = element of rank w - 1 in decreasing order
    int32_t lo = 0, hi = m - 1;
    const int32_t r = w - 1;
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        int32_t a = hv[lo], b = hv[mid], c = hv[hi];
        // median of the three as pivot
        const int32_t piv = a > b ? (b > c ? b : (a > c ? c : a)) : (a > c ? a : (b > c ? c : b));
        int32_t i = lo, j = hi;
        while (i <= j) {
            while (hv[i] > piv) ++i;
            while (hv[j] < piv) --j;
            if (i <= j) {
                const int32_t t = hv[i];
                hv[i] = hv[j];
                hv[j] = t;
                ++i;
                --j;
            }
        }
        if (r <= j)
            hi = j;
        else if (r >= i)
            lo = i;
        else
            break;
    }
    const int32_t tau = hv[r];
    int32_t c = 0;
    for (int32_t x = 0; x < m; ++x) c += hv[x] > tau;
    *above = c;
    return tau;
}

__device__ __forceinline__ void hp_swap(HpCell *B, int32_t x, int32_t y) {
    if (x != y) {
        const HpCell t = B[x];
        B[x] = B[y];
        B[y] = t;
    }
}

// Device-memory tables, one thread per query (queries whose cells outgrow
// the on-chip tables of k_hapl_wave, or all of them on request). Per query:
// A (previous cells) then B (current cells), each cap cells, and hcap hash
// entries. cnt[q] = result cells, written in order to the start of the
// query's A; -1 when the query needed more than cap cells at a position.
//
// With a band W the deletion step only extends a cell whose F passed on,
// f = max(H - q, F) - e, is at least tau, the W-th best score held after
// the match and insertion steps:
// the cells it would reach score at most f, scores only rise during the
// step, so tau never exceeds the W-th best score at the end of the step,
// and a cell scoring below that is neither kept nor the source of a kept
// cell's score (a deletion parent always scores more than its child's F).
// The band's cells and their H and E are therefore those of the full
// closure; F is not carried to the next position.
template <class V>
__global__ __launch_bounds__(64) void k_hapl(V ix, const uint8_t *__restrict__ Q, const int64_t *__restrict__ qse, int64_t nq,
                       HpParams p, HpCell *__restrict__ cells, uint32_t *__restrict__ hashes,
                       int32_t *__restrict__ hvals, int32_t *__restrict__ cnt,
                       unsigned long long *__restrict__ stats) {
    const int64_t qi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (qi >= nq) return;
    HpCell *A = cells + qi * 2 * (int64_t)p.cap;
    HpCell *B = A + p.cap;
    uint32_t *hash = hashes + qi * (int64_t)p.hcap;
    int32_t *hv = hvals + qi * (int64_t)p.cap;
    // qse: start and end of each query's codes, side by side
    const uint8_t *P = Q + qse[2 * qi];
    const int64_t L = qse[2 * qi + 1] - qse[2 * qi];
    uint64_t n_ext = 0, n_units = 0, n_cells = 0;
    int32_t nA = 1, nB = 0;
    {
        HpCell r;  // the root: the empty string, score 0
        r.k = 0;
        r.s = ix.size();
        r.hw = hp_pack(0, 0);
        r.ew = r.fw = 0;
        r.dirty = 0;
        A[0] = r;
    }
    bool full = false;
    for (int64_t t = L - 1; t >= 0 && !full; --t) {
        // hash entries are tagged with a 16-bit generation, 1 .. 65535
        const uint32_t gen = (uint32_t)((L - 1 - t) % 65535) + 1u;
        if (gen == 1u && t != L - 1)
            for (int32_t h = 0; h < p.hcap; ++h) hash[h] = 0u;
        const uint32_t a = P[t];
        nB = 0;
        // match / mismatch and insertion from the previous position's cells
        for (int32_t x = 0; x < nA && !full; ++x) {
            const HpCell c = A[x];
            const int32_t H = hp_val(c.hw);
            int64_t ck[4], ckr[4], cs[4];
            hp_children(ix, c.k, hp_rep(c.hw), c.s, ck, ckr, cs);
            ++n_ext;
            n_units += ix.units(c.k, c.k + c.s);
#pragma unroll 1
            for (int b = 0; b < 4; ++b) {
                const int64_t sb = hp_pick(cs, b);
                const int32_t v = H + ((uint32_t)(b + 1) == a ? p.match : -p.mismatch);
                if (!full && sb > 0 && v > 0) {
                    const int32_t j = hp_upsert(B, nB, hash, p, gen, hp_pick(ck, b), sb);
                    if (j < 0) {
                        full = true;
                    } else {
                        const uint64_t w = hp_pack(v, hp_pick(ckr, b));
                        if (w > B[j].hw) B[j].hw = w;
                    }
                }
            }
            if (full) break;
            const uint64_t iw = hp_gap(c.hw, c.ew, p);  // the insertion: the same string
            if (iw) {
                const int32_t j = hp_upsert(B, nB, hash, p, gen, c.k, c.s);
                if (j < 0) {
                    full = true;
                    break;
                }
                if (iw > B[j].ew) B[j].ew = iw;
                if (iw > B[j].hw) B[j].hw = iw;
            }
        }
        // deletion, repeated until no cell improves: a cell whose F rose
        // (a higher score, or a representative starting first) since it last
        // passed a deletion on is marked dirty; an offer that raises H raises
        // F too, since every deletion offer goes to both
        int32_t above = 0;
        const int32_t tau = (p.band > 0 && !full) ? hp_kth(B, nB, p.band, hv, &above) : 1;
        bool changed = true;
        while (changed && !full) {
            changed = false;
            for (int32_t x = 0; x < nB && !full; ++x) {
                if (!B[x].dirty) continue;
                B[x].dirty = 0;
                if (hp_val(B[x].hw) <= 0) continue;
                const uint64_t fw = hp_gap(B[x].hw, B[x].fw, p);
                const int32_t f = hp_val(fw);
                if (f <= 0 || f < tau) continue;
                int64_t ck[4], ckr[4], cs[4];
                hp_children(ix, B[x].k, hp_rep(fw), B[x].s, ck, ckr, cs);
                ++n_ext;
                n_units += ix.units(B[x].k, B[x].k + B[x].s);
#pragma unroll 1
                for (int b = 0; b < 4; ++b) {
                    const int64_t sb = hp_pick(cs, b);
                    if (!full && sb > 0) {
                        const int32_t j = hp_upsert(B, nB, hash, p, gen, hp_pick(ck, b), sb);
                        const uint64_t w = j < 0 ? 0 : hp_pack(f, hp_pick(ckr, b));
                        if (j < 0) {
                            full = true;
                        } else if (w > B[j].fw) {
                            B[j].fw = w;
                            if (w > B[j].hw) B[j].hw = w;
                            B[j].dirty = 1;
                            changed = true;
                        }
                    }
                }
            }
        }
        if (full) break;
        n_cells += (uint64_t)nB;
        // keep H > 0; with a band, the W best
        int32_t w = 0;
        for (int32_t x = 0; x < nB; ++x)
            if (hp_val(B[x].hw) > 0) B[w++] = B[x];
        if (p.band > 0 && w > p.band) {
            const int32_t tau = hp_kth(B, w, p.band, hv, &above);
            // the cells scoring above tau first, then those scoring tau
            int32_t a0 = 0;
            for (int32_t x = 0; x < w; ++x)
                if (hp_val(B[x].hw) > tau) hp_swap(B, a0++, x);
            int32_t e0 = a0;
            for (int32_t x = a0; x < w; ++x)
                if (hp_val(B[x].hw) == tau) hp_swap(B, e0++, x);
            // of the ties, the band's remaining places go to the smallest
            // (k, s)
            const int32_t r = p.band - above;
            if (e0 - a0 > r) {
                for (int32_t y = a0; y < a0 + r; ++y) {
                    int32_t best = y;
                    for (int32_t x = y + 1; x < e0; ++x)
                        if (B[x].k < B[best].k || (B[x].k == B[best].k && B[x].s < B[best].s)) best = x;
                    hp_swap(B, y, best);
                }
            }
            w = p.band;
        }
        for (int32_t x = 0; x < w; ++x) {
            HpCell c = B[x];
            c.dirty = 0;
            A[x] = c;
        }
        nA = w;
    }
    if (n_ext) {
        atomicAdd(&stats[0], (unsigned long long)n_ext);
        atomicAdd(&stats[1], (unsigned long long)n_units);
        atomicAdd(&stats[2], (unsigned long long)n_cells);
    }
    if (full) {
        cnt[qi] = -1;
        return;
    }
    if (L == 0) nA = 0;  // the root alone is not a result
    // order the result cells (insertion sort), then the redundancy filter
    for (int32_t x = 1; x < nA; ++x) {
        const HpCell c = A[x];
        int32_t y = x - 1;
        while (y >= 0 && hp_before(c, A[y])) {
            A[y + 1] = A[y];
            --y;
        }
        A[y + 1] = c;
    }
    int32_t w = 0;
    for (int32_t x = 0; x < nA; ++x) {
        const HpCell c = A[x];
        bool inside = false;
        for (int32_t y = 0; y < w && !inside; ++y) {
            const HpCell &q = A[y];
            const int64_t ckr = hp_rep(c.hw), qkr = hp_rep(q.hw);
            inside = (c.k >= q.k && c.k + c.s <= q.k + q.s) || (ckr >= qkr && ckr + c.s <= qkr + q.s);
        }
        if (!inside) A[w++] = c;
    }
    cnt[qi] = w;
}

// ---------------------------------------------------------------------------
// Queries on wavefronts, cells in LDS
// ---------------------------------------------------------------------------
//
// A query gets 64 / QPW lanes of one wavefront (QPW = 1 or 2 queries a
// wavefront). The lanes share the query's cells: each extends its own cells
// (so up to that many rank-all pairs of one query are in flight together)
// and inserts the results into a hash in LDS. A cell is claimed by
// allocating it, writing its key and publishing it in a hash slot with a
// compare-and-swap; a lane that loses the race to an equal key leaves its
// allocation unlinked (s = 0, scores at minus infinity), so no lane ever
// waits on another. Scores are raised with LDS atomic max. A query whose
// cells outgrow the LDS tables is finished by k_hapl instead (cnt = -2).
// The wavefront's barriers are reached by all its lanes: the queries of a
// wavefront step through their positions and deletion rounds together, a
// query that has finished (or moved) idling.
//
// CAP = cells one position may hold in LDS, PCAP = the previous position's
// cells (the band). Near the query's end the cells' strings are short and
// all their children occur, so a position can hold five cells per previous
// one (four children and the insertion): 64 cells cover bands up to 12 and
// 128 bands up to 25 that way, larger bands on 128 cells may move queries
// to device memory. Occupancy is set by LDS (allocated in 512-byte
// granules) and registers:
//   bands up to 12: two queries a wavefront, 64 cells and 16 previous ones
//     each (7.8 KB a wavefront; registers for four wavefronts a SIMD, so
//     32 queries a CU);
//   bands up to 32: two queries, 128 cells and 32 previous ones (13.3 KB:
//     11 wavefronts, 22 queries a CU);
//   else one query, 256 and 256 (21.0 KB: 7 queries a CU).
constexpr int HW_CAP_PAIR = 64;
constexpr int HW_PAIR_BAND = 12;
constexpr int HW_PAIR_PREV = 16;
constexpr int HW_CAP_SMALL = 128;
constexpr int HW_CAP_LARGE = 256;
constexpr int HW_SMALL_BAND = 32;
static_assert(HW_PAIR_PREV >= HW_PAIR_BAND, "the previous cells hold the band");

// HB = histogram bins, one per lane of the query. Hash slots: two per
// cell, four for the 64-cell tables, whose occupancy registers bound (the
// shorter probe chains are free there; eight cost more to clear at every
// position than they save).
// A cell's E comes from one previous cell only (the one of its node), so E
// is kept per previous cell (eW) and a cell names that cell (ci, index + 1;
// 0: no insertion reached it) instead of an E word per cell.
template <int CAP, int PCAP, int HB>
struct HwLds {
    static constexpr int HS = (CAP <= HW_CAP_PAIR ? 4 : 2) * CAP;
    using PIdx = typename std::conditional<(PCAP < 255), uint8_t, uint16_t>::type;
    int64_t ck[CAP], cs[CAP];  // current position's cells
    uint64_t cH[CAP], cF[CAP];  // packed scores with representatives
    int32_t slot[HS];  // cell index + 1, 0 = empty
    int64_t pk[PCAP], ps[PCAP];  // previous position's cells (at most the band)
    uint64_t pH[PCAP], pE[PCAP];
    uint64_t eW[PCAP];  // packed E each previous cell passes to its node's cell
    int32_t hist[HB];  // positive scores mx - i, for the band's threshold
    int32_t nC, nP, flag, changed, tcount;
    uint8_t cd[CAP];  // dirty (deletion step), then kept among the tied cells
    PIdx ci[CAP];
};

// Reductions over the HW lanes of one query (HW = 64 or 32).
template <int HW>
__device__ __forceinline__ int32_t hw_sum(int32_t v) {
    for (int o = HW / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <int HW>
__device__ __forceinline__ int32_t hw_maxr(int32_t v) {
    for (int o = HW / 2; o > 0; o >>= 1) v = hp_max(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ uint64_t hw_sum64(uint64_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int64_t hw_max64(int64_t v) {
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    return v;
}

// Index of the cell for (k, s), created when absent; -1 when the tables
// are full.
template <class LDS>
__device__ int32_t hw_upsert(LDS &S, int32_t cap, int64_t k, int64_t s) {
    constexpr int HS = LDS::HS;
    uint32_t h = hp_hash(k, s, HS - 1);
    int32_t j = -1;
    for (int probe = 0; probe < HS; ++probe) {
        int32_t v = __hip_atomic_load(&S.slot[h], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (v == 0) {
            if (j < 0) {
                j = atomicAdd(&S.nC, 1);
                if (j >= cap) return -1;
                S.ck[j] = k;
                S.cs[j] = s;
                S.cH[j] = 0;
                S.cF[j] = 0;
                S.cd[j] = 1;
                S.ci[j] = 0;
            }
            int32_t expected = 0;
            if (__hip_atomic_compare_exchange_strong(&S.slot[h], &expected, j + 1, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP))
                return j;
            v = expected;
        }
        const int32_t c = v - 1;
        if (S.ck[c] == k && S.cs[c] == s) {
            if (j >= 0) S.cs[j] = 0;  // the allocation stays unlinked (no score)
            return c;
        }
        h = (h + 1) & (HS - 1);
    }
    return -1;
}

// Histogram of the positive scores mx - (HW - 1) .. mx, mx the highest
// (bin i counts score mx - i), in two steps around a barrier: the maximum,
// the positive cells' number and cleared bins, then the counts.
template <int HW, class LDS>
__device__ void hw_hist_start(LDS &S, int32_t n, int hl, int32_t *mx_out, int32_t *pos_out) {
    int32_t mx = 0, c = 0;
    for (int32_t x = hl; x < n; x += HW) {
        const int32_t h = hp_val(S.cH[x]);
        if (h > 0) {
            ++c;
            mx = hp_max(mx, h);
        }
    }
    *pos_out = hw_sum<HW>(c);
    *mx_out = hw_maxr<HW>(mx);
    S.hist[hl] = 0;
}

template <int HW, class LDS>
__device__ void hw_hist_fill(LDS &S, int32_t n, int hl, int32_t mx) {
    for (int32_t x = hl; x < n; x += HW) {
        const int32_t h = hp_val(S.cH[x]);
        if (h > 0 && mx - h < HW) atomicAdd(&S.hist[mx - h], 1);
    }
}

// The w-th largest positive score from the histogram, when its bins hold
// at least w cells (else false): *above = cells scoring higher, *ties =
// cells scoring it. A scan of the bins across the query's lanes; hbase is
// the first lane of the query in the wavefront.
template <int HW, class LDS>
__device__ bool hw_hist_tau(const LDS &S, int32_t w, int hl, int hbase, int32_t mx, int32_t *tau,
                            int32_t *above, int32_t *ties) {
    const int32_t c = S.hist[hl];
    int32_t v = c;
    for (int d = 1; d < HW; d <<= 1) {
        const int32_t u = __shfl_up(v, d, HW);
        if (hl >= d) v += u;
    }
    unsigned long long m = __ballot(v >= w);
    if (HW < 64) m = (m >> hbase) & ((1ull << HW) - 1ull);
    if (m == 0) return false;
    const int i = __ffsll(m) - 1;
    const int32_t vi = __shfl(v, hbase + i), ci = __shfl(c, hbase + i);
    *tau = mx - i;
    *above = vi - ci;
    *ties = ci;
    return true;
}

// The same by a binary search over the scores 1 .. mx, each probe a count
// over the n cells (for thresholds below the histogram's range); the n
// cells hold at least w positive ones.
template <int HW, class LDS>
__device__ int32_t hw_kth_search(const LDS &S, int32_t n, int32_t w, int hl, int32_t mx, int32_t *above,
                                 int32_t *ties) {
    int32_t lo = 1, hi = mx;  // the largest v with w or more scores >= v
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo + 1) >> 1);
        int32_t k = 0;
        for (int32_t x = hl; x < n; x += HW) k += hp_val(S.cH[x]) >= mid;
        if (hw_sum<HW>(k) >= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    int32_t ka = 0, kt = 0;
    for (int32_t x = hl; x < n; x += HW) {
        ka += hp_val(S.cH[x]) > lo;
        kt += hp_val(S.cH[x]) == lo;
    }
    *above = hw_sum<HW>(ka);
    *ties = hw_sum<HW>(kt);
    return lo;
}

// One block of 64 threads (one wavefront) holds QPW queries; cap <= CAP
// cells per position. Query qi's results (at most outcap) go to
// wout[qi * outcap ..] in order, cnt[qi] = their number, or -2 when its
// cells outgrew cap.
template <class V, int CAP, int PCAP, int QPW>
__global__ __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(CAP >= 128 ? 2 : 4))) void k_hapl_wave(V ix, const uint8_t *__restrict__ Q,
                                                  const int64_t *__restrict__ qoff, int64_t nq, HpParams p,
                                                  int32_t cap, int32_t outcap, int64_t qbase,
                                                  rb3_hapl_t *__restrict__ wout, int32_t *__restrict__ cnt,
                                                  unsigned long long *__restrict__ stats) {
    constexpr int HW = 64 / QPW;  // lanes a query
    using LDS = HwLds<CAP, PCAP, HW>;
    __shared__ LDS SS[QPW];
    const int lane = threadIdx.x;
    const int hq = lane / HW, hl = lane % HW, hbase = hq * HW;
    LDS &S = SS[hq];
    const int64_t qi = blockIdx.x * (int64_t)QPW + hq;
    const bool real = qi < nq;
    const uint8_t *P = Q + (real ? qoff[qi] : 0);
    const int64_t L = real ? qoff[qi + 1] - qoff[qi] : 0;
    const int64_t Lmax = hw_max64(L);
    uint64_t n_ext = 0, n_units = 0, n_cells = 0;
    if (hl == 0) {  // the root: the empty string, score 0
        S.pk[0] = 0;
        S.ps[0] = ix.size();
        S.pH[0] = hp_pack(0, 0);
        S.pE[0] = 0;
        S.nP = 1;
        S.flag = 0;
    }
    __syncthreads();
    bool over = false;  // the cells outgrew the tables: the query moves
    for (int64_t step = 0; step < Lmax; ++step) {
        bool on = step < L && !over;
        const uint32_t a = on ? P[L - 1 - step] : 0u;
        if (on) {
            for (int h = hl; h < LDS::HS; h += HW) S.slot[h] = 0;
            if (hl == 0) S.nC = 0;
        }
        __syncthreads();
        // match / mismatch and insertion from the previous position's cells
        if (on) {
            const int32_t nP = S.nP;
            for (int32_t x = hl; x < nP; x += HW) {
                const int64_t k = S.pk[x], sz = S.ps[x];
                const uint64_t hw = S.pH[x];
                const int32_t H = hp_val(hw);
                int64_t ck[4], ckr[4], cs[4];
                hp_children(ix, k, hp_rep(hw), sz, ck, ckr, cs);
                ++n_ext;
                n_units += ix.units(k, k + sz);
                bool bad = false;
#pragma unroll 1
                for (int b = 0; b < 4; ++b) {
                    const int64_t sb = hp_pick(cs, b);
                    const int32_t v = H + ((uint32_t)(b + 1) == a ? p.match : -p.mismatch);
                    if (!bad && sb > 0 && v > 0) {
                        const int32_t j = hw_upsert(S, cap, hp_pick(ck, b), sb);
                        if (j < 0)
                            bad = true;
                        else
                            atomicMax((unsigned long long *)&S.cH[j], (unsigned long long)hp_pack(v, hp_pick(ckr, b)));
                    }
                }
                // the insertion: the same node and string
                const uint64_t iw = bad ? 0 : hp_gap(hw, S.pE[x], p);
                if (iw) {
                    const int32_t j = hw_upsert(S, cap, k, sz);
                    if (j < 0) {
                        bad = true;
                    } else {
                        // the only insertion into this node: plain stores
                        S.eW[x] = iw;
                        S.ci[j] = (typename LDS::PIdx)(x + 1);
                        atomicMax((unsigned long long *)&S.cH[j], (unsigned long long)iw);
                    }
                }
                if (bad) S.flag = 1;
            }
        }
        __syncthreads();
        if (on && S.flag) over = true;
        on = on && !over;
        // the band's threshold so far: the histogram of the top HW scores
        // is kept up to date through the deletion step (hm) when it holds
        // the band, else a search gives a fixed lower bound
        int32_t mx = 0, pos = 0, tau = 1, above = 0, ties = 0;
        bool hm = false;
        const bool banded = on && p.band > 0;
        if (banded) hw_hist_start<HW>(S, S.nC, hl, &mx, &pos);
        __syncthreads();
        if (banded) hw_hist_fill<HW>(S, S.nC, hl, mx);
        __syncthreads();
        if (banded && pos >= p.band) {
            hm = hw_hist_tau<HW>(S, p.band, hl, hbase, mx, &tau, &above, &ties);
            if (!hm) tau = hw_kth_search<HW>(S, S.nC, p.band, hl, mx, &above, &ties);
        }
        // deletion in rounds until no cell improves; a round extends the
        // dirty cells present at its start
        bool dl = on;
        for (;;) {
            if (dl && hl == 0) S.changed = 0;
            __syncthreads();
            if (dl) {
                if (hm) hw_hist_tau<HW>(S, p.band, hl, hbase, mx, &tau, &above, &ties);  // tau only rises
                const int32_t n0 = S.nC;
                for (int32_t x = hl; x < n0; x += HW) {
                    if (!S.cd[x]) continue;
                    S.cd[x] = 0;
                    const uint64_t hw = S.cH[x];
                    if (hp_val(hw) <= 0) continue;
                    const uint64_t fw = hp_gap(hw, S.cF[x], p);
                    const int32_t f = hp_val(fw);
                    if (f <= 0 || f < tau) continue;
                    const int64_t k = S.ck[x], sz = S.cs[x];
                    int64_t ck[4], ckr[4], cs[4];
                    hp_children(ix, k, hp_rep(fw), sz, ck, ckr, cs);
                    ++n_ext;
                    n_units += ix.units(k, k + sz);
                    bool bad = false;
#pragma unroll 1
                    for (int b = 0; b < 4; ++b) {
                        const int64_t sb = hp_pick(cs, b);
                        if (!bad && sb > 0) {
                            const int32_t j = hw_upsert(S, cap, hp_pick(ck, b), sb);
                            const unsigned long long w = j < 0 ? 0ull : hp_pack(f, hp_pick(ckr, b));
                            if (j < 0) {
                                bad = true;
                            } else if (atomicMax((unsigned long long *)&S.cF[j], w) < w) {
                                // every deletion offer goes to H as well, so
                                // H only changes when F does
                                const int32_t old = hp_val(atomicMax((unsigned long long *)&S.cH[j], w));
                                // a deletion never tops its parent, so f < mx
                                if (hm && old < f) {
                                    if (old > 0 && mx - old < HW) atomicSub(&S.hist[mx - old], 1);
                                    if (mx - f < HW) atomicAdd(&S.hist[mx - f], 1);
                                }
                                S.cd[j] = 1;
                                S.changed = 1;
                            }
                        }
                    }
                    if (bad) S.flag = 1;
                }
            }
            __syncthreads();
            if (dl) {
                if (S.flag) {
                    over = true;
                    dl = false;
                } else if (!S.changed) {
                    dl = false;
                }
            }
            if (__ballot(dl) == 0) break;
        }
        on = on && !over;
        // keep H > 0; with a band, the W best (ties: smaller k, then s)
        const int32_t nC = on ? S.nC : 0;
        if (on && hl == 0) n_cells += (uint64_t)nC;
        bool cut = false;
        const bool rebuild = on && p.band > 0 && !hm;
        if (on && p.band > 0 && hm) {
            hw_hist_tau<HW>(S, p.band, hl, hbase, mx, &tau, &above, &ties);
            cut = true;
        }
        if (rebuild) hw_hist_start<HW>(S, nC, hl, &mx, &pos);
        __syncthreads();
        if (rebuild) hw_hist_fill<HW>(S, nC, hl, mx);
        __syncthreads();
        if (rebuild && pos >= p.band) {
            if (!hw_hist_tau<HW>(S, p.band, hl, hbase, mx, &tau, &above, &ties))
                tau = hw_kth_search<HW>(S, nC, p.band, hl, mx, &above, &ties);
            cut = true;
        }
        const int32_t r = p.band - above;
        const bool rank_ties = on && cut && ties > r;
        if (on && hl == 0) {
            S.nP = 0;
            S.tcount = 0;
        }
        __syncthreads();
        // the tied cells' keys into the previous-cells arrays (free now,
        // PCAP of them); each tied cell's rank among the tied cells decides
        // (in cd), counted over that list or, when it overflowed, over all
        // cells
        if (rank_ties) {
            for (int32_t x = hl; x < nC; x += HW) {
                if (hp_val(S.cH[x]) == tau) {
                    const int32_t d = atomicAdd(&S.tcount, 1);
                    if (d < PCAP) {
                        S.pk[d] = S.ck[x];
                        S.ps[d] = S.cs[x];
                    }
                }
            }
        }
        __syncthreads();
        if (rank_ties) {
            const int32_t T = S.tcount;
            for (int32_t x = hl; x < nC; x += HW) {
                if (hp_val(S.cH[x]) == tau) {
                    const int64_t k = S.ck[x], sz = S.cs[x];
                    int32_t rank = 0;
                    if (T <= PCAP) {
                        for (int32_t y = 0; y < T; ++y) rank += S.pk[y] < k || (S.pk[y] == k && S.ps[y] < sz);
                    } else {
                        for (int32_t y = 0; y < nC; ++y)
                            rank += hp_val(S.cH[y]) == tau && (S.ck[y] < k || (S.ck[y] == k && S.cs[y] < sz));
                    }
                    S.cd[x] = rank < r;
                }
            }
        }
        __syncthreads();
        if (on) {
            for (int32_t x = hl; x < nC; x += HW) {
                const int32_t H = hp_val(S.cH[x]);
                bool keep = H > 0;
                if (keep && cut) keep = H > tau || (H == tau && (!rank_ties || S.cd[x]));
                if (keep) {
                    const int32_t d = atomicAdd(&S.nP, 1);
                    S.pk[d] = S.ck[x];
                    S.ps[d] = S.cs[x];
                    S.pH[d] = S.cH[x];
                    S.pE[d] = S.ci[x] ? S.eW[S.ci[x] - 1] : 0;
                }
            }
        }
        __syncthreads();
    }
    n_ext = hw_sum64(n_ext);
    n_units = hw_sum64(n_units);
    n_cells = hw_sum64(n_cells);
    if (lane == 0 && n_ext) {
        atomicAdd(&stats[0], (unsigned long long)n_ext);
        atomicAdd(&stats[1], (unsigned long long)n_units);
        atomicAdd(&stats[2], (unsigned long long)n_cells);
    }
    if (hl != 0 || !real) return;
    if (over) {
        cnt[qi] = -2;
        return;
    }
    // the cells of the query's start, ordered, then the redundancy filter
    const int32_t n = L == 0 ? 0 : S.nP;  // the root alone is not a result
    for (int32_t x = 1; x < n; ++x) {
        const int64_t k = S.pk[x], sz = S.ps[x];
        const uint64_t hw = S.pH[x];
        const int32_t H = hp_val(hw);
        int32_t y = x - 1;
        while (y >= 0 && (hp_val(S.pH[y]) < H ||
                          (hp_val(S.pH[y]) == H && (S.pk[y] > k || (S.pk[y] == k && S.ps[y] > sz))))) {
            S.pk[y + 1] = S.pk[y];
            S.ps[y + 1] = S.ps[y];
            S.pH[y + 1] = S.pH[y];
            --y;
        }
        S.pk[y + 1] = k;
        S.ps[y + 1] = sz;
        S.pH[y + 1] = hw;
    }
    rb3_hapl_t *out = wout + qi * (int64_t)outcap;
    int32_t w = 0;
    for (int32_t x = 0; x < n; ++x) {
        const int64_t k = S.pk[x], kr = hp_rep(S.pH[x]), sz = S.ps[x];
        bool inside = false;
        for (int32_t y = 0; y < w && !inside; ++y)
            inside = (k >= out[y].k && k + sz <= out[y].k + out[y].s) ||
                     (kr >= out[y].krc && kr + sz <= out[y].krc + out[y].s);
        if (!inside) {
            rb3_hapl_t o;
            o.k = k;
            o.krc = kr;
            o.s = sz;
            o.score = hp_val(S.pH[x]);
            o.qid = (int32_t)(qbase + qi);
            out[w++] = o;
        }
    }
    cnt[qi] = w;
}

// Result records in order: query qidx[i]'s cells (of the thread tables)
// go to out[off[qidx[i]] ..].
__global__ void k_hapl_gather(const HpCell *__restrict__ cells, int64_t nq, int32_t cap,
                              const int32_t *__restrict__ cnt, const int64_t *__restrict__ off,
                              const int64_t *__restrict__ qidx, int64_t qbase, rb3_hapl_t *__restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const HpCell *A = cells + i * 2 * (int64_t)cap;
    const int64_t qi = qidx[i];
    const int32_t c = cnt[i];
    for (int32_t x = 0; x < c; ++x) {
        rb3_hapl_t r;
        r.k = A[x].k;
        r.krc = hp_rep(A[x].hw);
        r.s = A[x].s;
        r.score = hp_val(A[x].hw);
        r.qid = (int32_t)(qbase + qi);
        out[off[qi] + x] = r;
    }
}

// The same for the results of k_hapl_wave (queries it finished).
__global__ void k_hapl_wave_gather(const rb3_hapl_t *__restrict__ wout, int64_t nq, int32_t outcap,
                                   const int32_t *__restrict__ cnt, const int64_t *__restrict__ off,
                                   rb3_hapl_t *__restrict__ out) {
    const int64_t qi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (qi >= nq) return;
    const int32_t c = cnt[qi];
    for (int32_t x = 0; x < c; ++x) out[off[qi] + x] = wout[qi * (int64_t)outcap + x];
}

template <class V>
static int hapl_run_v(Ctx &c, const V &view, const char *name, const char *wname, const uint8_t *d_codes,
                      const int64_t *qlens, int64_t nq, const rb3_hapl_opts &o, int64_t out_cap, rb3_hapl_t *d_out,
                      int64_t *h_off, int64_t *h_bad, int64_t *h_stats) {
    HpParams p;
    p.match = o.match;
    p.mismatch = o.mismatch;
    p.gap_open = o.gap_open;
    p.gap_ext = o.gap_ext;
    p.band = o.band;
    p.cap = o.max_cells;
    int32_t h = 1;
    while (h < 2 * o.max_cells) h <<= 1;
    p.hcap = h;
    const bool wave = !o.device_tables;
    // LDS tables by band: two queries a wavefront with 64 cells each, one
    // with 128, or one with 256
    const int kind = (o.band > 0 && o.band <= HW_PAIR_BAND) ? 0 : (o.band > 0 && o.band <= HW_SMALL_BAND) ? 1 : 2;
    const int32_t wcap = std::min<int32_t>(kind == 0 ? HW_CAP_PAIR : kind == 1 ? HW_CAP_SMALL : HW_CAP_LARGE,
                                           o.max_cells);
    const int32_t outcap = o.band > 0 ? std::min<int32_t>(o.band, wcap) : wcap;
    std::vector<int64_t> qoff(nq + 1);
    qoff[0] = 0;
    for (int64_t i = 0; i < nq; ++i) qoff[i + 1] = qoff[i] + qlens[i];
    // a chunk's queries all fit the device-memory tables, so that those the
    // LDS tables cannot hold are finished in one launch
    const int64_t per_t = 2 * (int64_t)p.cap * (int64_t)sizeof(HpCell) + (int64_t)p.hcap * 4 + (int64_t)p.cap * 4;
    const int64_t per_w = (int64_t)outcap * (int64_t)sizeof(rb3_hapl_t) + 4;
    int64_t chunk = std::min<int64_t>(nq, std::max<int64_t>(1, HAPL_SCRATCH / per_t));
    if (wave) chunk = std::min<int64_t>(chunk, std::max<int64_t>(1, HAPL_SCRATCH / per_w));
    chunk = std::min<int64_t>(chunk, (int64_t)1 << 30);
    DBuf dq, wout, wcnt, cells, hash, hvals, tcnt, tq, doff, dst;
    RB3_ALLOC(dq, &c, (nq + 1) * sizeof(int64_t));
    RB3_ALLOC(doff, &c, (size_t)chunk * sizeof(int64_t));
    RB3_ALLOC(dst, &c, 4 * sizeof(unsigned long long));
    if (wave) {
        RB3_ALLOC(wout, &c, (size_t)chunk * (size_t)outcap * sizeof(rb3_hapl_t));
        RB3_ALLOC(wcnt, &c, (size_t)chunk * sizeof(int32_t));
    }
    RB3_HIP(hipMemsetAsync(dst.p, 0, 4 * sizeof(unsigned long long), c.stream));
    RB3_HIP(hipMemcpyAsync(dq.p, qoff.data(), (nq + 1) * sizeof(int64_t), hipMemcpyHostToDevice, c.stream));
    std::vector<int32_t> hc(chunk), ht;
    std::vector<int64_t> sub, hq;
    int64_t tcap = 0;   // queries the device-memory tables are allocated for
    int64_t moved = 0;  // queries the LDS tables could not hold
    h_off[0] = 0;
    for (int64_t q0 = 0; q0 < nq; q0 += chunk) {
        const int64_t m = std::min(chunk, nq - q0);
        sub.clear();
        if (wave) {
            if (kind == 0)
                RB3_LAUNCH(wname, (k_hapl_wave<V, HW_CAP_PAIR, HW_PAIR_PREV, 2>), dim3((uint32_t)((m + 1) / 2)), dim3(64), 0,
                           c.stream, view, d_codes, dq.as<int64_t>() + q0, m, p, wcap, outcap, q0,
                           wout.as<rb3_hapl_t>(), wcnt.as<int32_t>(), dst.as<unsigned long long>());
            else if (kind == 1)
                RB3_LAUNCH(wname, (k_hapl_wave<V, HW_CAP_SMALL, HW_SMALL_BAND, 2>), dim3((uint32_t)((m + 1) / 2)),
                           dim3(64), 0, c.stream, view, d_codes, dq.as<int64_t>() + q0, m, p, wcap, outcap, q0,
                           wout.as<rb3_hapl_t>(), wcnt.as<int32_t>(), dst.as<unsigned long long>());
            else
                RB3_LAUNCH(wname, (k_hapl_wave<V, HW_CAP_LARGE, HW_CAP_LARGE, 1>), dim3((uint32_t)m), dim3(64), 0,
                           c.stream, view, d_codes, dq.as<int64_t>() + q0, m, p, wcap, outcap, q0,
                           wout.as<rb3_hapl_t>(), wcnt.as<int32_t>(), dst.as<unsigned long long>());
            RB3_HIP(hipMemcpyAsync(hc.data(), wcnt.p, m * sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
            RB3_HIP(hipStreamSynchronize(c.stream));
            for (int64_t i = 0; i < m; ++i)
                if (hc[i] == -2) sub.push_back(i);
            moved += (int64_t)sub.size();
        } else {
            for (int64_t i = 0; i < m; ++i) sub.push_back(i);
        }
        const int64_t ns = (int64_t)sub.size();
        if (ns > 0) {
            if (ns > tcap) {
                cells.reset();
                hash.reset();
                hvals.reset();
                tcnt.reset();
                tq.reset();
                tcap = ns;
                RB3_ALLOC(cells, &c, (size_t)tcap * 2 * (size_t)p.cap * sizeof(HpCell));
                RB3_ALLOC(hash, &c, (size_t)tcap * (size_t)p.hcap * 4);
                RB3_ALLOC(hvals, &c, (size_t)tcap * (size_t)p.cap * 4);
                RB3_ALLOC(tcnt, &c, (size_t)tcap * sizeof(int32_t));
                RB3_ALLOC(tq, &c, (size_t)tcap * 3 * sizeof(int64_t));
            }
            // start and end of each query's codes, then its index in the chunk
            hq.resize(3 * ns);
            for (int64_t i = 0; i < ns; ++i) {
                hq[2 * i] = qoff[q0 + sub[i]];
                hq[2 * i + 1] = qoff[q0 + sub[i] + 1];
                hq[2 * ns + i] = sub[i];
            }
            RB3_HIP(hipMemcpyAsync(tq.p, hq.data(), 3 * ns * sizeof(int64_t), hipMemcpyHostToDevice, c.stream));
            RB3_HIP(hipMemsetAsync(hash.p, 0, (size_t)ns * (size_t)p.hcap * 4, c.stream));
            RB3_LAUNCH(name, k_hapl<V>, grid_for(ns, 64, 1 << 30), dim3(64), 0, c.stream, view, d_codes,
                       tq.as<int64_t>(), ns, p, cells.as<HpCell>(), hash.as<uint32_t>(), hvals.as<int32_t>(),
                       tcnt.as<int32_t>(), dst.as<unsigned long long>());
            ht.resize(ns);
            RB3_HIP(hipMemcpyAsync(ht.data(), tcnt.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
            RB3_HIP(hipStreamSynchronize(c.stream));
            for (int64_t i = 0; i < ns; ++i) {
                if (ht[i] < 0) {
                    *h_bad = q0 + sub[i];
                    return RB3_ELIMIT;
                }
                hc[sub[i]] = ht[i];
            }
        }
        for (int64_t i = 0; i < m; ++i) h_off[q0 + i + 1] = h_off[q0 + i] + hc[i];
        if (h_off[q0 + m] <= out_cap && h_off[q0 + m] > h_off[q0]) {
            RB3_HIP(hipMemcpyAsync(doff.p, h_off + q0, m * sizeof(int64_t), hipMemcpyHostToDevice, c.stream));
            if (wave)
                RB3_LAUNCH("hapl_wave_gather", k_hapl_wave_gather, grid_for(m, 64, 1 << 30), dim3(64), 0, c.stream,
                           wout.as<rb3_hapl_t>(), m, outcap, wcnt.as<int32_t>(), doff.as<int64_t>(), d_out);
            if (ns > 0)
                RB3_LAUNCH("hapl_gather", k_hapl_gather, grid_for(ns, 64, 1 << 30), dim3(64), 0, c.stream,
                           cells.as<HpCell>(), ns, p.cap, tcnt.as<int32_t>(), doff.as<int64_t>(),
                           tq.as<int64_t>() + 2 * ns, q0, d_out);
            // the offsets and counts are rewritten by the next chunk
            RB3_HIP(hipStreamSynchronize(c.stream));
        }
    }
    unsigned long long hs[4];
    RB3_HIP(hipMemcpyAsync(hs, dst.p, sizeof(hs), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipStreamSynchronize(c.stream));
    for (int i = 0; i < 3; ++i) h_stats[i] = (int64_t)hs[i];
    h_stats[3] = moved;
    return RB3_OK;
}

int hapl_run(Ctx &c, const DevIndex &ix, const RleView *rle, const uint8_t *d_codes, const int64_t *qlens,
             int64_t nq, const rb3_hapl_opts &o, int64_t out_cap, rb3_hapl_t *d_out, int64_t *h_off,
             int64_t *h_bad, int64_t *h_stats) {
    if (rle)
        return hapl_run_v(c, RleQView{*rle}, "hapl_rle", "hapl_wave_rle", d_codes, qlens, nq, o, out_cap, d_out,
                          h_off, h_bad, h_stats);
    return hapl_run_v(c, PlainView{ix}, "hapl", "hapl_wave", d_codes, qlens, nq, o, out_cap, d_out, h_off, h_bad,
                      h_stats);
}

}  // namespace rb3
