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
// One thread per query. Its cells live in device scratch: the previous and
// the current position's cells (48 bytes each) and an open-addressing hash
// of the current ones keyed by (k, s), whose entries carry the position's
// generation so that it never needs clearing between positions.
#include "views.h"

#include <algorithm>
#include <vector>

namespace rb3 {

constexpr int32_t HP_NEG = -1000000000;

struct HpCell {
    int64_t k, kr, s;
    int32_t H, E, F, dirty;
    int64_t pad;
};

struct HpParams {
    int32_t match, mismatch, gap_open, gap_ext, band, cap, hcap;
};

__device__ __forceinline__ int32_t hp_max(int32_t a, int32_t b) { return a > b ? a : b; }

__device__ __forceinline__ bool hp_before(const HpCell &a, const HpCell &b) {
    if (a.H != b.H) return a.H > b.H;
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

__device__ __forceinline__ uint32_t hp_hash(int64_t k, int64_t s, uint32_t mask) {
    uint64_t z = (uint64_t)k * 0x9E3779B97F4A7C15ull ^ ((uint64_t)s + 0x632BE59BD9B4E019ull) * 0xC2B2AE3D27D4EB4Full;
    z ^= z >> 29;
    return (uint32_t)z & mask;
}

// Index of the current position's cell for (k, s), created when absent;
// -1 when the table is full.
__device__ __forceinline__ int32_t hp_upsert(HpCell *T, int32_t &nT, uint32_t *hash, const HpParams &p, uint32_t gen,
                                             int64_t k, int64_t kr, int64_t s) {
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
        c.kr = kr;
        c.s = s;
        c.H = c.E = c.F = HP_NEG;
        c.dirty = 1;
        c.pad = 0;
        T[j] = c;
        hash[h] = (gen << 16) | (uint32_t)j;
        return j;
    }
}

// Per query: A (previous cells) then B (current cells), each cap cells, and
// hcap hash entries. cnt[q] = result cells, written in order to the start
// of the query's A; -1 when the query needed more than cap cells at a
// position.
template <class V>
__global__ void k_hapl(V ix, const uint8_t *__restrict__ Q, const int64_t *__restrict__ qoff, int64_t nq,
                       HpParams p, HpCell *__restrict__ cells, uint32_t *__restrict__ hashes,
                       int32_t *__restrict__ cnt) {
    const int64_t qi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (qi >= nq) return;
    HpCell *A = cells + qi * 2 * (int64_t)p.cap;
    HpCell *B = A + p.cap;
    uint32_t *hash = hashes + qi * (int64_t)p.hcap;
    const uint8_t *P = Q + qoff[qi];
    const int64_t L = qoff[qi + 1] - qoff[qi];
    int32_t nA = 1, nB = 0;
    {
        HpCell r;
        r.k = 0;
        r.kr = 0;
        r.s = ix.size();
        r.H = 0;
        r.E = r.F = HP_NEG;
        r.dirty = 0;
        r.pad = 0;
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
            int64_t ck[4], ckr[4], cs[4];
            hp_children(ix, c.k, c.kr, c.s, ck, ckr, cs);
            for (int b = 0; b < 4; ++b) {
                if (cs[b] <= 0) continue;
                const int32_t j = hp_upsert(B, nB, hash, p, gen, ck[b], ckr[b], cs[b]);
                if (j < 0) {
                    full = true;
                    break;
                }
                B[j].H = hp_max(B[j].H, c.H + ((uint32_t)(b + 1) == a ? p.match : -p.mismatch));
            }
            if (full) break;
            const int32_t j = hp_upsert(B, nB, hash, p, gen, c.k, c.kr, c.s);
            if (j < 0) {
                full = true;
                break;
            }
            const int32_t e = hp_max(c.H - p.gap_open, c.E) - p.gap_ext;
            B[j].E = hp_max(B[j].E, e);
            B[j].H = hp_max(B[j].H, B[j].E);
        }
        // deletion, repeated until no cell improves: a cell whose H or F
        // rose since it last passed its F on is marked dirty
        bool changed = true;
        while (changed && !full) {
            changed = false;
            for (int32_t x = 0; x < nB && !full; ++x) {
                if (!B[x].dirty) continue;
                B[x].dirty = 0;
                if (B[x].H <= 0) continue;
                const int32_t f = hp_max(B[x].H - p.gap_open, B[x].F) - p.gap_ext;
                if (f <= 0) continue;
                int64_t ck[4], ckr[4], cs[4];
                hp_children(ix, B[x].k, B[x].kr, B[x].s, ck, ckr, cs);
                for (int b = 0; b < 4; ++b) {
                    if (cs[b] <= 0) continue;
                    const int32_t j = hp_upsert(B, nB, hash, p, gen, ck[b], ckr[b], cs[b]);
                    if (j < 0) {
                        full = true;
                        break;
                    }
                    if (f > B[j].F) {
                        B[j].F = f;
                        if (f > B[j].H) B[j].H = f;
                        B[j].dirty = 1;
                        changed = true;
                    }
                }
            }
        }
        if (full) break;
        // keep H > 0; with a band, the W best
        int32_t w = 0;
        for (int32_t x = 0; x < nB; ++x)
            if (B[x].H > 0) B[w++] = B[x];
        if (p.band > 0 && w > p.band) {
            // selection of the band's cells to the front
            for (int32_t y = 0; y < p.band; ++y) {
                int32_t best = y;
                for (int32_t x = y + 1; x < w; ++x)
                    if (hp_before(B[x], B[best])) best = x;
                if (best != y) {
                    const HpCell tmp = B[y];
                    B[y] = B[best];
                    B[best] = tmp;
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
            inside = (c.k >= q.k && c.k + c.s <= q.k + q.s) || (c.kr >= q.kr && c.kr + c.s <= q.kr + q.s);
        }
        if (!inside) A[w++] = c;
    }
    cnt[qi] = w;
}

// Result records of a batch in order: query qi's cells go to out[off[qi] ..].
__global__ void k_hapl_gather(const HpCell *__restrict__ cells, int64_t nq, int32_t cap,
                              const int32_t *__restrict__ cnt, const int64_t *__restrict__ off, int64_t qbase,
                              rb3_hapl_t *__restrict__ out) {
    const int64_t qi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (qi >= nq) return;
    const HpCell *A = cells + qi * 2 * (int64_t)cap;
    const int32_t c = cnt[qi];
    for (int32_t x = 0; x < c; ++x) {
        rb3_hapl_t r;
        r.k = A[x].k;
        r.krc = A[x].kr;
        r.s = A[x].s;
        r.score = A[x].H;
        r.qid = (int32_t)(qbase + qi);
        out[off[qi] + x] = r;
    }
}

template <class V>
static int hapl_run_v(Ctx &c, const V &view, const char *name, const uint8_t *d_codes, const int64_t *qlens,
                      int64_t nq, const rb3_hapl_opts &o, int64_t out_cap, rb3_hapl_t *d_out, int64_t *h_off,
                      int64_t *h_bad) {
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
    std::vector<int64_t> qoff(nq + 1);
    qoff[0] = 0;
    for (int64_t i = 0; i < nq; ++i) qoff[i + 1] = qoff[i] + qlens[i];
    const int64_t per = 2 * (int64_t)p.cap * (int64_t)sizeof(HpCell) + (int64_t)p.hcap * 4;
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(nq, HAPL_SCRATCH / per));
    DBuf dq, cells, hash, cnt, doff;
    RB3_ALLOC(dq, &c, (nq + 1) * sizeof(int64_t));
    RB3_ALLOC(cells, &c, (size_t)chunk * 2 * (size_t)p.cap * sizeof(HpCell));
    RB3_ALLOC(hash, &c, (size_t)chunk * (size_t)p.hcap * 4);
    RB3_ALLOC(cnt, &c, (size_t)chunk * sizeof(int32_t));
    RB3_ALLOC(doff, &c, (size_t)chunk * sizeof(int64_t));
    RB3_HIP(hipMemcpyAsync(dq.p, qoff.data(), (nq + 1) * sizeof(int64_t), hipMemcpyHostToDevice, c.stream));
    std::vector<int32_t> hc(chunk);
    h_off[0] = 0;
    for (int64_t q0 = 0; q0 < nq; q0 += chunk) {
        const int64_t m = std::min(chunk, nq - q0);
        RB3_HIP(hipMemsetAsync(hash.p, 0, (size_t)m * (size_t)p.hcap * 4, c.stream));
        RB3_LAUNCH(name, k_hapl<V>, grid_for(m, 64, 1 << 30), dim3(64), 0, c.stream, view, d_codes,
                   dq.as<int64_t>() + q0, m, p, cells.as<HpCell>(), hash.as<uint32_t>(), cnt.as<int32_t>());
        RB3_HIP(hipMemcpyAsync(hc.data(), cnt.p, m * sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
        RB3_HIP(hipStreamSynchronize(c.stream));
        for (int64_t i = 0; i < m; ++i) {
            if (hc[i] < 0) {
                *h_bad = q0 + i;
                return RB3_ELIMIT;
            }
            h_off[q0 + i + 1] = h_off[q0 + i] + hc[i];
        }
        if (h_off[q0 + m] <= out_cap && h_off[q0 + m] > h_off[q0]) {
            RB3_HIP(hipMemcpyAsync(doff.p, h_off + q0, m * sizeof(int64_t), hipMemcpyHostToDevice, c.stream));
            RB3_LAUNCH("hapl_gather", k_hapl_gather, grid_for(m, 64, 1 << 30), dim3(64), 0, c.stream,
                       cells.as<HpCell>(), m, p.cap, cnt.as<int32_t>(), doff.as<int64_t>(), q0, d_out);
            // the offsets and counts are rewritten by the next chunk
            RB3_HIP(hipStreamSynchronize(c.stream));
        }
    }
    return RB3_OK;
}

int hapl_run(Ctx &c, const DevIndex &ix, const RleView *rle, const uint8_t *d_codes, const int64_t *qlens,
             int64_t nq, const rb3_hapl_opts &o, int64_t out_cap, rb3_hapl_t *d_out, int64_t *h_off,
             int64_t *h_bad) {
    if (rle)
        return hapl_run_v(c, RleQView{*rle}, "hapl_rle", d_codes, qlens, nq, o, out_cap, d_out, h_off, h_bad);
    return hapl_run_v(c, PlainView{ix}, "hapl", d_codes, qlens, nq, o, out_cap, d_out, h_off, h_bad);
}

}  // namespace rb3
