// Locating suffixes with suffix-array samples (Sec. 2.4, Algorithm 2).
//
// The samples are kept by text position (a suffix whose position in its
// merge batch is a multiple of the sampling distance s, or that starts its
// strand), so from any row at most s - 1 LF steps reach a sampled row, and a
// walk never has to cross a sentinel: the row of a strand's first suffix is
// itself sampled. A sampled row's value is (strand, offset); a row reached
// after k steps from row i gives i the position (strand, offset + k).
#include "rb3_internal.h"

namespace rb3 {

// Symbol at row r of the BWT from its block.
__device__ __forceinline__ int block_symbol(const Block &B, int64_t r) {
    const int o = (int)(r & (BLK_SYMS - 1));
    const uint64_t p0 = o < 64 ? u64_lo(B.q0) : u64_hi(B.q0);
    const uint64_t p1 = o < 64 ? u64_lo(B.q1) : u64_hi(B.q1);
    const uint64_t p2 = o < 64 ? u64_lo(B.q2) : u64_hi(B.q2);
    const int b = o & 63;
    return (int)(((p0 >> b) & 1ull) | (((p1 >> b) & 1ull) << 1) | (((p2 >> b) & 1ull) << 2));
}

// One lane per row. Each step requests the row's sample word and its BWT
// block together; a sampled row ends the walk, otherwise LF moves to the
// suffix one position earlier.
__global__ void k_locate(DevIndex ix, DevSmp sm, const int64_t *__restrict__ rows, int64_t n,
                         int64_t *__restrict__ strand, int64_t *__restrict__ off, int32_t *__restrict__ err,
                         unsigned long long *__restrict__ steps) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    uint64_t my_steps = 0;
    if (i < n) {
        int64_t r = rows[i];
        int64_t st = -1, of = -1;
        if (r >= 0 && r < ix.n) {
            for (int64_t k = 0; k < (int64_t)sm.rate; ++k) {
                const Block B = load_block(ix.blk, r >> BLK_SHIFT);
                int64_t idx = 0;
                if (smp_rank(sm, r, &idx)) {
                    if (idx < sm.nsmp) {
                        const uint64_t v = sm.val[idx];
                        st = (int64_t)(v >> SMP_ID_SHIFT);
                        of = (int64_t)(v & SMP_OFF_MASK) + k;
                    }
                    break;
                }
                const int c = block_symbol(B, r);
                if (c < 1 || c > 5) break;  // a sentinel row is always sampled
                r = pi_from_block(ix, B, c, r);
                ++my_steps;
            }
        }
        if (st < 0) atomicOr(err, 1);
        strand[i] = st;
        off[i] = of;
    }
    uint64_t t = my_steps;
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if ((threadIdx.x & 63) == 0 && t) atomicAdd(steps, (unsigned long long)t);
}

int locate_rows(Ctx &c, const DevIndex &ix, const DevSmp &sm, const int64_t *d_rows, int64_t n,
                int64_t *d_strand, int64_t *d_off, int32_t *d_err, unsigned long long *d_steps) {
    if (n == 0) return RB3_OK;
    RB3_LAUNCH("locate", k_locate, grid_for(n, 256, 1 << 30), dim3(256), 0, c.stream, ix, sm, d_rows, n, d_strand,
               d_off, d_err, d_steps);
    return RB3_OK;
}

// Locate1 (Algorithm 2): one occurrence in [lo, hi). Intervals (l, h, o)
// are kept in a small per-lane list in LDS and taken largest first; an
// interval holding a sampled row ends the search with that sample's value
// plus o; otherwise its backward extensions by A, C, G, T, N (from rank-all
// at l and at h) join the list. The test for a sentinel in the interval
// that the printed procedure makes is covered by the sample test, since a
// row whose BWT symbol is $ starts its strand and is sampled. When the list
// is full, a new interval replaces the smallest one if it is larger. Every
// row reaches a sample within s - 1 steps, so the search ends within s - 1
// levels below any interval it keeps.
constexpr int L1_WG = 128;
constexpr int L1_CAP = 8;

__global__ void __launch_bounds__(L1_WG) k_locate1(DevIndex ix, DevSmp sm, const int64_t *__restrict__ qlo,
                                                   const int64_t *__restrict__ qhi, int64_t n,
                                                   int64_t *__restrict__ strand, int64_t *__restrict__ off,
                                                   int32_t *__restrict__ err, unsigned long long *__restrict__ steps) {
    __shared__ int64_t hl[L1_CAP][L1_WG];
    __shared__ int64_t hh[L1_CAP][L1_WG];
    __shared__ int32_t ho[L1_CAP][L1_WG];
    const int t = threadIdx.x;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + t;
    uint64_t my_steps = 0;
    if (i < n) {
        const int64_t lo = qlo[i], hi = qhi[i];
        int64_t st = -1, of = -1;
        bool bad = false;
        if (lo < 0 || hi > ix.n || lo > hi) {
            bad = true;
        } else if (lo < hi) {
            int nh = 1;
            hl[0][t] = lo;
            hh[0][t] = hi;
            ho[0][t] = 0;
            // a generous bound: each kept interval is at most s - 1 levels
            // above a sample, and each level adds at most 5 intervals
            const int64_t limit = (int64_t)(sm.rate + 1) * 5 * L1_CAP + 16;
            int64_t iter = 0;
            while (nh > 0 && st < 0) {
                if (++iter > limit) {
                    bad = true;
                    break;
                }
                int j = 0;
                int64_t best = hh[0][t] - hl[0][t];
                for (int q = 1; q < nh; ++q) {
                    const int64_t w = hh[q][t] - hl[q][t];
                    if (w > best) {
                        best = w;
                        j = q;
                    }
                }
                const int64_t l = hl[j][t], h = hh[j][t];
                const int32_t o = ho[j][t];
                --nh;
                hl[j][t] = hl[nh][t];
                hh[j][t] = hh[nh][t];
                ho[j][t] = ho[nh][t];
                int64_t rl = 0, rh = 0;
                smp_rank(sm, l, &rl);
                smp_rank(sm, h, &rh);
                if (rh > rl) {
                    if (rl < sm.nsmp) {
                        const uint64_t v = sm.val[rl];
                        st = (int64_t)(v >> SMP_ID_SHIFT);
                        of = (int64_t)(v & SMP_OFF_MASK) + o;
                    } else {
                        bad = true;
                    }
                    break;
                }
                int64_t p0[6], p1[6];
                pi_all2(ix, l, h, p0, p1);
                ++my_steps;
                for (int a = 1; a <= 5; ++a) {
                    const int64_t nl = p0[a], nhh = p1[a];
                    if (nhh <= nl) continue;
                    int slot = nh;
                    if (nh == L1_CAP) {
                        // replace the smallest kept interval if this one is larger
                        int sj = 0;
                        int64_t sw = hh[0][t] - hl[0][t];
                        for (int q = 1; q < L1_CAP; ++q) {
                            const int64_t w = hh[q][t] - hl[q][t];
                            if (w < sw) {
                                sw = w;
                                sj = q;
                            }
                        }
                        if (nhh - nl <= sw) continue;
                        slot = sj;
                    } else {
                        ++nh;
                    }
                    hl[slot][t] = nl;
                    hh[slot][t] = nhh;
                    ho[slot][t] = o + 1;
                }
            }
            if (st < 0) bad = true;
        }
        if (bad) atomicOr(err, 1);
        strand[i] = st;
        off[i] = of;
    }
    uint64_t tot = my_steps;
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
    if ((t & 63) == 0 && tot) atomicAdd(steps, (unsigned long long)tot);
}

int locate_one(Ctx &c, const DevIndex &ix, const DevSmp &sm, const int64_t *d_lo, const int64_t *d_hi,
               int64_t n, int64_t *d_strand, int64_t *d_off, int32_t *d_err, unsigned long long *d_steps) {
    if (n == 0) return RB3_OK;
    RB3_LAUNCH("locate1", k_locate1, grid_for(n, L1_WG, 1 << 30), dim3(L1_WG), 0, c.stream, ix, sm, d_lo, d_hi,
               n, d_strand, d_off, d_err, d_steps);
    return RB3_OK;
}

}  // namespace rb3
