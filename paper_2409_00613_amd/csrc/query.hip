// Queries on the device-resident BWT: backward-search counts (Sec. 2.3) and
// SMEM finding (Sec. 2.6, Algorithm 4) over SA bi-interval extensions on the
// double-strand BWT (Sec. 2.5, Algorithm 3).
#include "rb3_internal.h"

namespace rb3 {

// [lo, hi) of each query. The search runs over the whole query even after
// the interval empties, because lo of the full query is part of the answer.
__global__ void k_count(DevIndex ix, const uint8_t *__restrict__ q, const int64_t *__restrict__ qoff,
                        int64_t nq, int64_t *__restrict__ lo_out, int64_t *__restrict__ hi_out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq) return;
    int64_t a0 = qoff[i], a1 = qoff[i + 1];
    int64_t lo = 0, hi = ix.n;
    for (int64_t t = a1 - 1; t >= a0; --t) {
        int a = q[t];
        if (lo == hi) {
            lo = pi_sym(ix, a, lo);
            hi = lo;
        } else if ((lo >> BLK_SHIFT) == (hi >> BLK_SHIFT)) {
            Block B = load_block(ix.blk, lo >> BLK_SHIFT);
            lo = pi_from_block(ix, B, a, lo);
            hi = pi_from_block(ix, B, a, hi);
        } else {
            lo = pi_sym(ix, a, lo);
            hi = pi_sym(ix, a, hi);
        }
    }
    lo_out[i] = lo;
    hi_out[i] = hi;
}

int count_queries(Ctx &c, const DevIndex &ix, const uint8_t *d_q, const int64_t *d_qoff, int64_t nq,
                  int64_t *d_lo, int64_t *d_hi) {
    if (nq == 0) return RB3_OK;
    RB3_LAUNCH("count", k_count, grid_for(nq, 256, 1 << 30), dim3(256), 0, c.stream, ix, d_q, d_qoff, nq,
               d_lo, d_hi);
    return RB3_OK;
}

// ---------------------------------------------------------------------------
// SMEM
// ---------------------------------------------------------------------------

struct BiInt {
    int64_t k, kr, s;  // lo(P), lo(rc P), occ(P)
};

__device__ __forceinline__ int comp_sym(int c) { return (c == 0 || c == 5) ? c : 5 - c; }

// Algorithm 3, BackwardExt: the bi-interval of aP from that of P.
__device__ __forceinline__ BiInt backward_ext(const DevIndex &ix, const BiInt &x, int a) {
    int64_t p0[6], p1[6];
    pi_all(ix, x.k, p0);
    pi_all(ix, x.k + x.s, p1);
    BiInt r;
    int64_t kr = x.kr;
    int abar = comp_sym(a);
    for (int b = 0; b < abar; ++b) {
        int bb = comp_sym(b);
        kr += p1[bb] - p0[bb];  // occ(comp(b) P)
    }
    r.kr = kr;
    r.s = p1[a] - p0[a];
    r.k = p0[a];
    return r;
}

// Algorithm 3, ForwardExt: the bi-interval of Pa, by extending rc(P)
// backwards with comp(a) and swapping.
__device__ __forceinline__ BiInt forward_ext(const DevIndex &ix, const BiInt &x, int a) {
    BiInt y;
    y.k = x.kr;
    y.kr = x.k;
    y.s = x.s;
    BiInt z = backward_ext(ix, y, comp_sym(a));
    BiInt r;
    r.k = z.kr;
    r.kr = z.k;
    r.s = z.s;
    return r;
}

__device__ __forceinline__ void emit_smem(rb3_smem_t *out, int64_t cap, unsigned long long *total, int64_t qid,
                                          int32_t seq, int64_t st, int64_t en, const BiInt &x) {
    unsigned long long slot = atomicAdd(total, 1ull);
    if ((int64_t)slot < cap) {
        rb3_smem_t r;
        r.start = st;
        r.end = en;
        r.occ = x.s;
        r.k = x.k;
        r.krc = x.kr;
        r.qid = (int32_t)qid;
        r.pad = seq;
        out[slot] = r;
    }
}

// Algorithm 4, one query per lane. Readings where the printed algorithm is
// silent: the interval reported with [i, e) is the one before the failing
// forward extension; if the forward loop reaches the end of P, e = |P| and
// the search stops; when the second backward loop finishes without a
// failure the next start is i + 1.
__global__ void k_smem(DevIndex ix, const uint8_t *__restrict__ q, const int64_t *__restrict__ qoff,
                       int64_t nq, int32_t ell, int64_t smin, rb3_smem_t *__restrict__ out, int64_t cap,
                       unsigned long long *__restrict__ total, uint32_t *__restrict__ cnt) {
    int64_t qi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (qi >= nq) return;
    const uint8_t *P = q + qoff[qi];
    const int64_t L = qoff[qi + 1] - qoff[qi];
    int32_t found = 0;
    int64_t i = 0;
    const BiInt empty = {0, 0, ix.n};
    while (i < L) {
        if (i + ell > L) break;
        BiInt x = empty;
        int64_t next = -1;
        for (int64_t j = i + ell - 1; j >= i; --j) {
            x = backward_ext(ix, x, P[j]);
            if (x.s < smin) {
                next = j + 1;
                break;
            }
        }
        if (next >= 0) {
            i = next;
            continue;
        }
        int64_t j = i + ell;
        for (; j < L; ++j) {
            BiInt y = forward_ext(ix, x, P[j]);
            if (y.s < smin) break;
            x = y;
        }
        int64_t e = j;
        emit_smem(out, cap, total, qi, found, i, e, x);
        ++found;
        if (e >= L) break;
        x = empty;
        next = i + 1;
        for (j = e; j >= i + 1; --j) {
            x = backward_ext(ix, x, P[j]);
            if (x.s < smin) {
                next = j + 1;
                break;
            }
        }
        i = next;
    }
    cnt[qi] = (uint32_t)found;
}

// Put the records of each query in order: out[off[qid] + seq].
__global__ void k_smem_order(const rb3_smem_t *__restrict__ tmp, int64_t total,
                             const uint32_t *__restrict__ off, rb3_smem_t *__restrict__ out) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < total;
         r += (int64_t)gridDim.x * blockDim.x) {
        rb3_smem_t x = tmp[r];
        int64_t pos = (int64_t)off[x.qid] + x.pad;
        x.pad = 0;
        out[pos] = x;
    }
}

// Full SMEM call: unordered records into tmp (capacity cap), per-query counts,
// offsets, ordered copy into out. Returns the total in *h_total.
int smem_run(Ctx &c, const DevIndex &ix, const uint8_t *d_q, const int64_t *d_qoff, int64_t nq,
             int32_t min_len, int64_t min_occ, int64_t cap, rb3_smem_t *d_tmp, rb3_smem_t *d_out,
             uint32_t *d_cnt, uint32_t *d_off, unsigned long long *d_total, int64_t *h_total) {
    RB3_HIP(hipMemsetAsync(d_total, 0, sizeof(unsigned long long), c.stream));
    if (nq > 0)
        RB3_LAUNCH("smem", k_smem, grid_for(nq, 64, 1 << 30), dim3(64), 0, c.stream, ix, d_q, d_qoff, nq,
                   min_len, min_occ, d_tmp, cap, d_total, d_cnt);
    unsigned long long tot = 0;
    RB3_HIP(hipMemcpyAsync(&tot, d_total, sizeof(tot), hipMemcpyDeviceToHost, c.stream));
    RB3_TRY(scan_u32(c, d_cnt, d_off, nq + 1, false, false, nullptr));
    RB3_HIP(hipStreamSynchronize(c.stream));
    *h_total = (int64_t)tot;
    if ((int64_t)tot <= cap && tot > 0)
        RB3_LAUNCH("smem_order", k_smem_order, grid_for((int64_t)tot, 256 * 4), dim3(256), 0, c.stream, d_tmp,
                   (int64_t)tot, d_off, d_out);
    return RB3_OK;
}

}  // namespace rb3
