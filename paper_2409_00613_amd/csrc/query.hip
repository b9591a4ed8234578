// Queries on the device-resident BWT: backward-search counts (Sec. 2.3) and
// SMEM finding (Sec. 2.6, Algorithm 4) over SA bi-interval extensions on the
// double-strand BWT (Sec. 2.5, Algorithm 3).
#include "views.h"

#include <vector>

namespace rb3 {

// [lo, hi) of each query. The search runs over the whole query even after
// the interval empties, because lo of the full query is part of the answer.
template <class V>
__global__ void k_count(V ix, const uint8_t *__restrict__ q, const int64_t *__restrict__ qoff, int64_t nq,
                        int64_t *__restrict__ lo_out, int64_t *__restrict__ hi_out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq) return;
    int64_t a0 = qoff[i], a1 = qoff[i + 1];
    int64_t lo = 0, hi = ix.size();
    for (int64_t t = a1 - 1; t >= a0; --t) ix.step(q[t], lo, hi);
    lo_out[i] = lo;
    hi_out[i] = hi;
}

int count_queries(Ctx &c, const DevIndex &ix, const uint8_t *d_q, const int64_t *d_qoff, int64_t nq,
                  int64_t *d_lo, int64_t *d_hi) {
    if (nq == 0) return RB3_OK;
    RB3_LAUNCH("count", k_count<PlainView>, grid_for(nq, 256, 1 << 30), dim3(256), 0, c.stream, PlainView{ix},
               d_q, d_qoff, nq, d_lo, d_hi);
    return RB3_OK;
}

int count_queries_rle(Ctx &c, const RleView &v, const uint8_t *d_q, const int64_t *d_qoff, int64_t nq,
                      int64_t *d_lo, int64_t *d_hi) {
    if (nq == 0) return RB3_OK;
    RB3_LAUNCH("count_rle", k_count<RleQView>, grid_for(nq, 256, 1 << 30), dim3(256), 0, c.stream, RleQView{v},
               d_q, d_qoff, nq, d_lo, d_hi);
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
template <class V>
__device__ __forceinline__ BiInt backward_ext(const V &ix, const BiInt &x, int a) {
    int64_t p0[6], p1[6];
    ix.pi2(x.k, x.k + x.s, p0, p1);
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

// ---------------------------------------------------------------------------
// Algorithm 4 over query segments
// ---------------------------------------------------------------------------
//
// A query is cut into segments of S positions (S from the batch size, see
// smem_run). Algorithm 4 is run
// from each segment's first position and stops once its start passes the
// segment's end (forward extensions still read past it). Started at an
// arbitrary position c, the algorithm reports exactly the SMEMs of length
// >= min_len whose start is at least c, except that its very first report
// may be [c, e(c)) although e(c) <= e(c-1): that one is contained in an
// earlier SMEM, which an earlier segment reported, so it is dropped when its
// end does not exceed the largest end reported by the earlier segments of
// the query (k_smem_fix).
//
// Readings where the printed algorithm is silent: the interval reported with
// [i, e) is the one before the failing forward extension; if the forward
// loop reaches the end of P, e = |P| and the search stops; when the second
// backward loop finishes without a failure the next start is i + 1.

struct Seg {
    int64_t qoff;  // offset of the query's codes
    int32_t qlen;  // query length
    int32_t qid;
    int32_t c0, c1;  // segment [c0, c1) of the query
};

enum { PH_START = 0, PH_BACK1 = 1, PH_FWD = 2, PH_BACK2 = 3 };

constexpr int SMEM_WG = 256;

// One lane per segment, persistent. Each turn of the loop every busy lane
// performs one extension (two rank-all block reads); a lane that finishes
// its segment takes the next one from a shared queue.
template <class V>
__global__ void __launch_bounds__(SMEM_WG) k_smem_seg(V ix, const uint8_t *__restrict__ q,
                                                      const Seg *__restrict__ segs, int64_t nseg, int32_t ell,
                                                      int64_t smin, uint32_t *__restrict__ qhead,
                                                      rb3_smem_t *__restrict__ tmp, int64_t cap,
                                                      unsigned long long *__restrict__ total,
                                                      uint32_t *__restrict__ segcnt, int64_t *__restrict__ segfirst,
                                                      int64_t *__restrict__ seglast,
                                                      unsigned long long *__restrict__ exts) {
    const int lane = threadIdx.x & 63;
    const BiInt empty = {0, 0, ix.size()};
    bool busy = false, exhausted = false;
    int64_t g = 0;
    const uint8_t *P = q;
    int64_t L = 0, c1 = 0, i = 0, j = 0;
    int phase = PH_START;
    BiInt x = empty;
    uint32_t nrec = 0;
    int64_t first_end = -1, last_end = -1;
    uint64_t nexts = 0, nblks = 0;
    for (;;) {
        uint64_t idle = __ballot(!busy);
        if (idle && !exhausted) {
            int first = __ffsll((unsigned long long)idle) - 1;
            uint32_t nidle = (uint32_t)__popcll(idle);
            uint32_t base = 0;
            if (lane == first) base = atomicAdd(qhead, nidle);
            base = __shfl(base, first);
            if ((int64_t)base + nidle >= nseg) exhausted = true;
            if (!busy) {
                int64_t slot = (int64_t)base + __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                if (slot < nseg) {
                    Seg sg = segs[slot];
                    g = slot;
                    P = q + sg.qoff;
                    L = sg.qlen;
                    i = sg.c0;
                    c1 = sg.c1;
                    phase = PH_START;
                    nrec = 0;
                    first_end = last_end = -1;
                    busy = true;
                }
            }
        }
        if (__ballot(busy) == 0) break;
        bool emit = false, done = false;
        int64_t em_start = 0, em_end = 0;
        BiInt em_x = empty;
        if (busy && phase == PH_START) {
            if (i >= c1 || i + ell > L) {
                done = true;
            } else {
                x = empty;
                j = i + ell - 1;
                phase = PH_BACK1;
            }
        }
        // every phase extends by one symbol; a forward extension is a
        // backward one of the reverse-complement interval (Algorithm 3), so
        // all busy lanes share one extension call and its block reads
        const bool fwd = phase == PH_FWD;
        const bool need = busy && !done && !(fwd && j >= L);
        BiInt y = x;
        if (need) {
            const int a = P[j];
            const BiInt in = fwd ? BiInt{x.kr, x.k, x.s} : x;
            const BiInt z = backward_ext(ix, in, fwd ? comp_sym(a) : a);
            y = fwd ? BiInt{z.kr, z.k, z.s} : z;
            ++nexts;
            // index blocks the extension read (rank-all at k and k + s)
            nblks += ix.units(in.k, in.k + in.s);
        }
        if (busy && !done) {
            if (phase == PH_BACK1) {
                x = y;
                if (x.s < smin) {
                    i = j + 1;
                    phase = PH_START;
                } else if (j == i) {
                    j = i + ell;
                    phase = PH_FWD;
                } else {
                    --j;
                }
            } else if (phase == PH_FWD) {
                const bool stop = j >= L || y.s < smin;
                if (stop) {
                    emit = true;
                    em_start = i;
                    em_end = j;
                    em_x = x;
                    if (j >= L) {
                        done = true;  // an SMEM reaching the end: no later start can add one
                    } else {
                        x = empty;
                        phase = PH_BACK2;  // j stays at e
                    }
                } else {
                    x = y;
                    ++j;
                }
            } else if (phase == PH_BACK2) {
                x = y;
                if (x.s < smin) {
                    i = j + 1;
                    phase = PH_START;
                } else if (j == i + 1) {
                    i = i + 1;
                    phase = PH_START;
                } else {
                    --j;
                }
            }
        }
        uint64_t em = __ballot(emit);
        if (em) {
            int first = __ffsll((unsigned long long)em) - 1;
            unsigned long long base = 0;
            if (lane == first) base = atomicAdd(total, (unsigned long long)__popcll(em));
            base = __shfl(base, first);
            if (emit) {
                unsigned long long slot = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(em >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)em, 0u));
                if ((int64_t)slot < cap) {
                    rb3_smem_t r;
                    r.start = em_start;
                    r.end = em_end;
                    r.occ = em_x.s;
                    r.k = em_x.k;
                    r.krc = em_x.kr;
                    r.qid = (int32_t)g;  // segment; k_smem_order restores the query id
                    r.pad = (int32_t)nrec;
                    tmp[slot] = r;
                }
                if (nrec == 0) first_end = em_end;
                last_end = em_end;
                ++nrec;
            }
        }
        if (done) {
            segcnt[g] = nrec;
            segfirst[g] = first_end;
            seglast[g] = last_end;
            busy = false;
        }
    }
    uint64_t t = nexts, b = nblks;
    for (int o = 32; o > 0; o >>= 1) {
        t += __shfl_xor(t, o);
        b += __shfl_xor(b, o);
    }
    if (lane == 0 && t) {
        atomicAdd(&exts[0], (unsigned long long)t);
        atomicAdd(&exts[1], (unsigned long long)b);
    }
}

// Per segment: whether its first report is contained in an SMEM of an
// earlier segment of the same query (its end does not pass the largest end
// reported before it in the query), and how many reports it keeps. One wave
// per query walks its segments 64 at a time with a running maximum.
__global__ void k_smem_fix(const int64_t *__restrict__ qseg, int64_t nq, const uint32_t *__restrict__ segcnt,
                           const int64_t *__restrict__ segfirst, const int64_t *__restrict__ seglast,
                           uint32_t *__restrict__ drop, uint32_t *__restrict__ kept) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t qq = wave; qq < nq; qq += nwaves) {
        const int64_t s0 = qseg[qq], s1 = qseg[qq + 1];
        int64_t carry = -1;  // largest end reported by the segments before this run
        for (int64_t base = s0; base < s1; base += 64) {
            const int64_t g = base + lane;
            const bool in = g < s1;
            const int64_t v = in ? seglast[g] : -1;
            int64_t incl = v;
            for (int d = 1; d < 64; d <<= 1) {
                const int64_t t = __shfl_up(incl, d);
                if (lane >= d && t > incl) incl = t;
            }
            int64_t excl = __shfl_up(incl, 1);
            if (lane == 0) excl = -1;
            if (carry > excl) excl = carry;
            if (in) {
                const uint32_t n = segcnt[g];
                const uint32_t d = (n > 0 && segfirst[g] <= excl) ? 1u : 0u;
                drop[g] = d;
                kept[g] = n - d;
            }
            const int64_t tot = __shfl(incl, 63);
            if (tot > carry) carry = tot;
        }
    }
}

// Query offsets: out_off[q] = offset of the first segment at or after the
// query's first one (segments of a query are consecutive).
__global__ void k_smem_qoff(const int64_t *__restrict__ qseg, int64_t nq, const uint32_t *__restrict__ segoff,
                            int64_t *__restrict__ out_off) {
    for (int64_t qq = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; qq <= nq;
         qq += (int64_t)gridDim.x * blockDim.x)
        out_off[qq] = segoff[qseg[qq]];
}

// Put the kept reports in order: segment order, then report order.
__global__ void k_smem_order(const rb3_smem_t *__restrict__ tmp, int64_t total, const Seg *__restrict__ segs,
                             const uint32_t *__restrict__ segoff, const uint32_t *__restrict__ drop,
                             rb3_smem_t *__restrict__ out) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < total;
         r += (int64_t)gridDim.x * blockDim.x) {
        rb3_smem_t x = tmp[r];
        int64_t g = x.qid;
        uint32_t d = drop[g];
        if (d && x.pad == 0) continue;
        int64_t pos = (int64_t)segoff[g] + x.pad - d;
        x.qid = segs[g].qid;
        x.pad = 0;
        out[pos] = x;
    }
}

template <class V>
static int smem_run_v(Ctx &c, const V &ix, const char *kname, const uint8_t *d_q, const int64_t *qlens, int64_t nq,
                      int32_t min_len, int64_t min_occ, int64_t out_cap, rb3_smem_t *d_out, int64_t *d_out_off,
                      int64_t *h_kept, int64_t *h_exts) {
    // segment table: segments short enough that the batch fills the GPU
    // with lanes. Each segment repeats some work at its start (the first
    // min_len-symbol check, and the tail of an SMEM begun in the segment
    // before), so segments stay long when the batch alone fills the GPU and
    // shrink to SMEM_SEG_MIN for small batches, where latency matters.
    int64_t bases = 0;
    for (int64_t qq = 0; qq < nq; ++qq) bases += qlens[qq];
    const int64_t target = c.smem_segs > 0 ? c.smem_segs : SMEM_TARGET_SEGS;
    const int64_t smin = c.smem_seg_min > 0 ? c.smem_seg_min : SMEM_SEG_MIN;
    int64_t S = bases / target;
    S = S < smin ? smin : (S > SMEM_SEG ? SMEM_SEG : S);
    if (c.smem_seg_fixed > 0) {
        S = c.smem_seg_fixed;
    } else if (c.smem_seg_fixed == 0) {
        const int64_t t = tuned_smem_segment(c.device, ix.size(), bases, nq);
        if (t > 0) S = t;
    }
    std::vector<Seg> segs;
    std::vector<int64_t> qseg(nq + 1);
    int64_t off = 0;
    for (int64_t qq = 0; qq < nq; ++qq) {
        qseg[qq] = (int64_t)segs.size();
        int64_t L = qlens[qq];
        if (L >= min_len) {
            for (int64_t c0 = 0; c0 < L; c0 += S) {
                Seg sg;
                sg.qoff = off;
                sg.qlen = (int32_t)L;
                sg.qid = (int32_t)qq;
                sg.c0 = (int32_t)c0;
                sg.c1 = (int32_t)(c0 + S < L ? c0 + S : L);
                segs.push_back(sg);
            }
        }
        off += L;
    }
    int64_t nseg = (int64_t)segs.size();
    qseg[nq] = nseg;
    // every segment drops at most one report, so out_cap + nseg raw reports
    // hold all kept ones whenever they fit in out_cap
    const int64_t cap = out_cap + nseg;
    DBuf d_segs, d_qseg, qh, tot, cnt, first, last, drop, kept, segoff, ext, tmpb;
    RB3_ALLOC(tmpb, &c, (cap > 0 ? cap : 1) * sizeof(rb3_smem_t));
    rb3_smem_t *d_tmp = tmpb.as<rb3_smem_t>();
    RB3_ALLOC(d_segs, &c, (nseg > 0 ? nseg : 1) * sizeof(Seg));
    RB3_ALLOC(d_qseg, &c, (nq + 1) * sizeof(int64_t));
    RB3_ALLOC(qh, &c, sizeof(uint32_t));
    RB3_ALLOC(tot, &c, sizeof(unsigned long long));
    RB3_ALLOC(ext, &c, 2 * sizeof(unsigned long long));
    RB3_ALLOC(cnt, &c, (nseg + 1) * sizeof(uint32_t));
    RB3_ALLOC(first, &c, (nseg + 1) * sizeof(int64_t));
    RB3_ALLOC(last, &c, (nseg + 1) * sizeof(int64_t));
    RB3_ALLOC(drop, &c, (nseg + 1) * sizeof(uint32_t));
    RB3_ALLOC(kept, &c, (nseg + 1) * sizeof(uint32_t));
    RB3_ALLOC(segoff, &c, (nseg + 1) * sizeof(uint32_t));
    if (nseg > 0)
        RB3_HIP(hipMemcpyAsync(d_segs.p, segs.data(), nseg * sizeof(Seg), hipMemcpyHostToDevice, c.stream));
    RB3_HIP(hipMemcpyAsync(d_qseg.p, qseg.data(), (nq + 1) * sizeof(int64_t), hipMemcpyHostToDevice, c.stream));
    RB3_HIP(hipMemsetAsync(qh.p, 0, sizeof(uint32_t), c.stream));
    RB3_HIP(hipMemsetAsync(tot.p, 0, sizeof(unsigned long long), c.stream));
    RB3_HIP(hipMemsetAsync(ext.p, 0, 2 * sizeof(unsigned long long), c.stream));
    RB3_HIP(hipMemsetAsync(kept.p, 0, (nseg + 1) * sizeof(uint32_t), c.stream));
    if (nseg > 0) {
        int64_t wgs = (nseg + SMEM_WG - 1) / SMEM_WG;
        if (wgs > 2048) wgs = 2048;
        RB3_LAUNCH(kname, k_smem_seg<V>, dim3((unsigned)wgs), dim3(SMEM_WG), 0, c.stream, ix, d_q,
                   d_segs.as<Seg>(), nseg, min_len, min_occ, qh.as<uint32_t>(), d_tmp, cap,
                   tot.as<unsigned long long>(), cnt.as<uint32_t>(), first.as<int64_t>(), last.as<int64_t>(),
                   ext.as<unsigned long long>());
        RB3_LAUNCH("smem_fix", k_smem_fix, grid_for(nq, 4, 1 << 20), dim3(256), 0, c.stream,
                   d_qseg.as<int64_t>(), nq, cnt.as<uint32_t>(), first.as<int64_t>(), last.as<int64_t>(),
                   drop.as<uint32_t>(), kept.as<uint32_t>());
    }
    RB3_TRY(scan_u32(c, kept.as<uint32_t>(), segoff.as<uint32_t>(), nseg + 1, false, false, nullptr));
    RB3_LAUNCH("smem_qoff", k_smem_qoff, grid_for(nq + 1, 256, 1 << 20), dim3(256), 0, c.stream,
               d_qseg.as<int64_t>(), nq, segoff.as<uint32_t>(), d_out_off);
    unsigned long long htot = 0, hext[2] = {0, 0};
    int64_t hkept = 0;
    RB3_HIP(hipMemcpyAsync(&htot, tot.p, sizeof(htot), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipMemcpyAsync(hext, ext.p, sizeof(hext), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipMemcpyAsync(&hkept, d_out_off + nq, sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipStreamSynchronize(c.stream));
    *h_kept = hkept;
    h_exts[0] = (int64_t)hext[0];
    h_exts[1] = (int64_t)hext[1];
    if ((int64_t)htot <= cap && hkept <= out_cap && htot > 0)
        RB3_LAUNCH("smem_order", k_smem_order, grid_for((int64_t)htot, 256 * 4), dim3(256), 0, c.stream, d_tmp,
                   (int64_t)htot, d_segs.as<Seg>(), segoff.as<uint32_t>(), drop.as<uint32_t>(), d_out);
    return RB3_OK;
}

int smem_run(Ctx &c, const DevIndex &ix, const uint8_t *d_q, const int64_t *qlens, int64_t nq, int32_t min_len,
             int64_t min_occ, int64_t out_cap, rb3_smem_t *d_out, int64_t *d_out_off, int64_t *h_kept,
             int64_t *h_exts) {
    return smem_run_v(c, PlainView{ix}, "smem", d_q, qlens, nq, min_len, min_occ, out_cap, d_out, d_out_off, h_kept,
                      h_exts);
}

int smem_run_rle(Ctx &c, const RleView &v, const uint8_t *d_q, const int64_t *qlens, int64_t nq, int32_t min_len,
                 int64_t min_occ, int64_t out_cap, rb3_smem_t *d_out, int64_t *d_out_off, int64_t *h_kept,
                 int64_t *h_exts) {
    return smem_run_v(c, RleQView{v}, "smem_rle", d_q, qlens, nq, min_len, min_occ, out_cap, d_out, d_out_off,
                      h_kept, h_exts);
}

}  // namespace rb3
