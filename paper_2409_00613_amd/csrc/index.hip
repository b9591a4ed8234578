// Symbol encoding, double-strand expansion, packing of the BWT into 64-byte
// blocks and the device-wide scan that writes occurrence checkpoints.
#include "rb3_internal.h"

namespace rb3 {

// Watson-Crick complement on codes (Sec. 2.5): A<->T, C<->G, N<->N, $<->$.
__device__ __forceinline__ uint8_t comp_code(int c) { return (uint8_t)(c == 5 ? 5 : (c == 0 ? 0 : 5 - c)); }

// Each thread encodes a run of 16 input bytes. String j (length L, input
// offset in_off[j]) becomes, at output offset k*(in_off[j] + j):
//   P_j $ [rc(P_j) $]          (k = 2 with both strands, else k = 1)
// so the sentinel of every strand is stored as code 0 right after it.
__global__ void k_encode_strands(const uint8_t *__restrict__ seq, const int64_t *__restrict__ in_off,
                                 int64_t m_in, int64_t total, int32_t both, uint8_t *__restrict__ Q,
                                 int32_t *__restrict__ err) {
    const int64_t RUN = 16;
    int64_t nruns = (total + RUN - 1) / RUN;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nruns;
         r += (int64_t)gridDim.x * blockDim.x) {
        int64_t i0 = r * RUN, i1 = i0 + RUN < total ? i0 + RUN : total;
        // largest j with in_off[j] <= i0
        int64_t lo = 0, hi = m_in;
        while (hi - lo > 1) {
            int64_t mid = (lo + hi) >> 1;
            if (in_off[mid] <= i0) lo = mid; else hi = mid;
        }
        int64_t j = lo;
        int64_t s0 = in_off[j], s1 = in_off[j + 1];
        int bad = 0;
        for (int64_t i = i0; i < i1; ++i) {
            while (i >= s1) {
                ++j;
                s0 = s1;
                s1 = in_off[j + 1];
            }
            int64_t t = i - s0, L = s1 - s0;
            int c = ascii_code(seq[i]);
            if (c < 0) {
                bad = 1;
                c = 1;
            }
            int64_t base = (both ? 2 : 1) * (s0 + j);
            Q[base + t] = (uint8_t)c;
            if (t == L - 1) Q[base + L] = 0;
            if (both) {
                Q[base + L + 1 + (L - 1 - t)] = comp_code(c);
                if (t == 0) Q[base + 2 * L + 1] = 0;
            }
        }
        if (bad) atomicOr(err, 1);
    }
}

__global__ void k_encode_plain(const uint8_t *__restrict__ seq, int64_t total, uint8_t *__restrict__ out,
                               int32_t *__restrict__ err) {
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int c = ascii_code(seq[i]);
        if (c < 0) {
            bad = 1;
            c = 1;
        }
        out[i] = (uint8_t)c;
    }
    if (bad) atomicOr(err, 1);
}

__global__ void k_check_codes(const uint8_t *__restrict__ codes, int64_t n, int32_t *__restrict__ err) {
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        bad |= codes[i] > 5;
    if (bad) atomicOr(err, 1);
}

int encode_strands(Ctx &c, const uint8_t *d_seq, const int64_t *lens, int64_t n_in, int32_t both,
                   uint8_t *d_Q, int64_t n_out, int32_t *d_err) {
    std::vector<int64_t> off(n_in + 1);
    off[0] = 0;
    for (int64_t j = 0; j < n_in; ++j) off[j + 1] = off[j] + lens[j];
    int64_t total = off[n_in];
    (void)n_out;
    DBuf d_off;
    RB3_ALLOC(d_off, &c, (n_in + 1) * sizeof(int64_t));
    RB3_HIP(hipMemcpyAsync(d_off.p, off.data(), (n_in + 1) * sizeof(int64_t), hipMemcpyHostToDevice,
                           c.stream));
    int64_t runs = (total + 15) / 16;
    RB3_LAUNCH("encode_strands", k_encode_strands, grid_for(runs, 256), dim3(256), 0, c.stream,
               d_seq, d_off.as<int64_t>(), n_in, total, both, d_Q, d_err);
    return RB3_OK;
}

int encode_plain(Ctx &c, const uint8_t *d_seq, const int64_t *lens, int64_t n_in, uint8_t *d_codes,
                 int64_t total, int32_t *d_err) {
    (void)lens;
    (void)n_in;
    if (total == 0) return RB3_OK;
    RB3_LAUNCH("encode_plain", k_encode_plain, grid_for(total, 256 * 16), dim3(256), 0, c.stream,
               d_seq, total, d_codes, d_err);
    return RB3_OK;
}

int check_codes(Ctx &c, const uint8_t *d_codes, int64_t n, int32_t *d_err) {
    RB3_LAUNCH("check_codes", k_check_codes, grid_for(n, 256 * 16), dim3(256), 0, c.stream, d_codes,
               n, d_err);
    return RB3_OK;
}

// ---------------------------------------------------------------------------
// Packing: one wave per 128-symbol block. Three ballots per 64 symbols give
// the bit-plane words directly. q[3] temporarily holds the block's own
// symbol counts as six bytes (count of code s in byte s); build_checkpoints
// turns them into checkpoints.
// ---------------------------------------------------------------------------
__global__ void k_pack(const uint8_t *__restrict__ codes, int64_t n, uint4 *__restrict__ blk,
                       int64_t nblk) {
    int lane = threadIdx.x & 63;
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t b = wave; b < nblk; b += nwaves) {
        int64_t p = (b << BLK_SHIFT) + lane;
        uint32_t c0 = p < n ? codes[p] : 7u;
        uint32_t c1 = p + 64 < n ? codes[p + 64] : 7u;
        uint64_t a0 = __ballot(c0 & 1), a1 = __ballot(c0 & 2), a2 = __ballot(c0 & 4);
        uint64_t b0 = __ballot(c1 & 1), b1 = __ballot(c1 & 2), b2 = __ballot(c1 & 4);
        uint32_t cnt = 0;
        if (lane < 6)
            cnt = __popcll(plane_match(a0, a1, a2, lane)) + __popcll(plane_match(b0, b1, b2, lane));
        uint32_t lo = 0, hi = 0;
        for (int s = 0; s < 6; ++s) {
            uint32_t v = __shfl(cnt, s);
            if (s < 4) lo |= v << (8 * s);
            else hi |= v << (8 * (s - 4));
        }
        uint4 *dst = blk + (b << 2);
        if (lane == 0) dst[0] = make_uint4((uint32_t)a0, (uint32_t)(a0 >> 32), (uint32_t)b0, (uint32_t)(b0 >> 32));
        if (lane == 1) dst[1] = make_uint4((uint32_t)a1, (uint32_t)(a1 >> 32), (uint32_t)b1, (uint32_t)(b1 >> 32));
        if (lane == 2) dst[2] = make_uint4((uint32_t)a2, (uint32_t)(a2 >> 32), (uint32_t)b2, (uint32_t)(b2 >> 32));
        if (lane == 3) dst[3] = make_uint4(lo, hi, 0u, 0u);
    }
}

int pack_codes(Ctx &c, const uint8_t *d_codes, int64_t n, uint4 *d_blk) {
    int64_t nblk = num_blocks(n);
    RB3_LAUNCH("pack", k_pack, grid_for(nblk, 4, 1 << 18), dim3(256), 0, c.stream, d_codes, n, d_blk,
               nblk);
    return RB3_OK;
}

__device__ __forceinline__ uint32_t local_count(const uint4 &q3, int s) {
    return s < 4 ? (q3.x >> (8 * s)) & 0xFFu : (q3.y >> (8 * (s - 4))) & 0xFFu;
}

// Sum of the per-block counts of each segment of SEG_BLKS blocks.
__global__ void k_seg_reduce(const uint4 *__restrict__ blk, int64_t nblk, uint32_t *__restrict__ segsum) {
    __shared__ uint32_t red[6][256];
    int64_t seg = blockIdx.x;
    uint32_t acc[6] = {0, 0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < SEG_BLKS; i += blockDim.x) {
        int64_t b = seg * SEG_BLKS + i;
        if (b < nblk) {
            uint4 q3 = blk[(b << 2) + 3];
            for (int s = 0; s < 6; ++s) acc[s] += local_count(q3, s);
        }
    }
    for (int s = 0; s < 6; ++s) red[s][threadIdx.x] = acc[s];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int s = 0; s < 6; ++s) red[s][threadIdx.x] += red[s][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 6) segsum[seg * 8 + threadIdx.x] = red[threadIdx.x][0];
}

// One workgroup: exclusive scan of the segment sums per symbol, totals, C[],
// and the superblock table.
__global__ void k_seg_scan(const uint32_t *__restrict__ segsum, int64_t nseg, int64_t *__restrict__ segoff,
                           int64_t *__restrict__ sb, int64_t nsb, int64_t *__restrict__ out12) {
    __shared__ int64_t buf[6][1024];
    __shared__ int64_t carry[6];
    int tid = threadIdx.x;
    if (tid < 6) carry[tid] = 0;
    __syncthreads();
    for (int64_t base = 0; base < nseg; base += 1024) {
        int64_t sidx = base + tid;
        for (int s = 0; s < 6; ++s) buf[s][tid] = sidx < nseg ? (int64_t)segsum[sidx * 8 + s] : 0;
        __syncthreads();
        // Hillis-Steele inclusive scan in LDS
        for (int d = 1; d < 1024; d <<= 1) {
            int64_t v[6];
            for (int s = 0; s < 6; ++s) v[s] = tid >= d ? buf[s][tid - d] : 0;
            __syncthreads();
            for (int s = 0; s < 6; ++s) buf[s][tid] += v[s];
            __syncthreads();
        }
        if (sidx < nseg)
            for (int s = 0; s < 6; ++s)
                segoff[sidx * 8 + s] = carry[s] + buf[s][tid] - (int64_t)segsum[sidx * 8 + s];
        __syncthreads();
        if (tid < 6) carry[tid] += buf[tid][1023];
        __syncthreads();
    }
    __shared__ int64_t C[6];
    if (tid == 0) {
        int64_t acc = 0;
        for (int s = 0; s < 6; ++s) {
            C[s] = acc;
            acc += carry[s];
        }
    }
    __syncthreads();
    if (tid < 6) {
        out12[tid] = C[tid];
        out12[6 + tid] = carry[tid];
    }
    for (int64_t i = tid; i < nsb; i += blockDim.x) {
        int64_t seg = i << (SB_BLK_SHIFT - 10);  // SEG_BLKS = 1024 = 2^10
        for (int s = 0; s < 6; ++s) sb[i * SB_STRIDE + s] = C[s] + segoff[seg * 8 + s];
        sb[i * SB_STRIDE + 6] = 0;
        sb[i * SB_STRIDE + 7] = 0;
    }
}

// Rewrite q[3] of every block: counts before the block, relative to its
// superblock.
__global__ void k_seg_final(uint4 *__restrict__ blk, int64_t nblk, const int64_t *__restrict__ segoff) {
    __shared__ uint32_t sc[5][256];
    int64_t seg = blockIdx.x;
    int tid = threadIdx.x;
    const int PER = SEG_BLKS / 256;  // 4 blocks per thread
    uint32_t loc[PER][5];
    uint32_t tot[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < PER; ++i) {
        int64_t b = seg * SEG_BLKS + tid * PER + i;
        uint4 q3 = b < nblk ? blk[(b << 2) + 3] : make_uint4(0, 0, 0, 0);
        for (int s = 0; s < 5; ++s) {
            loc[i][s] = tot[s];
            tot[s] += local_count(q3, s + 1);
        }
    }
    for (int s = 0; s < 5; ++s) sc[s][tid] = tot[s];
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        uint32_t v[5];
        for (int s = 0; s < 5; ++s) v[s] = tid >= d ? sc[s][tid - d] : 0;
        __syncthreads();
        for (int s = 0; s < 5; ++s) sc[s][tid] += v[s];
        __syncthreads();
    }
    int64_t sbseg = (seg >> (SB_BLK_SHIFT - 10)) << (SB_BLK_SHIFT - 10);
    uint32_t base[5];
    for (int s = 0; s < 5; ++s)
        base[s] = (uint32_t)(segoff[seg * 8 + s + 1] - segoff[sbseg * 8 + s + 1]) + sc[s][tid] - tot[s];
    for (int i = 0; i < PER; ++i) {
        int64_t b = seg * SEG_BLKS + tid * PER + i;
        if (b >= nblk) break;
        uint32_t v[5];
        for (int s = 0; s < 5; ++s) v[s] = base[s] + loc[i][s];
        blk[(b << 2) + 3] = pack_ckpt(v);
    }
}

int build_checkpoints(Ctx &c, uint4 *d_blk, int64_t n, int64_t *d_sb, int64_t C_out[6],
                      int64_t counts_out[6]) {
    int64_t nblk = num_blocks(n);
    int64_t nseg = (nblk + SEG_BLKS - 1) / SEG_BLKS;
    int64_t nsb = num_superblocks(n);
    DBuf segsum, segoff, out12;
    RB3_ALLOC(segsum, &c, nseg * 8 * sizeof(uint32_t));
    RB3_ALLOC(segoff, &c, nseg * 8 * sizeof(int64_t));
    RB3_ALLOC(out12, &c, 12 * sizeof(int64_t));
    RB3_LAUNCH("ckpt_reduce", k_seg_reduce, dim3((unsigned)nseg), dim3(256), 0, c.stream, d_blk, nblk,
               segsum.as<uint32_t>());
    RB3_LAUNCH("ckpt_scan", k_seg_scan, dim3(1), dim3(1024), 0, c.stream, segsum.as<uint32_t>(), nseg,
               segoff.as<int64_t>(), d_sb, nsb, out12.as<int64_t>());
    RB3_LAUNCH("ckpt_final", k_seg_final, dim3((unsigned)nseg), dim3(256), 0, c.stream, d_blk, nblk,
               segoff.as<int64_t>());
    int64_t h[12];
    RB3_HIP(hipMemcpyAsync(h, out12.p, sizeof(h), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipStreamSynchronize(c.stream));
    for (int s = 0; s < 6; ++s) {
        C_out[s] = h[s];
        counts_out[s] = h[6 + s];
    }
    return RB3_OK;
}

__global__ void k_unpack(const uint64_t *__restrict__ words, int64_t n, uint8_t *__restrict__ out) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        int64_t b = p >> BLK_SHIFT;
        int r = (int)(p & 127);
        int w = r >> 6, bit = r & 63;
        const uint64_t *q = words + b * 8;
        uint32_t c = (uint32_t)((q[w] >> bit) & 1u) | (uint32_t)(((q[2 + w] >> bit) & 1u) << 1) |
                     (uint32_t)(((q[4 + w] >> bit) & 1u) << 2);
        out[p] = (uint8_t)c;
    }
}

int unpack_codes(Ctx &c, const DevIndex &ix, uint8_t *d_codes) {
    if (ix.n == 0) return RB3_OK;
    RB3_LAUNCH("unpack", k_unpack, grid_for(ix.n, 256 * 8), dim3(256), 0, c.stream,
               (const uint64_t *)ix.blk, ix.n, d_codes);
    return RB3_OK;
}

}  // namespace rb3
