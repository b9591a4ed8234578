// Stable LSD radix sort of (uint64 key, uint32 value) pairs, 8-bit digits.
//
// Per pass: (1) per-tile digit histograms in LDS, (2) one exclusive scan of
// the digit-major histogram table, (3) a stable scatter. Tiles hold 8192
// keys, so that each digit's share of a tile (32 keys on average) leaves the
// scatter as whole lines. In the scatter each wave owns a contiguous run of
// 1024 keys of the tile and ranks keys with equal digits inside a 64-key
// step by matching the digit with 8 ballots, so no cross-wave
// synchronisation is needed inside the scatter loop.
#include "rb3_internal.h"

namespace rb3 {

constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_STEPS = 32;                       // 64-key steps per wave
constexpr int RS_WAVE_KEYS = 64 * RS_STEPS;        // 1024
constexpr int RS_TILE = RS_WAVES * RS_WAVE_KEYS;   // 8192

// Workgroups are dealt to the 8 XCDs round robin. Giving each XCD a
// contiguous range of tiles keeps the neighbouring pieces of each digit's
// output run, written by neighbouring tiles, in the same L2 (and, for the
// histograms, the neighbouring counts of each digit row).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
    const int64_t q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

__global__ void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n, int shift, uint32_t dmask,
                          uint32_t *__restrict__ H, int64_t ntiles) {
    __shared__ uint32_t h[RS_WAVES][256];
    int tid = threadIdx.x, wave = tid >> 6;
    for (int i = tid; i < RS_WAVES * 256; i += RS_THREADS) (&h[0][0])[i] = 0;
    __syncthreads();
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    int64_t base = tile * RS_TILE;
    // all loads first, then the counts, so the loads' latencies overlap
    constexpr int PER = RS_TILE / RS_THREADS;
    // (indices past the end read the last key, which is then not counted)
    uint64_t kk[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int64_t idx = base + (int64_t)i * RS_THREADS + tid;
        kk[i] = keys[idx < n ? idx : n - 1];
    }
#pragma unroll
    for (int i = 0; i < PER; ++i)
        if (base + (int64_t)i * RS_THREADS + tid < n) atomicAdd(&h[wave][(uint32_t)(kk[i] >> shift) & dmask], 1u);
    __syncthreads();
    for (int d = tid; d < 256; d += RS_THREADS)
        H[(int64_t)d * ntiles + tile] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
    // number of set bits of mask below this lane
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Scatter of one tile. The tile's keys are first ranked stably inside the
// tile and staged in LDS in digit order; then the workgroup writes them out
// with consecutive threads on consecutive output positions, so each digit's
// run leaves as whole lines instead of scattered 8- and 4-byte stores.
//
// Records travel in one of two forms: a key with a separate 32-bit value
// (KV), or, when the key's bits and the value fit together, one packed word
// key << pbits | value (PK), which moves 8 bytes instead of 12 per pass.
// IN: 0 = KV, 1 = key with its index as the implicit value, 2 = PK.
// OUT: 0 = KV, 1 = PK. shift selects the digit from the input word.
constexpr int SC_THREADS = 512;
constexpr int SC_WAVES = SC_THREADS / 64;
constexpr int SC_STEPS = RS_TILE / SC_THREADS;  // 64-key steps per wave

template <int IN, int OUT>
__global__ void __launch_bounds__(SC_THREADS) k_rs_scatter(const uint64_t *__restrict__ kin,
                                                           const uint32_t *__restrict__ vin, int pbits,
                                                           int64_t n, int shift, uint32_t dmask, int dbits,
                                                           const uint32_t *__restrict__ O, int64_t ntiles,
                                                           uint64_t *__restrict__ kout,
                                                           uint32_t *__restrict__ vout,
                                                           int32_t *__restrict__ guard) {
    // staged words: packed records whenever either side is packed
    constexpr bool STAGE_PK = IN == 2 || OUT == 1;
    __shared__ uint64_t sk[RS_TILE];
    __shared__ uint32_t sv[STAGE_PK ? 1 : RS_TILE];
    __shared__ uint32_t wbase[SC_WAVES][256];
    __shared__ uint32_t gbase[256];
    __shared__ uint32_t wsum[SC_WAVES];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint64_t vmask = (1ull << pbits) - 1ull;
    for (int i = tid; i < SC_WAVES * 256; i += SC_THREADS) (&wbase[0][0])[i] = 0;
    __syncthreads();
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t tile0 = tile * RS_TILE;
    const int64_t base = tile0 + (int64_t)wave * (64 * SC_STEPS);
    uint64_t k[SC_STEPS];
    uint32_t v[SC_STEPS];
    // the tile's digit offsets are read together with its keys, so the two
    // memory latencies overlap
    const uint32_t o = tid < 256 ? O[(int64_t)tid * ntiles + tile] : 0u;
    // all loads are issued before the first count, so their latencies overlap
#pragma unroll
    for (int j = 0; j < SC_STEPS; ++j) {
        const int64_t idx = base + j * 64 + lane;
        const bool ok = idx < n;
        k[j] = ok ? kin[idx] : 0ull;
        v[j] = IN == 0 ? (ok ? vin[idx] : 0u) : (IN == 1 ? (uint32_t)idx : 0u);
    }
#pragma unroll
    for (int j = 0; j < SC_STEPS; ++j)
        if (base + j * 64 + lane < n) atomicAdd(&wbase[wave][(uint32_t)(k[j] >> shift) & dmask], 1u);
    __syncthreads();
    // digit totals of the tile, their exclusive prefix (tile-local digit
    // starts), and per (wave, digit) local bases
    uint32_t tot = 0, cnt[SC_WAVES];
    if (tid < 256) {
#pragma unroll
        for (int w = 0; w < SC_WAVES; ++w) {
            cnt[w] = wbase[w][tid];
            tot += cnt[w];
        }
    }
    uint32_t inc = tot;
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(inc, d);
        if (lane >= d) inc += t;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    if (tid < 256) {
        uint32_t pre = inc - tot;
        for (int w = 0; w < wave; ++w) pre += wsum[w];
        gbase[tid] = o - pre;
        uint32_t run = pre;
#pragma unroll
        for (int w = 0; w < SC_WAVES; ++w) {
            wbase[w][tid] = run;
            run += cnt[w];
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SC_STEPS; ++j) {
        int64_t idx = base + j * 64 + lane;
        bool valid = idx < n;
        uint32_t d = (uint32_t)(k[j] >> shift) & dmask;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < dbits; ++b) {
            uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        uint32_t r = lane_rank(peers);
        uint32_t pos = 0;
        if (valid) pos = wbase[wave][d] + r;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (valid) {
            if (STAGE_PK) {
                sk[pos] = IN == 2 ? k[j] : ((k[j] << pbits) | (uint64_t)v[j]);
            } else {
                sk[pos] = k[j];
                sv[pos] = v[j];
            }
            if (r == 0) wbase[wave][d] = pos + (uint32_t)__popcll(peers);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    const int64_t tn = n - tile0 < RS_TILE ? n - tile0 : RS_TILE;
    // the digit of a staged word: packed words carry the key pbits higher
    const int sshift = (STAGE_PK && IN != 2) ? shift + pbits : shift;
    for (int i = tid; i < tn; i += SC_THREADS) {
        uint64_t w = sk[i];
        uint32_t d = (uint32_t)(w >> sshift) & dmask;
        uint32_t gpos = gbase[d] + (uint32_t)i;
        if ((int64_t)gpos < n) {
            if (OUT == 1) {
                kout[gpos] = w;
            } else if (STAGE_PK) {
                kout[gpos] = w >> pbits;
                vout[gpos] = (uint32_t)(w & vmask);
            } else {
                kout[gpos] = w;
                vout[gpos] = sv[i];
            }
        } else {
            atomicOr(guard, 1);
        }
    }
}

int radix_sort(Ctx &c, uint64_t *k_in, uint32_t *v_in, uint64_t *k_a, uint32_t *v_a, uint64_t *k_b,
               uint32_t *v_b, int64_t n, int lo_bit, int hi_bit, bool iota_vals, uint64_t **k_res,
               uint32_t **v_res, int32_t *d_guard, int *used_packed, int *used_passes) {
    if (used_packed) *used_packed = 0;
    if (used_passes) *used_passes = 0;
    if (n >= (int64_t)UINT32_MAX) {
        set_error(RB3_ELIMIT, "radix sort: too many records");
        return RB3_ELIMIT;
    }
    int64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
    DBuf H;
    RB3_ALLOC(H, &c, 256 * (ntiles > 0 ? ntiles : 1) * sizeof(uint32_t));
    if (hi_bit <= lo_bit || n == 0) {
        // nothing to sort: copy through
        RB3_HIP(hipMemcpyAsync(k_a, k_in, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, c.stream));
        if (iota_vals) {
            set_error(RB3_EINVAL, "radix sort: empty key range with implicit values");
            return RB3_EINVAL;
        }
        RB3_HIP(hipMemcpyAsync(v_a, v_in, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, c.stream));
        *k_res = k_a;
        *v_res = v_a;
        return RB3_OK;
    }
    const int npass = (hi_bit - lo_bit + 7) / 8;
    // packed records when the key and the record index fit one word (the
    // values are the indices, so they need bits_for(n - 1) bits)
    int pbits = 1;
    while (pbits < 32 && ((int64_t)1 << pbits) < n) ++pbits;
    const bool packed = iota_vals && npass >= 2 && hi_bit + pbits <= 64;
    if (used_packed) *used_packed = packed ? 1 : 0;
    if (used_passes) *used_passes = npass;
    const uint64_t *src_k = k_in;
    const uint32_t *src_v = v_in;
    int in_mode = iota_vals ? 1 : 0;
    uint64_t *dk = k_a;
    uint32_t *dv = v_a;
    int pass = 0;
    for (int shift = lo_bit; shift < hi_bit; shift += 8, ++pass) {
        const int dbits = hi_bit - shift < 8 ? hi_bit - shift : 8;
        const uint32_t dmask = (1u << dbits) - 1u;
        const bool last = pass == npass - 1;
        const int out_mode = packed && !last ? 1 : 0;
        const int in_shift = in_mode == 2 ? shift + pbits : shift;
        RB3_LAUNCH("sort_hist", k_rs_hist, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, c.stream, src_k, n,
                   in_shift, dmask, H.as<uint32_t>(), ntiles);
        RB3_TRY(scan_u32(c, H.as<uint32_t>(), H.as<uint32_t>(), 256 * ntiles, false, false, nullptr));
        const dim3 g((unsigned)ntiles), blk(SC_THREADS);
        uint32_t *H_ = H.as<uint32_t>();
        if (in_mode == 0 && out_mode == 0)
            RB3_LAUNCH("sort_scatter", (k_rs_scatter<0, 0>), g, blk, 0, c.stream, src_k, src_v, pbits, n, in_shift,
                       dmask, dbits, H_, ntiles, dk, dv, d_guard);
        else if (in_mode == 1 && out_mode == 0)
            RB3_LAUNCH("sort_scatter", (k_rs_scatter<1, 0>), g, blk, 0, c.stream, src_k, src_v, pbits, n, in_shift,
                       dmask, dbits, H_, ntiles, dk, dv, d_guard);
        else if (in_mode == 1 && out_mode == 1)
            RB3_LAUNCH("sort_scatter", (k_rs_scatter<1, 1>), g, blk, 0, c.stream, src_k, src_v, pbits, n, in_shift,
                       dmask, dbits, H_, ntiles, dk, dv, d_guard);
        else if (in_mode == 2 && out_mode == 1)
            RB3_LAUNCH("sort_scatter", (k_rs_scatter<2, 1>), g, blk, 0, c.stream, src_k, src_v, pbits, n, in_shift,
                       dmask, dbits, H_, ntiles, dk, dv, d_guard);
        else
            RB3_LAUNCH("sort_scatter", (k_rs_scatter<2, 0>), g, blk, 0, c.stream, src_k, src_v, pbits, n, in_shift,
                       dmask, dbits, H_, ntiles, dk, dv, d_guard);
        src_k = dk;
        src_v = dv;
        in_mode = out_mode == 1 ? 2 : 0;
        if (dk == k_a) {
            dk = k_b;
            dv = v_b;
        } else {
            dk = k_a;
            dv = v_a;
        }
    }
    *k_res = (uint64_t *)src_k;
    *v_res = (uint32_t *)src_v;
    return RB3_OK;
}

}  // namespace rb3
