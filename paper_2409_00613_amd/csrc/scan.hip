// Device-wide scans of uint32 arrays (sum or max), three passes:
// per-tile reduce, scan of the tile partials (in one workgroup, or
// recursively when there are more partials than one tile holds), per-tile
// rescan.
#include "rb3_internal.h"

namespace rb3 {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <bool MAX>
__device__ __forceinline__ uint32_t sop(uint32_t a, uint32_t b) {
    return MAX ? (a > b ? a : b) : a + b;
}

template <bool MAX>
__device__ __forceinline__ uint32_t wave_inclusive(uint32_t v) {
    int lane = threadIdx.x & 63;
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d);
        if (lane >= d) v = sop<MAX>(v, t);
    }
    return v;
}

// Exclusive scan of one value per thread across the workgroup; returns the
// exclusive prefix and writes the workgroup total to *total.
template <bool MAX>
__device__ uint32_t block_exclusive(uint32_t v, uint32_t *total) {
    __shared__ uint32_t wsum[SCAN_THREADS / 64];
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = wave_inclusive<MAX>(v);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < wave; ++w) pre = sop<MAX>(pre, wsum[w]);
    uint32_t tot = 0;
    for (int w = 0; w < SCAN_THREADS / 64; ++w) tot = sop<MAX>(tot, wsum[w]);
    uint32_t ex = __shfl_up(inc, 1);
    if (lane == 0) ex = 0;
    __syncthreads();
    *total = tot;
    return sop<MAX>(pre, ex);
}

template <bool MAX>
__global__ void k_scan_reduce(const uint32_t *__restrict__ in, int64_t n, uint32_t *__restrict__ part) {
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t acc = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < n) acc = sop<MAX>(acc, in[base + i]);
    uint32_t tot;
    block_exclusive<MAX>(acc, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// One workgroup of SCAN_THREADS: exclusive scan of the partials in place.
template <bool MAX>
__global__ void k_scan_parts(uint32_t *__restrict__ part, int64_t np, uint32_t *__restrict__ total) {
    uint32_t carry = 0;
    for (int64_t base = 0; base < np; base += SCAN_TILE) {
        int64_t b = base + (int64_t)threadIdx.x * SCAN_ITEMS;
        uint32_t v[SCAN_ITEMS];
        uint32_t acc = 0;
        for (int i = 0; i < SCAN_ITEMS; ++i) {
            v[i] = b + i < np ? part[b + i] : 0;
            acc = sop<MAX>(acc, v[i]);
        }
        uint32_t tot;
        uint32_t ex = block_exclusive<MAX>(acc, &tot);
        uint32_t run = sop<MAX>(carry, ex);
        for (int i = 0; i < SCAN_ITEMS; ++i) {
            if (b + i < np) part[b + i] = run;
            run = sop<MAX>(run, v[i]);
        }
        carry = sop<MAX>(carry, tot);
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <bool MAX>
__global__ void k_scan_down(const uint32_t *__restrict__ in, uint32_t *__restrict__ out, int64_t n,
                            const uint32_t *__restrict__ part, int inclusive) {
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t acc = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = base + i < n ? in[base + i] : 0;
        acc = sop<MAX>(acc, v[i]);
    }
    uint32_t tot;
    uint32_t ex = block_exclusive<MAX>(acc, &tot);
    uint32_t run = sop<MAX>(part[blockIdx.x], ex);
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        uint32_t nxt = sop<MAX>(run, v[i]);
        if (base + i < n) out[base + i] = inclusive ? nxt : run;
        run = nxt;
    }
}

int scan_u32(Ctx &c, const uint32_t *d_in, uint32_t *d_out, int64_t n, bool inclusive, bool max_op,
             uint32_t *d_total) {
    if (n <= 0) {
        if (d_total) RB3_HIP(hipMemsetAsync(d_total, 0, sizeof(uint32_t), c.stream));
        return RB3_OK;
    }
    int64_t np = (n + SCAN_TILE - 1) / SCAN_TILE;
    DBuf part;
    RB3_ALLOC(part, &c, np * sizeof(uint32_t));
    dim3 g((unsigned)np), b(SCAN_THREADS);
    if (max_op)
        RB3_LAUNCH("scan_reduce", k_scan_reduce<true>, g, b, 0, c.stream, d_in, n, part.as<uint32_t>());
    else
        RB3_LAUNCH("scan_reduce", k_scan_reduce<false>, g, b, 0, c.stream, d_in, n, part.as<uint32_t>());
    // The tile partials are scanned by one workgroup when they fit one of its
    // tiles, else by the same three steps one level up: a single workgroup
    // walking tens of thousands of partials serially costs more than the
    // two extra launches.
    if (np > SCAN_TILE) {
        RB3_TRY(scan_u32(c, part.as<uint32_t>(), part.as<uint32_t>(), np, false, max_op, d_total));
    } else if (max_op) {
        RB3_LAUNCH("scan_parts", k_scan_parts<true>, dim3(1), b, 0, c.stream, part.as<uint32_t>(), np, d_total);
    } else {
        RB3_LAUNCH("scan_parts", k_scan_parts<false>, dim3(1), b, 0, c.stream, part.as<uint32_t>(), np, d_total);
    }
    if (max_op)
        RB3_LAUNCH("scan_down", k_scan_down<true>, g, b, 0, c.stream, d_in, d_out, n, part.as<uint32_t>(),
                   (int)inclusive);
    else
        RB3_LAUNCH("scan_down", k_scan_down<false>, g, b, 0, c.stream, d_in, d_out, n, part.as<uint32_t>(),
                   (int)inclusive);
    return RB3_OK;
}

}  // namespace rb3
