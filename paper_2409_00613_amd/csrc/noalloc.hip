// rb3_count_noalloc: backward-search counts (Sec. 2.3) for callers that
// cannot allocate device memory. The work is that of rb3_count (the same
// encode and count kernels); every temporary the count needs lives in one
// fixed array of device memory that the library holds for the life of the
// process, one copy per device.
#include "rb3_internal.h"

#include <mutex>

namespace rb3 {

// The scratch array. In host code its name stands for a host-side shadow,
// not a device address: the device address is taken once per device with
// hipGetSymbolAddress and only that address is used from the host.
static __device__ __align__(256) uint8_t scratch[RB3_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEV = 64;
static std::mutex g_na_mu[MAX_DEV];
static void *g_na_ptr[MAX_DEV];

// The device address of scratch on the current device `dev` (taken on the
// first call there). Called with g_na_mu[dev] held.
static int scratch_ptr(int dev, uint8_t **out) {
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        RB3_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error(RB3_EDEVICE, "hipGetSymbolAddress gave a null address for the scratch array");
            return RB3_EDEVICE;
        }
        g_na_ptr[dev] = p;
    }
    *out = (uint8_t *)g_na_ptr[dev];
    return RB3_OK;
}

static inline int64_t up256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// Query offsets from the lengths: off[1..n] hold the lengths on entry and
// their inclusive prefix sums on exit, off[0] = 0. One workgroup: each
// thread sums a contiguous range, the range sums are scanned in LDS, then
// each thread rewrites its range. Also clears the error flag, so the launch
// that follows on the stream starts from zero.
constexpr int NA_SCAN_T = 1024;
__global__ void __launch_bounds__(NA_SCAN_T) k_na_offsets(int64_t *__restrict__ off, int64_t n,
                                                          int32_t *__restrict__ err) {
    __shared__ int64_t part[NA_SCAN_T];
    const int t = threadIdx.x;
    const int64_t per = (n + NA_SCAN_T - 1) / NA_SCAN_T;
    const int64_t a = 1 + (int64_t)t * per;
    const int64_t b = a + per < n + 1 ? a + per : n + 1;
    int64_t s = 0;
    for (int64_t i = a; i < b; ++i) s += off[i];
    part[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the range sums
    for (int d = 1; d < NA_SCAN_T; d <<= 1) {
        const int64_t v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = t > 0 ? part[t - 1] : 0;
    for (int64_t i = a; i < b; ++i) {
        run += off[i];
        off[i] = run;
    }
    if (t == 0) {
        off[0] = 0;
        *err = 0;
    }
}

// Bytes to codes, from src (the caller's device buffer, or the same
// scratch bytes when the queries were copied in from the host) to dst.
// Each element is read and written by one thread only, so src may equal dst.
__global__ void k_na_encode(const uint8_t *src, uint8_t *dst, int64_t total, int32_t *__restrict__ err) {
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int c = ascii_code(src[i]);
        if (c < 0) {
            bad = 1;
            c = 1;
        }
        dst[i] = (uint8_t)c;
    }
    if (bad) atomicOr(err, 1);
}

int count_noalloc(const DevIndex &ix, int dev, hipStream_t stream, const uint8_t *q, const int64_t *qlens,
                  int64_t n_q, int64_t total, int32_t mem, int64_t *lo, int64_t *hi) {
    if (dev < 0 || dev >= MAX_DEV) {
        set_error(RB3_EINVAL, "device ordinal out of range for the scratch table");
        return RB3_EINVAL;
    }
    // scratch layout: error flag | offsets (n_q + 1) | codes (total) |
    // staged lo, hi (host outputs only)
    const int64_t o_off = 256;
    const int64_t o_codes = o_off + up256((n_q + 1) * (int64_t)sizeof(int64_t));
    const int64_t o_lo = o_codes + up256(total > 0 ? total : 1);
    const int64_t o_hi = o_lo + (mem == RB3_MEM_HOST ? up256(n_q * (int64_t)sizeof(int64_t)) : 0);
    const int64_t need = o_hi + (mem == RB3_MEM_HOST ? up256(n_q * (int64_t)sizeof(int64_t)) : 0);
    if (need > (int64_t)RB3_NOALLOC_SCRATCH_BYTES) {
        set_error(RB3_ELIMIT, "rb3_count_noalloc: the queries need " + std::to_string(need) +
                                  " bytes of scratch, more than the fixed " +
                                  std::to_string((long long)RB3_NOALLOC_SCRATCH_BYTES));
        return RB3_ELIMIT;
    }
    std::lock_guard<std::mutex> lk(g_na_mu[dev]);
    uint8_t *base = nullptr;
    RB3_TRY(scratch_ptr(dev, &base));
    int32_t *d_err = (int32_t *)base;
    int64_t *d_off = (int64_t *)(base + o_off);
    uint8_t *d_codes = base + o_codes;
    int64_t *d_lo = mem == RB3_MEM_HOST ? (int64_t *)(base + o_lo) : lo;
    int64_t *d_hi = mem == RB3_MEM_HOST ? (int64_t *)(base + o_hi) : hi;
    Ctx c;  // no allocator is ever called through it
    c.device = dev;
    c.stream = stream;
    RB3_HIP(hipMemcpyAsync(d_off + 1, qlens, n_q * sizeof(int64_t), hipMemcpyHostToDevice, stream));
    RB3_LAUNCH("noalloc_offsets", k_na_offsets, dim3(1), dim3(NA_SCAN_T), 0, stream, d_off, n_q, d_err);
    const uint8_t *d_seq = q;
    if (mem == RB3_MEM_HOST && total > 0) {
        // the bytes are encoded in place
        RB3_HIP(hipMemcpyAsync(d_codes, q, total, hipMemcpyHostToDevice, stream));
        d_seq = d_codes;
    }
    if (total > 0)
        RB3_LAUNCH("noalloc_encode", k_na_encode, grid_for(total, 256 * 16), dim3(256), 0, stream, d_seq, d_codes,
                   total, d_err);
    int32_t bad = 0;
    RB3_HIP(hipMemcpyAsync(&bad, d_err, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    RB3_HIP(hipStreamSynchronize(stream));
    if (bad) {
        set_error(RB3_EINVAL, "byte outside ACGTNacgtn in a query");
        return RB3_EINVAL;
    }
    RB3_TRY(count_queries(c, ix, d_codes, d_off, n_q, d_lo, d_hi));
    if (mem == RB3_MEM_HOST) {
        RB3_HIP(hipMemcpyAsync(lo, d_lo, n_q * sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        RB3_HIP(hipMemcpyAsync(hi, d_hi, n_q * sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    }
    RB3_HIP(hipStreamSynchronize(stream));
    return RB3_OK;
}

}  // namespace rb3
