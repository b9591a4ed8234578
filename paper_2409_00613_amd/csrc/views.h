// The two device index forms behind one interface, for kernels that run
// on either: the 3-bit-plane index (one 64-byte block per rank) and the
// run-length static one (one 128-byte block per rank, decoded up to the
// position). pi2 gives C[c] + rank_c at both positions for every symbol c,
// that is, the SA-interval starts of every backward extension (Sec. 2.3).
#pragma once

#include "rle.h"

namespace rb3 {

struct PlainView {
    DevIndex ix;
    __host__ __device__ int64_t size() const { return ix.n; }
    // one backward-search step of both ends for symbol a
    __device__ __forceinline__ void step(int a, int64_t &lo, int64_t &hi) const {
        // the symbol and both ends' blocks are requested together (the
        // second block read is the first one again when they share it)
        const Block Bl = load_block(ix.blk, lo >> BLK_SHIFT);
        const Block Bh = load_block(ix.blk, hi >> BLK_SHIFT);
        lo = pi_from_block(ix, Bl, a, lo);
        hi = pi_from_block(ix, Bh, a, hi);
    }
    __device__ __forceinline__ void pi2(int64_t k0, int64_t k1, int64_t o0[6], int64_t o1[6]) const {
        pi_all2(ix, k0, k1, o0, o1);
    }
    // distinct index blocks that rank-all at k0 and k1 reads
    __device__ __forceinline__ uint64_t units(int64_t k0, int64_t k1) const {
        return 1 + ((k0 >> BLK_SHIFT) != (k1 >> BLK_SHIFT));
    }
};

// o[a] as a sum of masked terms: a select chain over a register array is
// turned into an indexed load from scratch memory by the compiler.
__device__ __forceinline__ int64_t pick6(const int64_t o[6], int a) {
    int64_t r = 0;
#pragma unroll
    for (int c = 0; c < 6; ++c) r += o[c] & -(int64_t)(a == c);
    return r;
}

struct RleQView {
    RleView v;
    __host__ __device__ int64_t size() const { return v.n; }
    __device__ __forceinline__ void pi2(int64_t k0, int64_t k1, int64_t o0[6], int64_t o1[6]) const {
        rle_occ_all(v, k0, o0);
        rle_occ_all(v, k1, o1);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            o0[c] += v.C[c];
            o1[c] += v.C[c];
        }
    }
    __device__ __forceinline__ void step(int a, int64_t &lo, int64_t &hi) const {
        int64_t o0[6], o1[6];
        pi2(lo, hi, o0, o1);
        lo = pick6(o0, a);
        hi = pick6(o1, a);
    }
    // 128-byte blocks decoded (ends at a segment start or at n read none)
    __device__ __forceinline__ uint64_t units(int64_t k0, int64_t k1) const {
        return (uint64_t)((k0 & (RLE_SEG - 1)) != 0 && k0 < v.n) + (uint64_t)((k1 & (RLE_SEG - 1)) != 0 && k1 < v.n);
    }
};

}  // namespace rb3
