// Internal definitions shared by the HIP kernels and the host side of the
// library. gfx950 (CDNA4) only: wave64, 64-byte index blocks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "rb3.h"

namespace rb3 {

// ---------------------------------------------------------------------------
// Index layout in HBM
// ---------------------------------------------------------------------------
//
// The BWT B[0..n) of codes $=0 A=1 C=2 G=3 T=4 N=5 is cut into blocks of 128
// symbols. Block b is 64 bytes = 4 x uint4:
//   q[0], q[1], q[2] : bit planes 0, 1, 2 of the 128 codes. As two uint64
//                      words (lo = symbols 0..63, hi = 64..127), bit r of a
//                      word is symbol r.
//   q[3]             : occurrence checkpoint. The number of A, C, G, T, N in
//                      B[S, 128 b), where S is the start of b's superblock,
//                      as 24-bit fields at bit offsets 0, 24, 48, 72, 96 of
//                      the 128-bit word (lo 64 bits first).
// A superblock covers 2^24 symbols (2^17 blocks); its table entry holds eight
// int64: entry[c] = C[c] + (occurrences of c before the superblock) for
// c = 0..5, so C + rank is one add away. Positions past n hold code 7, which
// matches no symbol. There are n/128 + 1 blocks, so a rank at k = n reads a
// real block.
//
// One rank therefore touches one 64-byte block plus one superblock entry
// (a table of n/2^24 * 64 bytes that stays in cache).
constexpr int BLK_SHIFT = 7;
constexpr int64_t BLK_SYMS = 128;
constexpr int SB_SHIFT = 24;
constexpr int SB_BLK_SHIFT = SB_SHIFT - BLK_SHIFT;  // blocks per superblock = 2^17
constexpr int SB_STRIDE = 8;
constexpr uint32_t CNT_MASK = 0xFFFFFFu;

// Blocks per scan segment when checkpoints are rebuilt (divides 2^17).
constexpr int SEG_BLKS = 1024;

struct DevIndex {
    const uint4 *blk;   // nblk * 4
    const int64_t *sb;  // nsb * SB_STRIDE
    int64_t n;          // BWT length (symbols, sentinels included)
    int64_t m;          // sentinels
    int64_t C[8];       // C[0..5], C[6] = n
};

__host__ __device__ inline int64_t num_blocks(int64_t n) { return (n >> BLK_SHIFT) + 1; }
__host__ __device__ inline int64_t num_superblocks(int64_t n) { return (n >> SB_SHIFT) + 1; }

__device__ __forceinline__ uint64_t u64_lo(const uint4 &q) {
    return (uint64_t)q.x | ((uint64_t)q.y << 32);
}
__device__ __forceinline__ uint64_t u64_hi(const uint4 &q) {
    return (uint64_t)q.z | ((uint64_t)q.w << 32);
}

// Bits of a plane word pair where the code equals sym (0..7).
__device__ __forceinline__ uint64_t plane_match(uint64_t p0, uint64_t p1, uint64_t p2, int sym) {
    uint64_t a = (sym & 1) ? p0 : ~p0;
    uint64_t b = (sym & 2) ? p1 : ~p1;
    uint64_t c = (sym & 4) ? p2 : ~p2;
    return a & b & c;
}

__device__ __forceinline__ uint64_t low_mask(int o) {  // bits [0, o), o in [0, 64]
    return o >= 64 ? ~0ull : ((1ull << o) - 1ull);
}

// 24-bit checkpoint field f (0..4 for A..N) of q[3]: bits 24 f .. 24 f + 23
// of the 128-bit word, taken without branches (lanes of a wave usually ask
// for different fields) and with shifts only, so the block stays in
// registers (indexing its 32-bit parts by a variable would put it in
// scratch memory).
__device__ __forceinline__ uint32_t ckpt_field(const uint4 &q3, int f) {
    const uint64_t c0 = u64_lo(q3), c1 = u64_hi(q3);
    const uint32_t bit = 24u * (uint32_t)f;  // 0, 24, 48, 72, 96
    const uint64_t low = (c0 >> (bit & 63u)) | ((c1 << 1) << (63u - (bit & 63u)));
    const uint64_t v = bit < 64u ? low : (c1 >> (bit - 64u));
    return (uint32_t)v & CNT_MASK;
}

__device__ __forceinline__ uint4 pack_ckpt(const uint32_t c[5]) {
    uint64_t c0 = (uint64_t)c[0] | ((uint64_t)c[1] << 24) | ((uint64_t)c[2] << 48);
    uint64_t c1 = ((uint64_t)c[2] >> 16) | ((uint64_t)c[3] << 8) | ((uint64_t)c[4] << 32);
    return make_uint4((uint32_t)c0, (uint32_t)(c0 >> 32), (uint32_t)c1, (uint32_t)(c1 >> 32));
}

struct Block {
    uint4 q0, q1, q2, q3;
};

__device__ __forceinline__ Block load_block(const uint4 *blk, int64_t b) {
    const uint4 *p = blk + (b << 2);
    Block r;
    r.q0 = p[0];
    r.q1 = p[1];
    r.q2 = p[2];
    r.q3 = p[3];
    return r;
}

// Occurrences of sym in the first o symbols of the block (o in [0, 128]).
__device__ __forceinline__ int inblock_count(const Block &B, int sym, int o) {
    uint64_t lo = plane_match(u64_lo(B.q0), u64_lo(B.q1), u64_lo(B.q2), sym);
    if (o <= 64) return __popcll(lo & low_mask(o));
    uint64_t hi = plane_match(u64_hi(B.q0), u64_hi(B.q1), u64_hi(B.q2), sym);
    return __popcll(lo) + __popcll(hi & low_mask(o - 64));
}

// pi_B(a, k) = C(a) + rank_B(a, k) for a in 1..5 (Table 1), given the block
// holding position k.
__device__ __forceinline__ int64_t pi_from_block(const DevIndex &ix, const Block &B, int a,
                                                 int64_t k) {
    int o = (int)(k & (BLK_SYMS - 1));
    return ix.sb[(k >> SB_SHIFT) * SB_STRIDE + a] + (int64_t)ckpt_field(B.q3, a - 1) +
           inblock_count(B, a, o);
}

__device__ __forceinline__ int64_t pi_sym(const DevIndex &ix, int a, int64_t k) {
    Block B = load_block(ix.blk, k >> BLK_SHIFT);
    return pi_from_block(ix, B, a, k);
}

// pi_B(c, k) for every c in 0..5, from the block holding k and the
// superblock row s of k. rank($, k) is k minus the other ranks.
__device__ __forceinline__ void pi_all_from(const DevIndex &ix, const Block &B, const int64_t s[6], int64_t k,
                                            int64_t out[6]) {
    int o = (int)(k & (BLK_SYMS - 1));
    uint64_t l0 = u64_lo(B.q0), l1 = u64_lo(B.q1), l2 = u64_lo(B.q2);
    uint64_t h0 = u64_hi(B.q0), h1 = u64_hi(B.q1), h2 = u64_hi(B.q2);
    uint64_t mlo = low_mask(o < 64 ? o : 64);
    uint64_t mhi = o > 64 ? low_mask(o - 64) : 0ull;
    int64_t others = 0;
    for (int a = 1; a <= 5; ++a) {
        int cnt = __popcll(plane_match(l0, l1, l2, a) & mlo) + __popcll(plane_match(h0, h1, h2, a) & mhi);
        out[a] = s[a] + (int64_t)ckpt_field(B.q3, a - 1) + cnt;
        others += out[a] - ix.C[a];
    }
    out[0] = k - others;  // C[0] = 0
}

__device__ __forceinline__ void load_sb_row(const DevIndex &ix, int64_t k, int64_t s[6]) {
    const int64_t *r = ix.sb + (k >> SB_SHIFT) * SB_STRIDE;
    s[0] = 0;
#pragma unroll
    for (int a = 1; a <= 5; ++a) s[a] = r[a];
}

// pi_all at two positions; every load of both is issued before any use,
// so the two random block reads overlap.
__device__ __forceinline__ void pi_all2(const DevIndex &ix, int64_t k0, int64_t k1, int64_t out0[6],
                                        int64_t out1[6]) {
    int64_t s0[6], s1[6];
    load_sb_row(ix, k0, s0);
    load_sb_row(ix, k1, s1);
    const Block B0 = load_block(ix.blk, k0 >> BLK_SHIFT);
    const Block B1 = load_block(ix.blk, k1 >> BLK_SHIFT);
    // keep the scheduler from moving the first block's use above the
    // second block's loads
    __builtin_amdgcn_sched_barrier(0);
    pi_all_from(ix, B0, s0, k0, out0);
    pi_all_from(ix, B1, s1, k1, out1);
}

// ASCII -> code: A=1 C=2 G=3 T=4 N=5 in either case; -1 for anything else.
__device__ __forceinline__ int ascii_code(uint32_t ch) {
    switch (ch | 0x20u) {
    case 'a': return 1;
    case 'c': return 2;
    case 'g': return 3;
    case 't': return 4;
    case 'n': return 5;
    default: return -1;
    }
}

// ---------------------------------------------------------------------------
// Host-side context
// ---------------------------------------------------------------------------

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    rb3_alloc_fn alloc = nullptr;
    rb3_free_fn free_fn = nullptr;
    void *alloc_ctx = nullptr;
    int64_t chunk_len = 0;
    int32_t launch_per_string = 0;
    int64_t smem_segs = 0;     // SMEM segments to aim for per call; 0 = SMEM_TARGET_SEGS
    int64_t smem_seg_min = 0;  // shortest SMEM segment; 0 = SMEM_SEG_MIN
    int64_t smem_seg_fixed = 0;  // fixed SMEM segment length; 0 = tuned or from the batch; -1 = from the batch
    int32_t both = 1;
    int32_t ssa = 0;           // suffix-array sampling distance (0: no samples)
    // Frees are deferred until flush(), called after the stream has drained,
    // so that a caching allocator never hands out memory a queued kernel
    // still uses.
    std::vector<void *> deferred;

    void *dmalloc(size_t bytes);
    void dfree(void *p) { if (p) deferred.push_back(p); }
    void free_now(void *p);
    int flush();  // synchronize the stream, then release deferred buffers
};

// RAII device buffer owned through a Ctx.
struct DBuf {
    Ctx *ctx = nullptr;
    void *p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { reset(); }
    void reset() {
        if (p && ctx) ctx->dfree(p);
        p = nullptr;
        bytes = 0;
    }
    // returns false on allocation failure
    bool alloc(Ctx *c, size_t nbytes) {
        reset();
        ctx = c;
        bytes = nbytes;
        p = c->dmalloc(nbytes ? nbytes : 16);
        return p != nullptr;
    }
    void *release() {
        void *r = p;
        p = nullptr;
        return r;
    }
    template <class T> T *as() const { return (T *)p; }
};

// Consistency guards: kernels that index through computed positions check
// them and set a bit here instead of touching memory out of range.
enum {
    GUARD_SORT = 1,
    GUARD_GATHER = 2,
    GUARD_RERANK = 4,
    GUARD_COMPACT = 8,
    GUARD_INTERLEAVE = 16,
    GUARD_PLACE = 32,
    GUARD_SAMPLE = 64,
    GUARD_CHAIN = 128
};

// Error state: thread-local message for rb3_strerror.
void set_error(int code, const std::string &msg);

// A failed HIP call: record and return RB3_EDEVICE.
#define RB3_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t _e = (call);                                                        \
        if (_e != hipSuccess) {                                                        \
            ::rb3::set_error(RB3_EDEVICE, std::string(#call) + ": " + hipGetErrorString(_e)); \
            return RB3_EDEVICE;                                                        \
        }                                                                              \
    } while (0)

#define RB3_TRY(expr)          \
    do {                       \
        int _r = (expr);       \
        if (_r != RB3_OK) return _r; \
    } while (0)

#define RB3_ALLOC(buf, ctx, nbytes)                                                    \
    do {                                                                               \
        if (!(buf).alloc((ctx), (nbytes))) {                                           \
            ::rb3::set_error(RB3_ENOMEM, "device allocation failed (" #buf ")");       \
            return RB3_ENOMEM;                                                         \
        }                                                                              \
    } while (0)

// Kernel-launch profiling (events around launches when enabled).
struct ProfScope {
    const char *name;
    hipStream_t stream;
    void *ev0 = nullptr;
    ProfScope(const char *nm, hipStream_t s);
    ~ProfScope();
};

int check_launch(const char *name);

#define RB3_LAUNCH(name, kernel, grid, block, shmem, stream, ...)                      \
    do {                                                                               \
        ::rb3::ProfScope _ps(name, stream);                                            \
        hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);           \
        RB3_TRY(::rb3::check_launch(name));                                            \
    } while (0)

// Grid for a grid-stride loop over `work` items with `per_block` items/block.
inline dim3 grid_for(int64_t work, int64_t per_block, int64_t cap = 1 << 20) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return dim3((unsigned)g);
}

// ---------------------------------------------------------------------------
// Host launchers implemented in the .hip files
// ---------------------------------------------------------------------------

// index.hip
int encode_strands(Ctx &c, const uint8_t *d_seq, const int64_t *lens, int64_t n_in, int32_t both,
                   uint8_t *d_Q, int64_t n_out, int32_t *d_err);
int encode_plain(Ctx &c, const uint8_t *d_seq, const int64_t *lens, int64_t n_in, uint8_t *d_codes,
                 int64_t total, int32_t *d_err);
int pack_codes(Ctx &c, const uint8_t *d_codes, int64_t n, uint4 *d_blk);
int build_checkpoints(Ctx &c, uint4 *d_blk, int64_t n, int64_t *d_sb, int64_t C_out[6],
                      int64_t counts_out[6]);
int unpack_codes(Ctx &c, const DevIndex &ix, uint8_t *d_codes);
int check_codes(Ctx &c, const uint8_t *d_codes, int64_t n, int32_t *d_err);

// scan.hip
int scan_u32(Ctx &c, const uint32_t *d_in, uint32_t *d_out, int64_t n, bool inclusive,
             bool max_op, uint32_t *d_total);

// sort.hip: stable LSD radix sort of (key, value) by key bits [lo_bit, hi_bit).
// If vals_in is null the values are the input indices. Result lands in
// (*k_res, *v_res), one of the two buffer pairs.
// The input pair (k_in, v_in) is left untouched.
int radix_sort(Ctx &c, uint64_t *k_in, uint32_t *v_in, uint64_t *k_a, uint32_t *v_a, uint64_t *k_b,
               uint32_t *v_b, int64_t n, int lo_bit, int hi_bit, bool iota_vals, uint64_t **k_res,
               uint32_t **v_res, int32_t *d_guard, int *used_packed, int *used_passes = nullptr);

// A piece of a new strand walked by one lane of the LF-chain kernel.
struct Chunk {
    int64_t p0;     // position in Q of the chunk's first symbol
    int32_t len;    // symbols in the chunk
    int32_t last;   // 1 if the chunk ends at the strand's sentinel
    int32_t first;  // 1 if the chunk starts at the strand's first symbol
    int32_t pad;
};

// Zero bytes after the last code of a merge batch (Q): word and line reads
// past the end stay inside the buffer.
constexpr int64_t Q_PAD = 128;

// chunks.hip: the chunks of the n2 codes at d_Q (strands each followed by
// their sentinel, Q_PAD zero bytes past the end), in string order, at most
// lmax symbols each and cut at content-defined positions; perm receives the
// order in which the chain kernel's lanes take them (uint32 chunk indices).
int make_chunks(Ctx &c, const uint8_t *d_Q, int64_t n2, int64_t lmax, DBuf &chunks, int64_t *nch_out, DBuf &perm,
                int32_t *d_guard);

// api.cpp: the merge-failure test hook (rb3_test_fail_merge_after). Returns
// RB3_EDEVICE, with a message, when the hook names this stage of a merge
// (1 insertion ranks, 2 radix sort, 3 tie resolution, 4 interleave, 5
// checkpoints), else RB3_OK.
int fault_point(int stage);

// merge.hip
struct MergeStats {
    int64_t n1 = 0, m1 = 0, n2 = 0, m2 = 0;
    uint32_t group_hist[32] = {};  // mixed-symbol tied groups by floor(log2(size))
    int64_t chunks = 0, chunk_len = 0;
    int64_t chain_steps = 0;      // rank steps in the chain phase (point + interval)
    int64_t fixup_steps = 0;      // rank steps replayed by fix-up passes
    int64_t fixup_index_steps = 0;  // fix-up steps whose interval spanned more than 64 rows (read the index)
    int64_t fixup_segments = 0;   // segments of the fix-up's folded rank maps
    int64_t fixup_passes = 0;
    int64_t fixup_run_max = 0;    // most chunks one fix-up lane completed
    int64_t key_syms = 0;         // symbols per initial sort key
    int64_t sort_bits = 0;
    int64_t sort_packed = 0;      // 1 when the sort moved packed 8-byte records
    int64_t sort_passes = 0;      // passes over the records (8-bit digits)
    int64_t tied_records = 0;     // records in non-singleton groups after the sort
    int64_t tie_groups = 0;       // tied groups whose members carry different symbols
    int64_t tie_pairs = 0;        // ... of which have two members
    int64_t tie_block_reads = 0;  // chunk reads refining groups of more than 64
    int64_t tie_small_reads = 0;  // key reads refining groups of 2..8
    int64_t tie_max_depth = 0;    // deepest comparison those needed
    int64_t tie_deep_reads = 0;   // key reads of groups handed to the deep walk
    int64_t max_group = 0;        // largest such group
    int64_t tie_doubling = 0;     // 1 if prefix doubling ordered the ties
    int64_t tie_rounds = 0;       // doubling rounds
    int64_t tie_work = 0;         // key reads of the symbol walk over groups of 9+,
                                  // or active records summed over doubling rounds
};

// Suffix-array samples (Sec. 2.4), kept by text position: the suffix at
// position p of a merge batch is sampled when p is a multiple of the
// sampling distance s or starts its strand, so every strand has a sample at
// offset 0 and at least one in any s consecutive positions. A bit per BWT
// row marks the sampled rows: per 128-row block one 32-byte record of four
// words (the block's two bit words, the number of samples before the block,
// padding), so that a locate step reads one line for its block's samples.
// val holds each sampled row's position, in row order, packed as
// strand << SMP_ID_SHIFT | offset.
constexpr int SMP_ID_SHIFT = 40;
constexpr uint64_t SMP_OFF_MASK = (1ull << SMP_ID_SHIFT) - 1;
constexpr int64_t SMP_MAX_STRANDS = (int64_t)1 << (64 - SMP_ID_SHIFT);

constexpr int SMP_REC = 4;  // words per block record

struct DevSmp {
    const uint64_t *rec;   // SMP_REC words per block (fewer than 2^32 samples)
    const uint64_t *val;   // nsmp
    int64_t nsmp;
    int32_t rate;
};

struct IndexData {
    Ctx ctx;
    int64_t n = 0, m = 0;
    int64_t C[6] = {0, 0, 0, 0, 0, 0};
    uint4 *blk = nullptr;  // owned
    int64_t *sb = nullptr; // owned
    // samples (owned; null when ctx.ssa == 0)
    uint64_t *smp_rec = nullptr;
    uint64_t *smp_val = nullptr;
    int64_t nsmp = 0;
    MergeStats last;
    DevSmp smp() const {
        DevSmp s;
        s.rec = smp_rec;
        s.val = smp_val;
        s.nsmp = nsmp;
        s.rate = ctx.ssa;
        return s;
    }
    DevIndex dev() const {
        DevIndex d;
        d.blk = blk;
        d.sb = sb;
        d.n = n;
        d.m = m;
        for (int i = 0; i < 6; ++i) d.C[i] = C[i];
        d.C[6] = n;
        d.C[7] = 0;
        return d;
    }
};

// d_Q: the n2 codes of the m2 new strands, each followed by its sentinel
// (code 0), then Q_PAD zero bytes of padding.
// With samples (ix.ctx.ssa > 0) the merged index's sample arrays are
// returned through smp (bits, cnt, val, nsmp); otherwise smp is untouched.
struct SmpOut {
    uint64_t *rec = nullptr;
    uint64_t *val = nullptr;
    int64_t nsmp = 0;
};
int merge_into(Ctx &c, IndexData &ix, const uint8_t *d_Q, const int64_t *strand_lens, int64_t m2,
               int64_t n2, uint4 **new_blk, int64_t **new_sb, int64_t new_C[6], MergeStats &st,
               SmpOut *smp);

// Rank of sampled rows before row r (and whether r is sampled): the count of
// r's block plus the set bits below r in it. Rows up to n are valid.
__device__ __forceinline__ bool smp_rank_rec(const uint64_t *rec, int64_t r, int64_t *rank) {
    const uint64_t *q = rec + (r >> BLK_SHIFT) * SMP_REC;
    const uint64_t w0 = q[0], w1 = q[1];
    const int64_t c = (int64_t)(uint32_t)q[2];
    const int o = (int)(r & (BLK_SYMS - 1));
    if (o < 64) {
        *rank = c + __popcll(w0 & low_mask(o));
        return (w0 >> o) & 1ull;
    }
    *rank = c + __popcll(w0) + __popcll(w1 & low_mask(o - 64));
    return (w1 >> (o - 64)) & 1ull;
}
__device__ __forceinline__ bool smp_rank(const DevSmp &s, int64_t r, int64_t *rank) {
    return smp_rank_rec(s.rec, r, rank);
}

// locate.hip
// Position (strand, offset) of each row: LF steps until a sampled row.
int locate_rows(Ctx &c, const DevIndex &ix, const DevSmp &sm, const int64_t *d_rows, int64_t n,
                int64_t *d_strand, int64_t *d_off, int32_t *d_err, unsigned long long *d_steps);
// One occurrence in each SA interval [lo, hi) (Locate1, Algorithm 2).
int locate_one(Ctx &c, const DevIndex &ix, const DevSmp &sm, const int64_t *d_lo, const int64_t *d_hi,
               int64_t n, int64_t *d_strand, int64_t *d_off, int32_t *d_err, unsigned long long *d_steps);

// query.hip
int count_queries(Ctx &c, const DevIndex &ix, const uint8_t *d_q, const int64_t *d_qoff,
                  int64_t nq, int64_t *d_lo, int64_t *d_hi);
// Query positions per SMEM segment: the batch's bases over
// SMEM_TARGET_SEGS, within [SMEM_SEG_MIN, SMEM_SEG].
constexpr int64_t SMEM_SEG = 4096;
constexpr int64_t SMEM_SEG_MIN = 32;
constexpr int64_t SMEM_SEG_BUSY = 128;  // shortest segment when batches share the GPU
constexpr int64_t SMEM_TARGET_SEGS = 262144;
// SMEMs of nq queries (codes at d_q, host lengths qlens). d_out_off
// (device, nq + 1) receives the per-query offsets; when all *h_kept reports
// fit in out_cap they are written in order to d_out. h_exts[0]: bi-interval
// extensions performed, h_exts[1]: distinct index blocks they read.
int smem_run(Ctx &c, const DevIndex &ix, const uint8_t *d_q, const int64_t *qlens, int64_t nq, int32_t min_len,
             int64_t min_occ, int64_t out_cap, rb3_smem_t *d_out, int64_t *d_out_off, int64_t *h_kept,
             int64_t *h_exts);

// hapl.hip: local haplotype enumeration (Algorithm 5 and the bi-interval
// filter) of nq queries (codes at d_codes, host lengths qlens) on ix, or on
// the run-length index when rle is set. Queries run in chunks whose cell
// tables fit HAPL_SCRATCH bytes. h_off (host, nq + 1) receives the
// per-query offsets; when everything fits out_cap the records are written
// in order to d_out. A query that needs more than o.max_cells cells at a
// position gives RB3_ELIMIT with its index in *h_bad. h_stats[0..3]:
// extensions (rank-all pairs), index blocks they read, cells held summed
// over the query positions, queries moved from LDS to device-memory tables.
constexpr int64_t HAPL_SCRATCH = (int64_t)16 << 30;
// A cell's scores travel packed with the reverse-complement start of their
// representative string in the low HAPL_KRC_BITS bits: the index must hold
// fewer than 2^HAPL_KRC_BITS symbols (and scores stay below 2^29).
constexpr int HAPL_KRC_BITS = 35;
struct RleView;
int hapl_run(Ctx &c, const DevIndex &ix, const RleView *rle, const uint8_t *d_codes, const int64_t *qlens,
             int64_t nq, const rb3_hapl_opts &o, int64_t out_cap, rb3_hapl_t *d_out, int64_t *h_off,
             int64_t *h_bad, int64_t *h_stats);

// api.cpp: one synchronous count / SMEM call on a context's stream (the
// caller flushes the context afterwards). total = sum of qlens. With rle
// set the call runs on that run-length index instead of ix.
struct RleView;
int run_count(Ctx &c, const DevIndex &ix, const uint8_t *q, const int64_t *qlens, int64_t n_q, int64_t total,
              int32_t mem, int64_t *lo, int64_t *hi, const RleView *rle = nullptr);
int run_smem(Ctx &c, const DevIndex &ix, const uint8_t *q, const int64_t *qlens, int64_t n_q, int64_t total,
             int32_t mem, int32_t min_len, int64_t min_occ, rb3_smem_t *out, int64_t out_cap, int64_t *out_off,
             int64_t *exts, const RleView *rle = nullptr);
// tune.cpp: the autotuner's table (see rb3_tune_merge / rb3_tune_smem).
std::string merge_tune_key(int dev, int64_t n1, int64_t n2, int64_t m2);
std::string smem_tune_key(int dev, int64_t n, int64_t bases, int64_t nq);
int64_t tuned_chunk_len(int dev, int64_t n1, int64_t n2, int64_t m2);        // 0: none
int64_t tuned_smem_segment(int dev, int64_t n, int64_t bases, int64_t nq);   // 0: none, -1: automatic
void tune_store(const std::string &key, int64_t v);

const DevIndex index_dev(const rb3_index *idx);
hipStream_t index_stream(const rb3_index *idx);
// noalloc.hip: rb3_count with every temporary in the library's fixed
// scratch array (no allocation). Arguments checked by the caller.
int count_noalloc(const DevIndex &ix, int dev, hipStream_t stream, const uint8_t *q, const int64_t *qlens,
                  int64_t n_q, int64_t total, int32_t mem, int64_t *lo, int64_t *hi);
int index_device(const rb3_index *idx);
int32_t index_both(const rb3_index *idx);

}  // namespace rb3
