/*
 * rb3.h - C ABI of the MI355X (gfx950) multi-string BWT library.
 *
 * The library keeps a multi-string Burrows-Wheeler transform of DNA strings
 * resident in device memory, merges new strings into it, and answers
 * backward-search counts and SMEM queries on it. The operations follow
 * H. Li, "BWT construction and search at the terabase scale" (arXiv
 * 2409.00613):
 *   - the BWT of an ordered string list with sentinels ordered by string
 *     index (Sec. 2.1), stored with both strands by default (Sec. 2.5);
 *   - merging new strings into an existing BWT (Sec. 2.2, Algorithm 1);
 *   - SA-interval counting by backward search (Sec. 2.3);
 *   - SMEM finding over SA bi-intervals (Sec. 2.5-2.6, Algorithms 3-4).
 *
 * Conventions shared by every call:
 *   - Every function returns int: RB3_OK (0) on success, a negative RB3_E*
 *     code otherwise. rb3_strerror() gives a message; for RB3_EDEVICE the
 *     message includes the HIP error of the failing call (thread-local).
 *     Nothing throws across the ABI.
 *   - Input strings are passed as ONE buffer of concatenated bytes plus a
 *     host array of int64 lengths. Bytes are ACGTN in either case; any other
 *     byte, and any string of length 0, gives RB3_EINVAL. The buffer lives in
 *     host memory (mem = RB3_MEM_HOST) or in device memory of the index's
 *     device (mem = RB3_MEM_DEVICE); the lengths are always host memory.
 *   - Symbol codes, where codes cross the ABI: $=0 A=1 C=2 G=3 T=4 N=5, the
 *     order $ < A < C < G < T < N of Sec. 2.2.
 *   - All positions and counts are int64.
 *   - The caller owns every buffer it passes; the library reads inputs and
 *     writes outputs only during the call. The library owns rb3_index objects
 *     until rb3_index_free().
 *   - Calls are synchronous: they enqueue work on the index's stream and
 *     return after it has completed.
 *   - Read-only calls (count, smem, info, export, clone) on one index may run
 *     concurrently from several host threads; rb3_merge needs exclusive
 *     access to its index.
 */
#ifndef RB3_H
#define RB3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RB3_OK = 0,
    RB3_EINVAL = -1,   /* bad argument: NULL, bad byte, empty string, bad size */
    RB3_ENOMEM = -2,   /* device or host allocation failed */
    RB3_EDEVICE = -3,  /* a HIP runtime call or kernel failed */
    RB3_ENOSPC = -4,   /* caller output buffer too small (sizes are reported) */
    RB3_ELIMIT = -5,   /* input beyond a documented size limit */
    RB3_EAGAIN = -6    /* the server's queue is full: poll results, then retry */
};

enum { RB3_MEM_HOST = 0, RB3_MEM_DEVICE = 1 };

/* Device-resident index: the BWT as 3-bit symbols in 64-byte blocks of 128
 * symbols with occurrence checkpoints, superblock counts and C[]. */
typedef struct rb3_index rb3_index;

/* Device allocator hooks. dev_alloc returns NULL on failure, else memory
 * aligned to at least 16 bytes (hipMalloc and PyTorch's caching allocator
 * give 256); a misaligned pointer is handed back to dev_free and the call
 * fails with RB3_ENOMEM. */
typedef void *(*rb3_alloc_fn)(size_t bytes, void *ctx);
typedef void (*rb3_free_fn)(void *ptr, void *ctx);

typedef struct rb3_opts {
    int32_t both_strands;  /* 1 (default): each input string P is followed by
                              its reverse complement, giving the list P0, rc(P0),
                              P1, rc(P1), ... of Sec. 2.5. 0: strings as given. */
    int32_t device;        /* HIP device ordinal (default 0) */
    void *stream;          /* hipStream_t for all work; NULL: a stream the
                              library creates for this index */
    rb3_alloc_fn dev_alloc; /* NULL: hipMalloc/hipFree */
    rb3_free_fn dev_free;
    void *alloc_ctx;
    int64_t chunk_len;     /* longest LF-chain chunk of a merge (chunks are cut
                              at content-defined positions, at most this long);
                              0 = default (2048, doubled while a batch would
                              make more than 2^17 chunks of that length) */
    int32_t launch_per_string; /* 0 (default): one launch of the LF-chain
                              kernel covers every chunk of every new string
                              of a merge. 1: the plain form, one launch per
                              new string (over that string's chunks); same
                              result, for measuring what batching gains. */
    int32_t ssa_rate;      /* suffix-array sampling distance s for rb3_locate
                              and rb3_locate1 (Sec. 2.4); 0 (default): no
                              samples. Taken at rb3_build and kept by every
                              merge: a suffix is sampled when its position in
                              its merge batch (the strands of the batch laid
                              end to end, each with its sentinel) is a
                              multiple of s, or when it starts its strand, so
                              a locate needs at most s - 1 LF steps. Costs
                              two bits per row plus 8 bytes per sample; an
                              index keeps fewer than 2^32 samples and 2^24
                              strands (RB3_ELIMIT otherwise). */
    int32_t occ_interval;  /* occurrence-checkpoint interval I of the index
                              (symbols per checkpoint, Table 1's occ sampled
                              every I symbols): 0 (default) = the library's
                              choice, else 128; other values give RB3_EINVAL. */
    int32_t smem_segment;  /* rb3_smem cuts long queries into segments of this
                              many positions, each searched by its own lane
                              (results do not depend on it). 0 (default): the
                              length rb3_tune_smem chose for the batch's size
                              class, else from the batch size (32 .. 4096).
                              Else 1 .. 2^20. */
} rb3_opts;

/* Fill *o with the defaults above. */
void rb3_opts_init(rb3_opts *o);

/*
 * rb3_build: the BWT of the ordered list expand(strings) (Sec. 2.1; with
 * both_strands, the double-strand list of Sec. 2.5). Equivalent to merging
 * the strings into an empty index.
 *   seq, lens, n_seqs, mem: the input strings (see conventions).
 *   *out receives a new index on success and is untouched on error.
 */
int rb3_build(const rb3_opts *o, const uint8_t *seq, const int64_t *lens, int64_t n_seqs,
              int32_t mem, rb3_index **out);

/*
 * rb3_merge: idx := BWT(list(idx) ++ expand(strings)) (Sec. 2.2, Algorithm 1).
 * Every sentinel already in idx orders before every new sentinel, and new
 * strings keep their input order. Per batch the number of new symbols
 * (sum of lengths plus one sentinel per strand) must be below 2^32 - 2^20
 * (RB3_ELIMIT otherwise). On error idx is unchanged.
 */
int rb3_merge(rb3_index *idx, const uint8_t *seq, const int64_t *lens, int64_t n_seqs,
              int32_t mem);

/*
 * rb3_count: SA interval [lo, hi) of each query by backward search
 * (Sec. 2.3): lo = number of suffixes smaller than the query, hi - lo =
 * number of occurrences. Queries are NOT reverse complemented. An empty
 * query gives [0, n). lo and hi are host arrays of n_q entries.
 */
int rb3_count(const rb3_index *idx, const uint8_t *q, const int64_t *qlens, int64_t n_q,
              int32_t mem, int64_t *lo, int64_t *hi);

/*
 * rb3_count_noalloc: rb3_count for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same arguments and results as rb3_count, except that lo
 * and hi are in the same memory as the queries (mem): host arrays for host
 * queries, device arrays for device queries. The call allocates nothing: its
 * temporaries (error flag, query offsets, symbol codes, and the staged
 * results when they go to host memory) live in one fixed scratch array of
 * RB3_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on
 * until the process ends. Queries that need more scratch than that give
 * RB3_ELIMIT: 256 bytes + the query bytes + 8 bytes per query (+ 16 bytes per
 * query for host results), each part rounded up to 256 bytes. Every call on
 * a device shares that device's array; the array keeps the last call's
 * contents, and calls from several host threads on one device take turns on
 * a lock (left to overlap they would race on the array).
 */
#define RB3_NOALLOC_SCRATCH_BYTES (32u << 20)
int rb3_count_noalloc(const rb3_index *idx, const uint8_t *q, const int64_t *qlens, int64_t n_q,
                      int32_t mem, int64_t *lo, int64_t *hi);

/* One SMEM: query interval [start, end), its occurrence count occ, and its
 * SA bi-interval starts k = lo(P[start,end)), krc = lo(rc(P[start,end)))
 * (Sec. 2.5). */
typedef struct rb3_smem_t {
    int64_t start, end, occ, k, krc;
    int32_t qid;
    int32_t pad;
} rb3_smem_t;

/*
 * rb3_smem: SMEMs of each query no shorter than min_len that occur at least
 * min_occ times (Sec. 2.6, Algorithm 4 over the extensions of Algorithm 3).
 * Results for query i are out[out_off[i] .. out_off[i+1]) in increasing
 * start. out (host, out_cap entries) and out_off (host, n_q + 1 entries)
 * are caller buffers. If out_cap is too small the call returns RB3_ENOSPC
 * with out_off filled, so the caller can size a retry. min_len >= 1 and
 * min_occ >= 1, else RB3_EINVAL. The index must hold both strands.
 */
int rb3_smem(const rb3_index *idx, const uint8_t *q, const int64_t *qlens, int64_t n_q,
             int32_t mem, int32_t min_len, int64_t min_occ, rb3_smem_t *out, int64_t out_cap,
             int64_t *out_off);

/* Work done by the calling thread's last successful rb3_smem call: the
 * number of bi-interval extensions (each reads rank-all at two positions,
 * k and k + s) and the number of distinct 64-byte index blocks those reads
 * touched (one per extension when both positions share a block, else two).
 * Either pointer may be NULL. */
int rb3_last_smem_stats(int64_t *extensions, int64_t *blocks);

/*
 * Local haplotype enumeration (Sec. 2.7-2.8, Algorithm 5): each query P is
 * aligned end to end (semi-globally) to the prefix DAWG of the index under
 * affine gaps, walking P from its end to its start. A DAWG node is an SA
 * interval (k, s); its children are its non-empty backward extensions by
 * A, C, G, T (Algorithm 3). A node holds every string with that interval
 * (X and XZ when each occurrence of X is followed by Z), whose reverse
 * complements have intervals of size s starting at different rows krc: a
 * cell reports the krc of the string with the smallest krc among the
 * node's strings whose alignment attains the cell's score. At each query position
 * the cells come from the previous position's cells by a match or mismatch
 * to a child (score match, or -mismatch; a query N mismatches every symbol)
 * and by an insertion (same node), then from the position's own cells by
 * deletions to children, repeated until no cell improves; a gap of length L
 * costs gap_open + L * gap_ext. Cells with score <= 0 are dropped and, with
 * band W > 0, only the W best cells are kept (ties: smaller k, then smaller
 * s). The start cell (query end, the whole index) has score 0. The result is
 * the cells left at the query's start, by decreasing score (same ties),
 * without those whose [k, k+s) or [krc, krc+s) lies inside the same
 * interval of a result before them.
 */
typedef struct rb3_hapl_opts {
    int32_t match;     /* score of a match, 1 .. 2^20 (default 1) */
    int32_t mismatch;  /* mismatch penalty, 0 .. 2^20 (default 4) */
    int32_t gap_open;  /* 0 .. 2^20 (default 6) */
    int32_t gap_ext;   /* 1 .. 2^20 (default 1) */
    int32_t band;      /* W, cells kept per query position; 0 keeps all (default 25) */
    int32_t max_cells; /* cells one query position may hold before the band, 1 .. 65535; 0 (default):
                          8 * band + 256 with a band, else 4096 */
    int32_t device_tables; /* 0 (default): each query's cells in LDS (half a wavefront's at bands up
                              to 32, a whole one's otherwise) while they fit (64, 128 or 256 a
                              position by band), else in device memory; 1: always in device memory */
} rb3_hapl_opts;

void rb3_hapl_opts_init(rb3_hapl_opts *o);

/* One result: the bi-interval (k, krc, s) and the alignment score. */
typedef struct rb3_hapl_t {
    int64_t k, krc, s;
    int32_t score;
    int32_t qid;
} rb3_hapl_t;

/*
 * rb3_hapl: the enumeration above for n_q queries (q, qlens, mem as in
 * rb3_count; o NULL = defaults). Results for query i are out[out_off[i] ..
 * out_off[i+1]) in result order; out (host, out_cap entries) and out_off
 * (host, n_q + 1) are caller buffers. RB3_ENOSPC when out_cap is too small
 * (out_off filled, so the caller can size a retry); RB3_ELIMIT when a query
 * needs more than max_cells cells at one position, match times a query's
 * length reaches 2^29, or the index holds 2^35 symbols or more; RB3_EINVAL
 * on options out of range or an index without both strands. With a band,
 * the deletion step holds only
 * the cells that can still reach the band (a cell is extended only when
 * the F it passes on is at least the band's lowest score so far), which
 * leaves the band's cells and scores unchanged. Device memory: the
 * results of the queries in flight (32 bytes each, at most the band's
 * number a query), and, for queries kept in device memory, about
 * 2 * max_cells * 48 + 12 * max_cells bytes each; queries run in chunks
 * whose device-memory tables would take at most 16 GiB (allocated only for
 * the queries moved there).
 */
int rb3_hapl(const rb3_index *idx, const rb3_hapl_opts *o, const uint8_t *q, const int64_t *qlens, int64_t n_q,
             int32_t mem, rb3_hapl_t *out, int64_t out_cap, int64_t *out_off);

/* Work done by the calling thread's last rb3_hapl or rb3_rle_hapl call that
 * reached the device: node extensions (each reads rank-all at k and k + s),
 * the index blocks those reads touched (as in rb3_last_smem_stats), the
 * cells held summed over all query positions, and the queries whose cells
 * outgrew the LDS tables and were finished in device memory. Any pointer
 * may be NULL. */
int rb3_last_hapl_stats(int64_t *extensions, int64_t *blocks, int64_t *cells, int64_t *moved);

/*
 * rb3_locate: position of the suffix at each row (Sec. 2.4): strand[i] is
 * the index of the strand holding row rows[i]'s suffix in the index's list
 * (strands numbered in the order they were added, both strands counted) and
 * offset[i] its offset in that strand (the strand's length for its
 * sentinel suffix). rows, strand and offset: n entries each, all in host
 * or all in device memory (mem); every row must be in [0, n_index), else
 * RB3_EINVAL. The index must have samples (ssa_rate > 0), else RB3_EINVAL.
 */
int rb3_locate(const rb3_index *idx, const int64_t *rows, int64_t n, int32_t mem, int64_t *strand,
               int64_t *offset);

/*
 * rb3_locate1: one occurrence in each SA interval [lo[i], hi[i]) (Locate1 of
 * Algorithm 2: the largest remaining interval is tested for a sampled row,
 * else extended backwards by every symbol). Outputs as rb3_locate; an empty
 * interval gives strand = offset = -1. Intervals must satisfy
 * 0 <= lo <= hi <= n_index, else RB3_EINVAL. Which occurrence is returned is
 * not specified; it is always one whose row lies in [lo, hi).
 */
int rb3_locate1(const rb3_index *idx, const int64_t *lo, const int64_t *hi, int64_t n, int32_t mem,
                int64_t *strand, int64_t *offset);

/* Sampling distance (0: no samples) and number of samples of an index. */
int rb3_ssa_info(const rb3_index *idx, int32_t *rate, int64_t *nsamples);

/* LF or rank-all steps taken by the calling thread's last successful
 * rb3_locate / rb3_locate1 call. */
int rb3_last_locate_stats(int64_t *lf_steps);

/* Size of the BWT n, number of sentinels m, and C[c] = number of symbols
 * smaller than c (Table 1) for c = 0..5. Any output pointer may be NULL. */
int rb3_info(const rb3_index *idx, int64_t *n, int64_t *m, int64_t C[6]);

/* Write the BWT as n symbol codes into codes (host, n bytes). */
int rb3_export(const rb3_index *idx, uint8_t *codes);

/* Build an index from n BWT symbol codes (host or device per mem), the BWT
 * of m strands whose lengths (sentinels excluded) are lens[0..m) (host).
 * Symbol-count check (Sec. 2.1: a BWT of m sentinel-terminated strings holds
 * each string's symbols plus one $ per string): the codes must be 0..5, hold
 * exactly m sentinels (0), and n must equal sum(lens[j] + 1); otherwise
 * RB3_EINVAL. Beyond these counts the codes are taken as given: the call
 * does not walk them to check that they form a BWT. */
int rb3_import(const rb3_opts *o, const uint8_t *codes, int64_t n, const int64_t *lens, int64_t m,
               int32_t mem, rb3_index **out);

/* Deep copy of an index on the same device. The copy uses the caller's
 * stream if the source was given one; otherwise it gets a stream of its own,
 * so either index may be freed first. The call returns after the copy. */
int rb3_clone(const rb3_index *src, rb3_index **out);

void rb3_index_free(rb3_index *idx);

const char *rb3_strerror(int err);

/*
 * Run-length static index: the BWT in the static, bit-packed run-length
 * form of Sec. 2.2 (Fig. 2b), for indices whose 3-bit-plane form would not
 * fit in device memory. It answers the same counts and SMEMs as the index
 * it was built from (pi_B by decoding, Table 1), but cannot be merged into.
 *
 * Format (all arrays little-endian):
 *   - B[0, n) is cut into segments of 2^20 symbols; each segment into its
 *     maximal runs of one symbol (pieces, at most 2^20 long).
 *   - A piece is coded as its symbol in 3 bits, then its length L in the
 *     Elias delta code (K - 1 zeros, N in K bits, the N - 1 low bits of L,
 *     where N is the bit length of L and K that of N); most significant bit
 *     first.
 *   - blocks: 128-byte blocks of 16 uint64 words. Words 0-1: header; words
 *     2-15: 896 stream bits, stream bit t at bit 63 - t % 64 of word
 *     2 + t / 64, unused bits 0. Header word 0: bits 0-19 the offset of the
 *     block's first symbol in its segment, 20-39 and 40-59 the occurrences
 *     of A and C in the segment before the block, 60-63 the low 4 bits of
 *     the block's piece count; word 1: bits 0-19, 20-39, 40-59 the
 *     occurrences of G, T, N before the block in the segment, 60-63 the
 *     high 4 bits of the piece count. A segment's pieces fill its blocks in
 *     order, greedily (a block takes pieces while their codes fit); every
 *     segment starts a new block.
 *   - segs: (nseg + 1) rows of 8 int64, nseg = ceil(n / 2^20): occurrences
 *     of $, A, C, G, T, N in B before the segment, the index of its first
 *     block, 0. Row nseg holds the totals and the number of blocks.
 *   - row: ((n - 1) >> row_shift) + 1 uint16; entry j is the block holding
 *     position j << row_shift, counted from its segment's first block.
 *
 * The object keeps its arrays in device memory of the index's device (from
 * the index's allocator, which must outlive it) and has a stream of its own,
 * so it outlives the index it was built from.
 */
typedef struct rb3_rle rb3_rle;

/* Build from an index. row_shift: 4..20, or 0 for the automatic choice
 * (the largest value in 4..16 with 2^row_shift <= n / (4 * blocks)). An
 * empty index gives RB3_EINVAL; 2^32 or more pieces give RB3_ELIMIT. */
int rb3_rle_build(const rb3_index *idx, int32_t row_shift, rb3_rle **out);

/* Load the three arrays (host memory; sizes as above, nblocks blocks) on
 * the device of o (NULL: defaults), after checking them against the format:
 * the table on the host, then every block's codes, offsets and header
 * counts and every index-row entry on the device. Data that fail a check
 * give RB3_EINVAL. both != 0 marks an index of both strands (for SMEMs). */
int rb3_rle_load(const rb3_opts *o, const uint64_t *blocks, int64_t nblocks, const int64_t *segs,
                 const uint16_t *row, int64_t n, int32_t row_shift, int32_t both, rb3_rle **out);

/* Sizes: symbols n, sentinels m, pieces (runs cut at segment starts),
 * blocks, the row shift, and the bytes of the three arrays. Any pointer may
 * be NULL. */
int rb3_rle_info(const rb3_rle *r, int64_t *n, int64_t *m, int64_t *runs, int64_t *blocks, int32_t *row_shift,
                 int64_t *bytes);

/* Copy the three arrays to host buffers sized from rb3_rle_info. */
int rb3_rle_image(const rb3_rle *r, uint64_t *blocks, int64_t *segs, uint16_t *row);

/* Decode the whole BWT into codes (host, n bytes). */
int rb3_rle_export(const rb3_rle *r, uint8_t *codes);

/* rb3_count and rb3_smem on the run-length index: same arguments, rules and
 * results. rb3_last_smem_stats then counts the 128-byte blocks decoded. */
int rb3_rle_count(const rb3_rle *r, const uint8_t *q, const int64_t *qlens, int64_t n_q, int32_t mem, int64_t *lo,
                  int64_t *hi);
int rb3_rle_smem(const rb3_rle *r, const uint8_t *q, const int64_t *qlens, int64_t n_q, int32_t mem,
                 int32_t min_len, int64_t min_occ, rb3_smem_t *out, int64_t out_cap, int64_t *out_off);

/* rb3_hapl on the run-length index: same arguments, rules and results. */
int rb3_rle_hapl(const rb3_rle *r, const rb3_hapl_opts *o, const uint8_t *q, const int64_t *qlens, int64_t n_q,
                 int32_t mem, rb3_hapl_t *out, int64_t out_cap, int64_t *out_off);

void rb3_rle_free(rb3_rle *r);

/*
 * Continuous-batching query server over one index.
 *
 * Requests (count or SMEM queries, one string each) are submitted from any
 * thread and answered asynchronously. Worker threads, each with its own HIP
 * stream and device memory pool, take every pending request up to the batch
 * limits whenever they are free, so requests that arrive while earlier
 * batches are on the GPU are admitted as soon as a worker and the device
 * memory budget allow, and batches overlap on the device. Results are the
 * same as those of rb3_count / rb3_smem on the same queries, whatever the
 * batching. The index must stay alive and must not be merged while a server
 * uses it.
 */
typedef struct rb3_server rb3_server;

enum { RB3_REQ_COUNT = 0, RB3_REQ_SMEM = 1 };

typedef struct rb3_server_opts {
    int32_t workers;            /* batches in flight at once (streams); default 4 */
    int32_t pad;
    int64_t max_batch_queries;  /* default 4096 */
    int64_t max_batch_bases;    /* query bases per batch; default 8 Mi */
    int64_t mem_budget;         /* device bytes for requests in flight; 0 (default):
                                   half of the device memory free when the server
                                   is created (at least 64 MiB) */
    int64_t max_queued;         /* requests waiting for a batch; a submission
                                   beyond it gives RB3_EAGAIN; default 65536 */
} rb3_server_opts;

typedef struct rb3_result {
    uint64_t ticket;
    int32_t kind;               /* RB3_REQ_COUNT or RB3_REQ_SMEM */
    int32_t status;             /* RB3_OK or the error of its batch */
    int64_t lo, hi;             /* count: SA interval */
    int64_t smem_off, n_smem;   /* SMEM: records recs[smem_off .. smem_off + n_smem) of the poll */
} rb3_result;

void rb3_server_opts_init(rb3_server_opts *so);
int rb3_server_create(const rb3_index *idx, const rb3_server_opts *so, rb3_server **out);
/* Queue one request; the query is copied. min_len / min_occ are used by SMEM
 * requests (>= 1). Invalid bytes give RB3_EINVAL at submission; a full queue
 * (max_queued requests waiting) gives RB3_EAGAIN and queues nothing. */
int rb3_server_submit(rb3_server *s, int32_t kind, const uint8_t *q, int64_t len, int32_t min_len,
                      int64_t min_occ, uint64_t *ticket);
/* Move finished results into res (res_cap entries) and their SMEM records into
 * recs (rec_cap entries). Waits up to wait_ms for a first result when none is
 * ready. RB3_ENOSPC (with *n_recs = records needed) when the next result does
 * not fit in an empty record buffer. */
int rb3_server_poll(rb3_server *s, int32_t wait_ms, rb3_result *res, int64_t res_cap, rb3_smem_t *recs,
                    int64_t rec_cap, int64_t *n_res, int64_t *n_recs);
/* Queue length, batches in flight, batches run, requests served, largest
 * batch, the time the workers spent running batches (microseconds, summed
 * over workers) and the device-memory budget in use. Any pointer may be
 * NULL. */
int rb3_server_stats(rb3_server *s, int64_t *queued, int64_t *inflight, int64_t *batches, int64_t *served,
                     int64_t *max_batch, int64_t *busy_us, int64_t *mem_budget);
/* Open-loop request driver for latency measurement: submits query i (kind,
 * min_len, min_occ shared) at arrival_s[i] seconds after the call starts
 * (arrival times non-decreasing), polls from a second thread, and writes
 * latency_s[i] = time from the arrival to the result. *wall_s (may be NULL)
 * receives the time until the last result. The results themselves are
 * discarded; results of other requests stay queued for their clients, but no
 * other thread may call rb3_server_poll while a replay runs (it could take
 * the replay's results). A submission refused with RB3_EAGAIN is retried
 * until accepted, its latency counting from its arrival time. The call
 * returns after every request is answered. */
int rb3_server_replay(rb3_server *s, int32_t kind, const uint8_t *q, const int64_t *qlens, int64_t n,
                      int32_t min_len, int64_t min_occ, const double *arrival_s, double *latency_s,
                      double *wall_s);
/* Stops the workers after their current batches; unpolled results are dropped. */
void rb3_server_free(rb3_server *s);

/*
 * Kernel timing. While enabled, every kernel the library launches is
 * bracketed by HIP events on the stream it runs on. rb3_prof_read
 * synchronizes those events and reports, per kernel name, the number of
 * launches and the summed GPU time in milliseconds. Names are copied into
 * names[i*32 .. i*32+31] (NUL-terminated). *n_out receives the number of
 * distinct kernels (entries beyond cap are not written). A merge runs its
 * tie kernels of different group sizes at the same time on three streams
 * (joined before the interleave): their times overlap, and each includes
 * waiting for the compute units the others hold.
 */
int rb3_prof_enable(int on);
int rb3_prof_reset(void);
int rb3_prof_read(char *names, int64_t *launches, double *ms, int64_t cap, int64_t *n_out);

/*
 * Autotuner. rb3_tune_merge times merges of the given strings into copies
 * of idx (idx itself is unchanged) at several LF-chain chunk lengths and
 * keeps the fastest for the size class (GPU architecture, log2 of the index
 * size, of the batch size and of the mean strand length); later merges with
 * chunk_len = 0 in their options use it. rb3_tune_smem times rb3_smem on the
 * given queries at several segment lengths (and the automatic rule) and
 * keeps the fastest for (architecture, log2 index size, log2 batch bases,
 * log2 mean query length); rb3_smem with smem_segment = 0 uses it (-1 in
 * *segment: the automatic rule won). The table is per process; with the
 * environment variable RB3_TUNE_CACHE set to a file path it is also read
 * from and written to that file. cand / ms (cap entries, may be NULL with
 * cap 0) receive each candidate and its time in milliseconds, *n_out their
 * number. The calls allocate like the merge / SMEM calls they time (the
 * merge tuner also a copy of the index).
 */
int rb3_tune_merge(rb3_index *idx, const uint8_t *seq, const int64_t *lens, int64_t n_seqs, int32_t mem,
                   int64_t *chunk_len, int64_t *cand, double *ms, int64_t cap, int64_t *n_out);
int rb3_tune_smem(const rb3_index *idx, const uint8_t *q, const int64_t *qlens, int64_t n_q, int32_t mem,
                  int32_t min_len, int64_t min_occ, int64_t *segment, int64_t *cand, double *ms, int64_t cap,
                  int64_t *n_out);

/*
 * Test hook for failure handling: while stage is nonzero, every rb3_merge
 * and rb3_build in the process stops after that stage of the merge and
 * returns RB3_EDEVICE (1 insertion ranks by LF chains, 2 radix sort of the
 * new suffixes, 3 ordering of tied suffixes, 4 interleave into the merged
 * BWT, 5 checkpoint rebuild), after the kernels already queued have run to
 * completion. 0 switches it off. The merge's strong guarantee means the
 * index is then unchanged; tests use this (with an allocator hook that
 * fails at a chosen allocation) to check that guarantee at every stage.
 */
int rb3_test_fail_merge_after(int32_t stage);

/* Last merge statistics: per-stage counters useful for throughput accounting
 * (suffixes inserted, rank steps, tie rounds, ...). keys receives up to cap
 * 32-byte names, vals their values. */
int rb3_merge_stats(const rb3_index *idx, char *keys, int64_t *vals, int64_t cap, int64_t *n_out);

#ifdef __cplusplus
}
#endif

#endif /* RB3_H */
