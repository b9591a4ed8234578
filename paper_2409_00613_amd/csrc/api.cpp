// C ABI of the library (see include/rb3.h): argument checks, host/device
// staging, ownership, error reporting and kernel-time profiling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "rb3_internal.h"
#include "rle.h"

struct rb3_index {
    rb3::IndexData d;
};

// Run-length static index: its arrays on the device and its own stream, so
// it outlives the index it was built from.
struct rb3_rle {
    rb3::Ctx ctx;
    uint64_t *blk = nullptr;
    int64_t *seg = nullptr;
    uint16_t *row = nullptr;
    int64_t n = 0, m = 0, nseg = 0, nblk = 0, npieces = 0;
    int32_t q = 0, both = 0;
    int64_t C[6] = {0, 0, 0, 0, 0, 0};
    rb3::RleView view() const {
        rb3::RleView v;
        v.blk = blk;
        v.seg = seg;
        v.row = row;
        v.n = n;
        v.m = m;
        v.nseg = nseg;
        v.nblk = nblk;
        for (int i = 0; i < 6; ++i) v.C[i] = C[i];
        v.C[6] = n;
        v.C[7] = 0;
        v.q = q;
        return v;
    }
};

namespace rb3 {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;
// work of the last rb3_hapl call of this thread: extensions, blocks, cells,
// queries moved to device-memory tables
static thread_local int64_t g_last_hapl[4] = {0, 0, 0, 0};
// extensions performed by the last rb3_smem call of this thread
static thread_local int64_t g_last_smem_exts[2] = {0, 0};
static thread_local int64_t g_last_locate_steps = 0;
static thread_local int g_err_code = 0;

void set_error(int code, const std::string &msg) {
    g_err_code = code;
    g_err = msg;
}

static int fail(int code, const char *msg) {
    set_error(code, msg);
    return code;
}

static std::atomic<int> g_fail_after{0};

int fault_point(int stage) {
    if (g_fail_after.load(std::memory_order_relaxed) != stage) return RB3_OK;
    set_error(RB3_EDEVICE, "merge stopped after stage " + std::to_string(stage) + " (test hook)");
    return RB3_EDEVICE;
}

int check_launch(const char *name) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(RB3_EDEVICE, std::string("launch of ") + name + ": " + hipGetErrorString(e));
        return RB3_EDEVICE;
    }
    return RB3_OK;
}

// ---------------------------------------------------------------------------
// memory
// ---------------------------------------------------------------------------
void *Ctx::dmalloc(size_t bytes) {
    if (alloc) {
        // kernels read buffers in 16-byte vectors and 8-byte words
        void *p = alloc(bytes, alloc_ctx);
        if (p && ((uintptr_t)p & 15u)) {
            if (free_fn) free_fn(p, alloc_ctx);
            return nullptr;
        }
        return p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void Ctx::free_now(void *p) {
    if (!p) return;
    if (free_fn) free_fn(p, alloc_ctx);
    else (void)hipFree(p);
}

int Ctx::flush() {
    hipError_t e = hipStreamSynchronize(stream);
    for (void *p : deferred) free_now(p);
    deferred.clear();
    if (e != hipSuccess) {
        set_error(RB3_EDEVICE, std::string("stream synchronize: ") + hipGetErrorString(e));
        return RB3_EDEVICE;
    }
    return RB3_OK;
}

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------
namespace {
struct ProfRec {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
std::vector<hipEvent_t> g_prof_pool;
struct Agg {
    int64_t launches = 0;
    double ms = 0;
};
std::map<std::string, Agg> g_prof_agg;

hipEvent_t prof_event() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void prof_drain_locked() {
    for (auto &r : g_prof_pending) {
        float ms = 0;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            Agg &g = g_prof_agg[r.name];
            g.launches += 1;
            g.ms += ms;
        }
        g_prof_pool.push_back(r.a);
        g_prof_pool.push_back(r.b);
    }
    g_prof_pending.clear();
}
}  // namespace

ProfScope::ProfScope(const char *nm, hipStream_t s) : name(nm), stream(s) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    hipEvent_t e = prof_event();
    if (e && hipEventRecord(e, s) == hipSuccess) ev0 = e;
}

ProfScope::~ProfScope() {
    if (!ev0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEvent_t e = prof_event();
    if (e && hipEventRecord(e, stream) == hipSuccess) {
        g_prof_pending.push_back({name, (hipEvent_t)ev0, e});
        if (g_prof_pending.size() > 4096) prof_drain_locked();
    }
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

static int ctx_from_opts(const rb3_opts *o, Ctx &c) {
    rb3_opts d;
    rb3_opts_init(&d);
    if (!o) o = &d;
    c.device = o->device;
    c.alloc = o->dev_alloc;
    c.free_fn = o->dev_free;
    c.alloc_ctx = o->alloc_ctx;
    c.chunk_len = o->chunk_len;
    c.launch_per_string = o->launch_per_string ? 1 : 0;
    c.both = o->both_strands ? 1 : 0;
    if ((c.alloc == nullptr) != (c.free_fn == nullptr)) return fail(RB3_EINVAL, "dev_alloc and dev_free must be given together");
    if (o->ssa_rate < 0 || o->ssa_rate > (1 << 24)) return fail(RB3_EINVAL, "ssa_rate must be in 0 .. 2^24");
    c.ssa = o->ssa_rate;
    if (o->occ_interval != 0 && o->occ_interval != (int32_t)BLK_SYMS)
        return fail(RB3_EINVAL, "occ_interval must be 0 or 128");
    if (o->smem_segment < 0 || o->smem_segment > (1 << 20)) return fail(RB3_EINVAL, "smem_segment must be in 0 .. 2^20");
    c.smem_seg_fixed = o->smem_segment;
    RB3_HIP(hipSetDevice(c.device));
    if (o->stream) {
        c.stream = (hipStream_t)o->stream;
        c.own_stream = false;
    } else {
        RB3_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
        c.own_stream = true;
    }
    return RB3_OK;
}

// A per-call working context: the index's configuration with its own list
// of deferred frees.
static Ctx call_ctx(const IndexData &d) {
    Ctx c;
    c.device = d.ctx.device;
    c.stream = d.ctx.stream;
    c.own_stream = false;
    c.alloc = d.ctx.alloc;
    c.free_fn = d.ctx.free_fn;
    c.alloc_ctx = d.ctx.alloc_ctx;
    c.chunk_len = d.ctx.chunk_len;
    c.launch_per_string = d.ctx.launch_per_string;
    c.both = d.ctx.both;
    c.ssa = d.ctx.ssa;
    c.smem_seg_fixed = d.ctx.smem_seg_fixed;
    return c;
}

// Finish a call: drain the stream, release temporaries, keep the first error.
static int finish(Ctx &c, int rc) {
    int r2 = c.flush();
    return rc != RB3_OK ? rc : r2;
}

static int check_strings(const uint8_t *seq, const int64_t *lens, int64_t n, int32_t mem, bool allow_empty,
                         int64_t *total) {
    if (n < 0 || (n > 0 && !lens)) return fail(RB3_EINVAL, "lengths array is NULL or count negative");
    if (mem != RB3_MEM_HOST && mem != RB3_MEM_DEVICE) return fail(RB3_EINVAL, "mem must be RB3_MEM_HOST or RB3_MEM_DEVICE");
    int64_t t = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (lens[j] < 0 || (!allow_empty && lens[j] == 0)) return fail(RB3_EINVAL, "string of length 0 (or negative)");
        t += lens[j];
    }
    if (t > 0 && !seq) return fail(RB3_EINVAL, "sequence buffer is NULL");
    *total = t;
    return RB3_OK;
}

// Device copy of a caller buffer (or the buffer itself when already there).
static int stage(Ctx &c, const uint8_t *p, int64_t bytes, int32_t mem, DBuf &hold, const uint8_t **dptr) {
    if (mem == RB3_MEM_DEVICE) {
        *dptr = p;
        return RB3_OK;
    }
    RB3_ALLOC(hold, &c, bytes > 0 ? bytes : 1);
    if (bytes > 0) RB3_HIP(hipMemcpyAsync(hold.p, p, bytes, hipMemcpyHostToDevice, c.stream));
    *dptr = hold.as<uint8_t>();
    return RB3_OK;
}

static int read_flag(Ctx &c, const int32_t *d_flag, int32_t *out) {
    RB3_HIP(hipMemcpyAsync(out, d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipStreamSynchronize(c.stream));
    return RB3_OK;
}

static int init_empty(Ctx &c, IndexData &d) {
    // zero symbols: one padding block (code 7 everywhere) and one superblock
    d.n = 0;
    d.m = 0;
    for (int i = 0; i < 6; ++i) d.C[i] = 0;
    DBuf blk, sb;
    RB3_ALLOC(blk, &c, 64);
    RB3_ALLOC(sb, &c, SB_STRIDE * sizeof(int64_t));
    RB3_HIP(hipMemsetAsync(blk.p, 0xFF, 48, c.stream));
    RB3_HIP(hipMemsetAsync((uint8_t *)blk.p + 48, 0, 16, c.stream));
    RB3_HIP(hipMemsetAsync(sb.p, 0, SB_STRIDE * sizeof(int64_t), c.stream));
    if (d.ctx.ssa > 0) {
        // one block's sample record, all zero
        DBuf srec;
        RB3_ALLOC(srec, &c, SMP_REC * sizeof(uint64_t));
        RB3_HIP(hipMemsetAsync(srec.p, 0, SMP_REC * sizeof(uint64_t), c.stream));
        d.smp_rec = srec.as<uint64_t>();
        d.smp_val = nullptr;
        d.nsmp = 0;
        srec.release();
    }
    d.blk = blk.as<uint4>();
    d.sb = sb.as<int64_t>();
    blk.release();
    sb.release();
    return RB3_OK;
}

// Merge expanded strings into d (strong guarantee: d unchanged on error).
static int do_merge(Ctx &c, IndexData &d, const uint8_t *seq, const int64_t *lens, int64_t n_seqs, int32_t mem) {
    int64_t total = 0;
    RB3_TRY(check_strings(seq, lens, n_seqs, mem, false, &total));
    if (n_seqs == 0) return RB3_OK;
    const int k = d.ctx.both ? 2 : 1;
    const int64_t m2 = k * n_seqs;
    const int64_t n2 = k * (total + n_seqs);
    const int64_t limit = (int64_t)UINT32_MAX - (1ll << 20);
    if (n2 >= limit) return fail(RB3_ELIMIT, "batch too large: new symbols must stay below 2^32 - 2^20");
    if (d.m + m2 >= (int64_t)INT32_MAX) return fail(RB3_ELIMIT, "too many strings");
    DBuf hold, Q, err;
    const uint8_t *d_seq = nullptr;
    RB3_TRY(stage(c, seq, total, mem, hold, &d_seq));
    // kernels read whole words and lines past a strand's end: zero bytes follow the codes
    RB3_ALLOC(Q, &c, n2 + Q_PAD);
    RB3_HIP(hipMemsetAsync(Q.as<uint8_t>() + n2, 0, Q_PAD, c.stream));
    RB3_ALLOC(err, &c, sizeof(int32_t));
    RB3_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), c.stream));
    RB3_TRY(encode_strands(c, d_seq, lens, n_seqs, d.ctx.both, Q.as<uint8_t>(), n2, err.as<int32_t>()));
    int32_t bad = 0;
    RB3_TRY(read_flag(c, err.as<int32_t>(), &bad));
    if (bad) return fail(RB3_EINVAL, "byte outside ACGTNacgtn in the input strings");
    hold.reset();
    std::vector<int64_t> slens(m2);
    for (int64_t j = 0; j < n_seqs; ++j)
        for (int s = 0; s < k; ++s) slens[j * k + s] = lens[j];
    uint4 *nb = nullptr;
    int64_t *nsb = nullptr;
    int64_t C[6];
    MergeStats st;
    SmpOut so;
    RB3_TRY(merge_into(c, d, Q.as<uint8_t>(), slens.data(), m2, n2, &nb, &nsb, C, st, &so));
    c.dfree(d.blk);
    c.dfree(d.sb);
    d.blk = nb;
    d.sb = nsb;
    if (d.ctx.ssa > 0) {
        c.dfree(d.smp_rec);
        c.dfree(d.smp_val);
        d.smp_rec = so.rec;
        d.smp_val = so.val;
        d.nsmp = so.nsmp;
    }
    d.n += n2;
    d.m += m2;
    for (int i = 0; i < 6; ++i) d.C[i] = C[i];
    d.last = st;
    return RB3_OK;
}


int run_count(Ctx &c, const DevIndex &ix, const uint8_t *q, const int64_t *qlens, int64_t n_q, int64_t total,
              int32_t mem, int64_t *lo, int64_t *hi, const RleView *rle) {
    DBuf hold, codes, err, off, dlo, dhi;
    const uint8_t *d_q = nullptr;
    RB3_TRY(stage(c, q, total, mem, hold, &d_q));
    RB3_ALLOC(codes, &c, total > 0 ? total : 1);
    RB3_ALLOC(err, &c, sizeof(int32_t));
    RB3_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), c.stream));
    RB3_TRY(encode_plain(c, d_q, qlens, n_q, codes.as<uint8_t>(), total, err.as<int32_t>()));
    std::vector<int64_t> hoff(n_q + 1);
    hoff[0] = 0;
    for (int64_t i = 0; i < n_q; ++i) hoff[i + 1] = hoff[i] + qlens[i];
    RB3_ALLOC(off, &c, (n_q + 1) * sizeof(int64_t));
    RB3_ALLOC(dlo, &c, n_q * sizeof(int64_t));
    RB3_ALLOC(dhi, &c, n_q * sizeof(int64_t));
    RB3_HIP(hipMemcpyAsync(off.p, hoff.data(), (n_q + 1) * sizeof(int64_t), hipMemcpyHostToDevice, c.stream));
    int32_t bad = 0;
    RB3_TRY(read_flag(c, err.as<int32_t>(), &bad));
    if (bad) return fail(RB3_EINVAL, "byte outside ACGTNacgtn in a query");
    if (rle)
        RB3_TRY(count_queries_rle(c, *rle, codes.as<uint8_t>(), off.as<int64_t>(), n_q, dlo.as<int64_t>(),
                                  dhi.as<int64_t>()));
    else
        RB3_TRY(count_queries(c, ix, codes.as<uint8_t>(), off.as<int64_t>(), n_q, dlo.as<int64_t>(),
                              dhi.as<int64_t>()));
    RB3_HIP(hipMemcpyAsync(lo, dlo.p, n_q * sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipMemcpyAsync(hi, dhi.p, n_q * sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipStreamSynchronize(c.stream));
    return RB3_OK;
}

int run_smem(Ctx &c, const DevIndex &ix, const uint8_t *q, const int64_t *qlens, int64_t n_q, int64_t total,
             int32_t mem, int32_t min_len, int64_t min_occ, rb3_smem_t *out, int64_t out_cap, int64_t *out_off,
             int64_t *exts, const RleView *rle) {
    DBuf hold, codes, err, ordered, coff;
    const uint8_t *d_q = nullptr;
    RB3_TRY(stage(c, q, total, mem, hold, &d_q));
    RB3_ALLOC(codes, &c, total > 0 ? total : 1);
    RB3_ALLOC(err, &c, sizeof(int32_t));
    RB3_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), c.stream));
    RB3_TRY(encode_plain(c, d_q, qlens, n_q, codes.as<uint8_t>(), total, err.as<int32_t>()));
    int32_t bad = 0;
    RB3_TRY(read_flag(c, err.as<int32_t>(), &bad));
    if (bad) return fail(RB3_EINVAL, "byte outside ACGTNacgtn in a query");
    RB3_ALLOC(ordered, &c, (out_cap > 0 ? out_cap : 1) * sizeof(rb3_smem_t));
    RB3_ALLOC(coff, &c, (n_q + 1) * sizeof(int64_t));
    int64_t kept = 0;
    if (rle)
        RB3_TRY(smem_run_rle(c, *rle, codes.as<uint8_t>(), qlens, n_q, min_len, min_occ, out_cap,
                             ordered.as<rb3_smem_t>(), coff.as<int64_t>(), &kept, exts));
    else
        RB3_TRY(smem_run(c, ix, codes.as<uint8_t>(), qlens, n_q, min_len, min_occ, out_cap, ordered.as<rb3_smem_t>(),
                         coff.as<int64_t>(), &kept, exts));
    RB3_HIP(hipMemcpyAsync(out_off, coff.p, (n_q + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
    if (kept <= out_cap && kept > 0)
        RB3_HIP(hipMemcpyAsync(out, ordered.p, kept * sizeof(rb3_smem_t), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipStreamSynchronize(c.stream));
    if (kept > out_cap) return fail(RB3_ENOSPC, "SMEM output buffer too small; out_off holds the sizes");
    return RB3_OK;
}

// Options in range, and match times every query length below 2^29 so that
// no score can overflow.
static int check_hapl(const rb3_hapl_opts &o, const int64_t *qlens, int64_t n_q) {
    const int32_t lim = 1 << 20;
    if (o.match < 1 || o.match > lim || o.mismatch < 0 || o.mismatch > lim || o.gap_open < 0 || o.gap_open > lim ||
        o.gap_ext < 1 || o.gap_ext > lim)
        return fail(RB3_EINVAL, "scores out of range");
    if (o.band < 0) return fail(RB3_EINVAL, "band must be >= 0");
    if (o.device_tables != 0 && o.device_tables != 1) return fail(RB3_EINVAL, "device_tables must be 0 or 1");
    if (o.max_cells < 0 || o.max_cells > 65535) return fail(RB3_EINVAL, "max_cells must be in 0 .. 65535");
    for (int64_t i = 0; i < n_q; ++i)
        if (qlens[i] * (int64_t)o.match >= ((int64_t)1 << 29))
            return fail(RB3_ELIMIT, "match score times query length reaches 2^29");
    return RB3_OK;
}

int run_hapl(Ctx &c, const DevIndex &ix, const uint8_t *q, const int64_t *qlens, int64_t n_q, int64_t total,
             int32_t mem, const rb3_hapl_opts &o, rb3_hapl_t *out, int64_t out_cap, int64_t *out_off,
             const RleView *rle) {
    DBuf hold, codes, err, recs;
    const uint8_t *d_q = nullptr;
    RB3_TRY(stage(c, q, total, mem, hold, &d_q));
    RB3_ALLOC(codes, &c, total > 0 ? total : 1);
    RB3_ALLOC(err, &c, sizeof(int32_t));
    RB3_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), c.stream));
    RB3_TRY(encode_plain(c, d_q, qlens, n_q, codes.as<uint8_t>(), total, err.as<int32_t>()));
    int32_t bad = 0;
    RB3_TRY(read_flag(c, err.as<int32_t>(), &bad));
    if (bad) return fail(RB3_EINVAL, "byte outside ACGTNacgtn in a query");
    hold.reset();
    RB3_ALLOC(recs, &c, (out_cap > 0 ? out_cap : 1) * sizeof(rb3_hapl_t));
    int64_t badq = -1;
    int64_t hst[4] = {0, 0, 0, 0};
    const int rc = hapl_run(c, ix, rle, codes.as<uint8_t>(), qlens, n_q, o, out_cap, recs.as<rb3_hapl_t>(), out_off,
                            &badq, hst);
    for (int i = 0; i < 4; ++i) g_last_hapl[i] = hst[i];
    if (rc != RB3_OK) {
        if (badq >= 0) {
            const std::string m = "query " + std::to_string(badq) + " needs more than max_cells (" +
                                  std::to_string(o.max_cells) + ") cells at one position";
            return fail(rc, m.c_str());
        }
        return rc;
    }
    const int64_t kept = out_off[n_q];
    if (kept > out_cap) return fail(RB3_ENOSPC, "haplotype output buffer too small; out_off holds the sizes");
    if (kept > 0) RB3_HIP(hipMemcpyAsync(out, recs.p, kept * sizeof(rb3_hapl_t), hipMemcpyDeviceToHost, c.stream));
    RB3_HIP(hipStreamSynchronize(c.stream));
    return RB3_OK;
}

const DevIndex index_dev(const rb3_index *idx) { return idx->d.dev(); }
int index_device(const rb3_index *idx) { return idx->d.ctx.device; }
hipStream_t index_stream(const rb3_index *idx) { return idx->d.ctx.stream; }
int32_t index_both(const rb3_index *idx) { return idx->d.ctx.both; }

}  // namespace rb3

using namespace rb3;

extern "C" {

void rb3_opts_init(rb3_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->both_strands = 1;
    o->device = 0;
}

const char *rb3_strerror(int err) {
    if (err != RB3_OK && err == g_err_code && !g_err.empty()) return g_err.c_str();
    switch (err) {
    case RB3_OK: return "ok";
    case RB3_EINVAL: return "invalid argument";
    case RB3_ENOMEM: return "out of memory";
    case RB3_EDEVICE: return "device error";
    case RB3_ENOSPC: return "output buffer too small";
    case RB3_ELIMIT: return "size limit exceeded";
    case RB3_EAGAIN: return "queue full, retry later";
    default: return "unknown error";
    }
}

int rb3_build(const rb3_opts *o, const uint8_t *seq, const int64_t *lens, int64_t n_seqs, int32_t mem,
              rb3_index **out) {
    if (!out) return fail(RB3_EINVAL, "out is NULL");
    if (n_seqs < 1) return fail(RB3_EINVAL, "rb3_build needs at least one string");
    int64_t total = 0;
    RB3_TRY(check_strings(seq, lens, n_seqs, mem, false, &total));
    rb3_index *ix = new (std::nothrow) rb3_index();
    if (!ix) return fail(RB3_ENOMEM, "host allocation failed");
    int rc = ctx_from_opts(o, ix->d.ctx);
    if (rc != RB3_OK) {
        delete ix;
        return rc;
    }
    Ctx c = call_ctx(ix->d);
    rc = init_empty(c, ix->d);
    if (rc == RB3_OK) rc = do_merge(c, ix->d, seq, lens, n_seqs, mem);
    rc = finish(c, rc);
    if (rc != RB3_OK) {
        rb3_index_free(ix);
        return rc;
    }
    *out = ix;
    return RB3_OK;
}

int rb3_merge(rb3_index *idx, const uint8_t *seq, const int64_t *lens, int64_t n_seqs, int32_t mem) {
    if (!idx) return fail(RB3_EINVAL, "index is NULL");
    RB3_HIP(hipSetDevice(idx->d.ctx.device));
    Ctx c = call_ctx(idx->d);
    int rc = do_merge(c, idx->d, seq, lens, n_seqs, mem);
    return finish(c, rc);
}

int rb3_count(const rb3_index *idx, const uint8_t *q, const int64_t *qlens, int64_t n_q, int32_t mem,
              int64_t *lo, int64_t *hi) {
    if (!idx) return fail(RB3_EINVAL, "index is NULL");
    if (n_q > 0 && (!lo || !hi)) return fail(RB3_EINVAL, "output arrays are NULL");
    int64_t total = 0;
    RB3_TRY(check_strings(q, qlens, n_q, mem, true, &total));
    if (n_q == 0) return RB3_OK;
    RB3_HIP(hipSetDevice(idx->d.ctx.device));
    Ctx c = call_ctx(idx->d);
    int rc = run_count(c, idx->d.dev(), q, qlens, n_q, total, mem, lo, hi);
    return finish(c, rc);
}

int rb3_count_noalloc(const rb3_index *idx, const uint8_t *q, const int64_t *qlens, int64_t n_q, int32_t mem,
                      int64_t *lo, int64_t *hi) {
    if (!idx) return fail(RB3_EINVAL, "index is NULL");
    if (n_q > 0 && (!lo || !hi)) return fail(RB3_EINVAL, "output arrays are NULL");
    int64_t total = 0;
    RB3_TRY(check_strings(q, qlens, n_q, mem, true, &total));
    if (n_q == 0) return RB3_OK;
    RB3_HIP(hipSetDevice(idx->d.ctx.device));
    return count_noalloc(idx->d.dev(), idx->d.ctx.device, idx->d.ctx.stream, q, qlens, n_q, total, mem, lo, hi);
}

int rb3_smem(const rb3_index *idx, const uint8_t *q, const int64_t *qlens, int64_t n_q, int32_t mem,
             int32_t min_len, int64_t min_occ, rb3_smem_t *out, int64_t out_cap, int64_t *out_off) {
    if (!idx) return fail(RB3_EINVAL, "index is NULL");
    if (!out_off) return fail(RB3_EINVAL, "out_off is NULL");
    if (min_len < 1 || min_occ < 1) return fail(RB3_EINVAL, "min_len and min_occ must be >= 1");
    if (out_cap < 0 || (out_cap > 0 && !out)) return fail(RB3_EINVAL, "bad output buffer");
    if (!idx->d.ctx.both) return fail(RB3_EINVAL, "SMEM finding needs an index of both strands");
    if (n_q >= (int64_t)INT32_MAX) return fail(RB3_ELIMIT, "too many queries");
    int64_t total = 0;
    RB3_TRY(check_strings(q, qlens, n_q, mem, true, &total));
    out_off[0] = 0;
    if (n_q == 0) return RB3_OK;
    RB3_HIP(hipSetDevice(idx->d.ctx.device));
    Ctx c = call_ctx(idx->d);
    int64_t exts[2] = {0, 0};
    int rc = run_smem(c, idx->d.dev(), q, qlens, n_q, total, mem, min_len, min_occ, out, out_cap, out_off, exts);
    if (rc == RB3_OK) {
        g_last_smem_exts[0] = exts[0];
        g_last_smem_exts[1] = exts[1];
    }
    return finish(c, rc);
}

void rb3_hapl_opts_init(rb3_hapl_opts *o) {
    if (!o) return;
    o->match = 1;
    o->mismatch = 4;
    o->gap_open = 6;
    o->gap_ext = 1;
    o->band = 25;
    o->max_cells = 0;
    o->device_tables = 0;
}

// The checks shared by both index forms; *o_out = the options to use.
static int hapl_args(const rb3_hapl_opts *o, const uint8_t *q, const int64_t *qlens, int64_t n_q, int32_t mem,
                     rb3_hapl_t *out, int64_t out_cap, int64_t *out_off, int32_t both, int64_t n,
                     rb3_hapl_opts *o_out, int64_t *total) {
    if (!out_off) return fail(RB3_EINVAL, "out_off is NULL");
    if (out_cap < 0 || (out_cap > 0 && !out)) return fail(RB3_EINVAL, "bad output buffer");
    if (!both) return fail(RB3_EINVAL, "haplotype enumeration needs an index of both strands");
    if (n >= ((int64_t)1 << rb3::HAPL_KRC_BITS))
        return fail(RB3_ELIMIT, "haplotype enumeration needs an index of fewer than 2^35 symbols");
    if (n_q >= (int64_t)INT32_MAX) return fail(RB3_ELIMIT, "too many queries");
    if (o)
        *o_out = *o;
    else
        rb3_hapl_opts_init(o_out);
    RB3_TRY(check_strings(q, qlens, n_q, mem, true, total));
    RB3_TRY(check_hapl(*o_out, qlens, n_q));
    if (o_out->max_cells == 0)
        o_out->max_cells = o_out->band > 0 ? (int32_t)std::min<int64_t>(65535, 8 * (int64_t)o_out->band + 256) : 4096;
    out_off[0] = 0;
    return RB3_OK;
}

int rb3_hapl(const rb3_index *idx, const rb3_hapl_opts *o, const uint8_t *q, const int64_t *qlens, int64_t n_q,
             int32_t mem, rb3_hapl_t *out, int64_t out_cap, int64_t *out_off) {
    if (!idx) return fail(RB3_EINVAL, "index is NULL");
    rb3_hapl_opts oo;
    int64_t total = 0;
    RB3_TRY(hapl_args(o, q, qlens, n_q, mem, out, out_cap, out_off, idx->d.ctx.both, idx->d.n, &oo, &total));
    if (n_q == 0) return RB3_OK;
    RB3_HIP(hipSetDevice(idx->d.ctx.device));
    Ctx c = call_ctx(idx->d);
    int rc = run_hapl(c, idx->d.dev(), q, qlens, n_q, total, mem, oo, out, out_cap, out_off, nullptr);
    return finish(c, rc);
}

int rb3_last_hapl_stats(int64_t *extensions, int64_t *blocks, int64_t *cells, int64_t *moved) {
    if (extensions) *extensions = g_last_hapl[0];
    if (blocks) *blocks = g_last_hapl[1];
    if (cells) *cells = g_last_hapl[2];
    if (moved) *moved = g_last_hapl[3];
    return RB3_OK;
}

int rb3_last_smem_stats(int64_t *extensions, int64_t *blocks) {
    if (extensions) *extensions = g_last_smem_exts[0];
    if (blocks) *blocks = g_last_smem_exts[1];
    return RB3_OK;
}

// Rows or interval ends in host or device memory, as int64 arrays on the
// device.
static int stage_i64(Ctx &c, const int64_t *p, int64_t n, int32_t mem, DBuf &hold, const int64_t **dptr) {
    const uint8_t *d = nullptr;
    RB3_TRY(stage(c, (const uint8_t *)p, n * (int64_t)sizeof(int64_t), mem, hold, &d));
    *dptr = (const int64_t *)d;
    return RB3_OK;
}

static int run_locate(Ctx &c, const IndexData &d, const int64_t *a, const int64_t *b, int64_t n, int32_t mem,
                      int64_t *strand, int64_t *offset) {
    DBuf ha, hb, ds, doff, err, stp;
    const int64_t *da = nullptr, *db = nullptr;
    RB3_TRY(stage_i64(c, a, n, mem, ha, &da));
    if (b) RB3_TRY(stage_i64(c, b, n, mem, hb, &db));
    // outputs go straight to the caller's arrays when they are device memory
    int64_t *os = strand, *oo = offset;
    if (mem == RB3_MEM_HOST) {
        RB3_ALLOC(ds, &c, n * sizeof(int64_t));
        RB3_ALLOC(doff, &c, n * sizeof(int64_t));
        os = ds.as<int64_t>();
        oo = doff.as<int64_t>();
    }
    RB3_ALLOC(err, &c, sizeof(int32_t));
    RB3_ALLOC(stp, &c, sizeof(unsigned long long));
    RB3_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), c.stream));
    RB3_HIP(hipMemsetAsync(stp.p, 0, sizeof(unsigned long long), c.stream));
    if (b)
        RB3_TRY(locate_one(c, d.dev(), d.smp(), da, db, n, os, oo, err.as<int32_t>(), stp.as<unsigned long long>()));
    else
        RB3_TRY(locate_rows(c, d.dev(), d.smp(), da, n, os, oo, err.as<int32_t>(), stp.as<unsigned long long>()));
    if (mem == RB3_MEM_HOST) {
        RB3_HIP(hipMemcpyAsync(strand, ds.p, n * sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
        RB3_HIP(hipMemcpyAsync(offset, doff.p, n * sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
    }
    unsigned long long steps = 0;
    RB3_HIP(hipMemcpyAsync(&steps, stp.p, sizeof(steps), hipMemcpyDeviceToHost, c.stream));
    int32_t bad = 0;
    RB3_TRY(read_flag(c, err.as<int32_t>(), &bad));
    if (bad) return fail(RB3_EINVAL, b ? "an interval is outside [0, n] or reversed" : "a row is outside [0, n)");
    g_last_locate_steps = (int64_t)steps;
    return RB3_OK;
}

int rb3_locate(const rb3_index *idx, const int64_t *rows, int64_t n, int32_t mem, int64_t *strand,
               int64_t *offset) {
    if (!idx) return fail(RB3_EINVAL, "index is NULL");
    if (idx->d.ctx.ssa <= 0) return fail(RB3_EINVAL, "the index has no suffix-array samples (ssa_rate = 0)");
    if (mem != RB3_MEM_HOST && mem != RB3_MEM_DEVICE) return fail(RB3_EINVAL, "bad mem");
    if (n < 0 || (n > 0 && (!rows || !strand || !offset))) return fail(RB3_EINVAL, "bad arguments");
    if (n == 0) return RB3_OK;
    if (mem == RB3_MEM_HOST)
        for (int64_t i = 0; i < n; ++i)
            if (rows[i] < 0 || rows[i] >= idx->d.n) return fail(RB3_EINVAL, "a row is outside [0, n)");
    RB3_HIP(hipSetDevice(idx->d.ctx.device));
    Ctx c = call_ctx(idx->d);
    int rc = run_locate(c, idx->d, rows, nullptr, n, mem, strand, offset);
    return finish(c, rc);
}

int rb3_locate1(const rb3_index *idx, const int64_t *lo, const int64_t *hi, int64_t n, int32_t mem,
                int64_t *strand, int64_t *offset) {
    if (!idx) return fail(RB3_EINVAL, "index is NULL");
    if (idx->d.ctx.ssa <= 0) return fail(RB3_EINVAL, "the index has no suffix-array samples (ssa_rate = 0)");
    if (mem != RB3_MEM_HOST && mem != RB3_MEM_DEVICE) return fail(RB3_EINVAL, "bad mem");
    if (n < 0 || (n > 0 && (!lo || !hi || !strand || !offset))) return fail(RB3_EINVAL, "bad arguments");
    if (n == 0) return RB3_OK;
    if (mem == RB3_MEM_HOST)
        for (int64_t i = 0; i < n; ++i)
            if (lo[i] < 0 || hi[i] > idx->d.n || lo[i] > hi[i])
                return fail(RB3_EINVAL, "an interval is outside [0, n] or reversed");
    RB3_HIP(hipSetDevice(idx->d.ctx.device));
    Ctx c = call_ctx(idx->d);
    int rc = run_locate(c, idx->d, lo, hi, n, mem, strand, offset);
    return finish(c, rc);
}

int rb3_ssa_info(const rb3_index *idx, int32_t *rate, int64_t *nsamples) {
    if (!idx) return fail(RB3_EINVAL, "index is NULL");
    if (rate) *rate = idx->d.ctx.ssa;
    if (nsamples) *nsamples = idx->d.nsmp;
    return RB3_OK;
}

int rb3_last_locate_stats(int64_t *lf_steps) {
    if (!lf_steps) return fail(RB3_EINVAL, "lf_steps is NULL");
    *lf_steps = g_last_locate_steps;
    return RB3_OK;
}

int rb3_info(const rb3_index *idx, int64_t *n, int64_t *m, int64_t C[6]) {
    if (!idx) return fail(RB3_EINVAL, "index is NULL");
    if (n) *n = idx->d.n;
    if (m) *m = idx->d.m;
    if (C)
        for (int i = 0; i < 6; ++i) C[i] = idx->d.C[i];
    return RB3_OK;
}

int rb3_export(const rb3_index *idx, uint8_t *codes) {
    if (!idx) return fail(RB3_EINVAL, "index is NULL");
    if (idx->d.n == 0) return RB3_OK;
    if (!codes) return fail(RB3_EINVAL, "codes is NULL");
    RB3_HIP(hipSetDevice(idx->d.ctx.device));
    Ctx c = call_ctx(idx->d);
    int rc = [&]() -> int {
        DBuf dc;
        RB3_ALLOC(dc, &c, idx->d.n);
        RB3_TRY(unpack_codes(c, idx->d.dev(), dc.as<uint8_t>()));
        RB3_HIP(hipMemcpyAsync(codes, dc.p, idx->d.n, hipMemcpyDeviceToHost, c.stream));
        return RB3_OK;
    }();
    return finish(c, rc);
}

int rb3_import(const rb3_opts *o, const uint8_t *codes, int64_t n, const int64_t *lens, int64_t m, int32_t mem,
               rb3_index **out) {
    if (!out) return fail(RB3_EINVAL, "out is NULL");
    if (n < 1 || !codes) return fail(RB3_EINVAL, "need at least one code");
    if (m < 1 || !lens) return fail(RB3_EINVAL, "need the lengths of the m >= 1 strands");
    if (mem != RB3_MEM_HOST && mem != RB3_MEM_DEVICE) return fail(RB3_EINVAL, "bad mem");
    {
        // a BWT of m strands of these lengths has n = sum (L_j + 1) symbols
        int64_t want = 0;
        for (int64_t j = 0; j < m; ++j) {
            if (lens[j] < 1) return fail(RB3_EINVAL, "a strand length is below 1");
            want += lens[j] + 1;
        }
        if (want != n) return fail(RB3_EINVAL, "symbol-count check: n differs from the sum of strand lengths + m");
    }
    if (o && o->ssa_rate != 0)
        return fail(RB3_EINVAL, "suffix-array samples need the strings: build the index with rb3_build");
    rb3_index *ix = new (std::nothrow) rb3_index();
    if (!ix) return fail(RB3_ENOMEM, "host allocation failed");
    int rc = ctx_from_opts(o, ix->d.ctx);
    if (rc != RB3_OK) {
        delete ix;
        return rc;
    }
    Ctx c = call_ctx(ix->d);
    rc = [&]() -> int {
        DBuf hold, err, blk, sb;
        const uint8_t *d_codes = nullptr;
        RB3_TRY(stage(c, codes, n, mem, hold, &d_codes));
        RB3_ALLOC(err, &c, sizeof(int32_t));
        RB3_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), c.stream));
        RB3_TRY(check_codes(c, d_codes, n, err.as<int32_t>()));
        int32_t bad = 0;
        RB3_TRY(read_flag(c, err.as<int32_t>(), &bad));
        if (bad) return fail(RB3_EINVAL, "code outside 0..5");
        RB3_ALLOC(blk, &c, num_blocks(n) * 64);
        RB3_ALLOC(sb, &c, num_superblocks(n) * SB_STRIDE * sizeof(int64_t));
        RB3_TRY(pack_codes(c, d_codes, n, blk.as<uint4>()));
        int64_t C[6], cnt[6];
        RB3_TRY(build_checkpoints(c, blk.as<uint4>(), n, sb.as<int64_t>(), C, cnt));
        if (cnt[0] != m) return fail(RB3_EINVAL, "symbol-count check: the codes hold a number of sentinels ($) other than m");
        ix->d.n = n;
        ix->d.m = cnt[0];
        for (int i = 0; i < 6; ++i) ix->d.C[i] = C[i];
        ix->d.blk = (uint4 *)blk.release();
        ix->d.sb = (int64_t *)sb.release();
        return RB3_OK;
    }();
    rc = finish(c, rc);
    if (rc != RB3_OK) {
        rb3_index_free(ix);
        return rc;
    }
    *out = ix;
    return RB3_OK;
}

int rb3_clone(const rb3_index *src, rb3_index **out) {
    if (!src || !out) return fail(RB3_EINVAL, "NULL argument");
    RB3_HIP(hipSetDevice(src->d.ctx.device));
    rb3_index *ix = new (std::nothrow) rb3_index();
    if (!ix) return fail(RB3_ENOMEM, "host allocation failed");
    ix->d.ctx = call_ctx(src->d);
    ix->d.ctx.own_stream = false;
    if (src->d.ctx.own_stream) {
        // the source's stream dies with the source: the copy gets its own
        hipStream_t s2 = nullptr;
        if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess) {
            delete ix;
            return fail(RB3_EDEVICE, "hipStreamCreateWithFlags failed");
        }
        // the copy below runs on the source's stream; the new stream starts after it
        ix->d.ctx.stream = s2;
        ix->d.ctx.own_stream = true;
    }
    Ctx c = call_ctx(src->d);
    int rc = [&]() -> int {
        DBuf blk, sb;
        size_t bb = num_blocks(src->d.n) * 64, sbb = num_superblocks(src->d.n) * SB_STRIDE * sizeof(int64_t);
        RB3_ALLOC(blk, &c, bb);
        RB3_ALLOC(sb, &c, sbb);
        RB3_HIP(hipMemcpyAsync(blk.p, src->d.blk, bb, hipMemcpyDeviceToDevice, c.stream));
        RB3_HIP(hipMemcpyAsync(sb.p, src->d.sb, sbb, hipMemcpyDeviceToDevice, c.stream));
        if (src->d.ctx.ssa > 0) {
            DBuf srec, sval;
            const int64_t nb = num_blocks(src->d.n);
            RB3_ALLOC(srec, &c, nb * SMP_REC * sizeof(uint64_t));
            RB3_HIP(hipMemcpyAsync(srec.p, src->d.smp_rec, nb * SMP_REC * sizeof(uint64_t), hipMemcpyDeviceToDevice,
                                   c.stream));
            if (src->d.nsmp > 0) {
                RB3_ALLOC(sval, &c, src->d.nsmp * sizeof(uint64_t));
                RB3_HIP(hipMemcpyAsync(sval.p, src->d.smp_val, src->d.nsmp * sizeof(uint64_t),
                                       hipMemcpyDeviceToDevice, c.stream));
            }
            ix->d.smp_rec = (uint64_t *)srec.release();
            ix->d.smp_val = src->d.nsmp > 0 ? (uint64_t *)sval.release() : nullptr;
            ix->d.nsmp = src->d.nsmp;
        }
        ix->d.n = src->d.n;
        ix->d.m = src->d.m;
        for (int i = 0; i < 6; ++i) ix->d.C[i] = src->d.C[i];
        ix->d.blk = (uint4 *)blk.release();
        ix->d.sb = (int64_t *)sb.release();
        return RB3_OK;
    }();
    rc = finish(c, rc);
    if (rc != RB3_OK) {
        rb3_index_free(ix);
        return rc;
    }
    *out = ix;
    return RB3_OK;
}

void rb3_index_free(rb3_index *idx) {
    if (!idx) return;
    (void)hipSetDevice(idx->d.ctx.device);
    if (idx->d.ctx.stream) (void)hipStreamSynchronize(idx->d.ctx.stream);
    Ctx c = call_ctx(idx->d);
    c.free_now(idx->d.blk);
    c.free_now(idx->d.sb);
    c.free_now(idx->d.smp_rec);
    c.free_now(idx->d.smp_val);
    if (idx->d.ctx.own_stream && idx->d.ctx.stream) (void)hipStreamDestroy(idx->d.ctx.stream);
    delete idx;
}

// The autotuner's trials: candidates timed on clones (merge) or on the
// index itself (SMEM, read-only), inputs staged on the device once.
int rb3_tune_merge(rb3_index *idx, const uint8_t *seq, const int64_t *lens, int64_t n_seqs, int32_t mem,
                   int64_t *chunk_len, int64_t *cand, double *ms, int64_t cap, int64_t *n_out) {
    if (!idx || !chunk_len) return fail(RB3_EINVAL, "NULL argument");
    if (idx->d.n == 0) return fail(RB3_EINVAL, "tuning needs a non-empty index (a build has no chains)");
    if (cap < 0 || (cap > 0 && (!cand || !ms))) return fail(RB3_EINVAL, "bad output arrays");
    int64_t total = 0;
    RB3_TRY(check_strings(seq, lens, n_seqs, mem, false, &total));
    if (n_seqs == 0) return fail(RB3_EINVAL, "no strings to tune on");
    RB3_HIP(hipSetDevice(idx->d.ctx.device));
    const int k = idx->d.ctx.both ? 2 : 1;
    const int64_t m2 = k * n_seqs, n2 = k * (total + n_seqs);
    Ctx c = call_ctx(idx->d);
    const int64_t cands[] = {1024, 2048, 4096, 8192};
    std::vector<std::pair<int64_t, double>> res;
    int rc = [&]() -> int {
        DBuf hold;
        const uint8_t *d_seq = nullptr;
        RB3_TRY(stage(c, seq, total, mem, hold, &d_seq));
        RB3_TRY(c.flush());
        for (int trial = -1; trial < (int)(sizeof(cands) / sizeof(cands[0])); ++trial) {
            const int64_t CL = cands[trial < 0 ? 1 : trial];
            if (n2 / CL > ((int64_t)1 << 21)) continue;  // more chunks than lanes in flight
            rb3_index *cl = nullptr;
            RB3_TRY(rb3_clone(idx, &cl));
            cl->d.ctx.chunk_len = CL;
            Ctx cc = call_ctx(cl->d);
            RB3_HIP(hipStreamSynchronize(cc.stream));
            const auto t0 = std::chrono::steady_clock::now();
            int r = do_merge(cc, cl->d, d_seq, lens, n_seqs, RB3_MEM_DEVICE);
            r = finish(cc, r);
            const auto t1 = std::chrono::steady_clock::now();
            rb3_index_free(cl);
            RB3_TRY(r);
            if (trial >= 0) res.push_back({CL, std::chrono::duration<double, std::milli>(t1 - t0).count()});
        }
        return RB3_OK;
    }();
    rc = finish(c, rc);
    if (rc != RB3_OK) return rc;
    if (res.empty()) return fail(RB3_EINVAL, "batch too large for every candidate chunk length");
    size_t best = 0;
    for (size_t j = 0; j < res.size(); ++j)
        if (res[j].second < res[best].second) best = j;
    *chunk_len = res[best].first;
    tune_store(merge_tune_key(idx->d.ctx.device, idx->d.n, n2, m2), res[best].first);
    for (int64_t j = 0; j < (int64_t)res.size() && j < cap; ++j) {
        cand[j] = res[j].first;
        ms[j] = res[j].second;
    }
    if (n_out) *n_out = (int64_t)res.size();
    return RB3_OK;
}

int rb3_tune_smem(const rb3_index *idx, const uint8_t *q, const int64_t *qlens, int64_t n_q, int32_t mem,
                  int32_t min_len, int64_t min_occ, int64_t *segment, int64_t *cand, double *ms, int64_t cap,
                  int64_t *n_out) {
    if (!idx || !segment) return fail(RB3_EINVAL, "NULL argument");
    if (min_len < 1 || min_occ < 1) return fail(RB3_EINVAL, "min_len and min_occ must be >= 1");
    if (!idx->d.ctx.both) return fail(RB3_EINVAL, "SMEM finding needs an index of both strands");
    if (cap < 0 || (cap > 0 && (!cand || !ms))) return fail(RB3_EINVAL, "bad output arrays");
    int64_t total = 0;
    RB3_TRY(check_strings(q, qlens, n_q, mem, true, &total));
    if (n_q == 0 || total == 0) return fail(RB3_EINVAL, "no queries to tune on");
    RB3_HIP(hipSetDevice(idx->d.ctx.device));
    // -1: the automatic rule (from the batch size)
    const int64_t cands[] = {-1, 64, 128, 256, 512, 1024, 2048, 4096};
    std::vector<std::pair<int64_t, double>> res;
    Ctx c = call_ctx(idx->d);
    int rc = [&]() -> int {
        DBuf hold;
        const uint8_t *d_q = nullptr;
        RB3_TRY(stage(c, q, total, mem, hold, &d_q));
        RB3_TRY(c.flush());
        int64_t ocap = total / 16 + 16 * n_q + 16;
        std::vector<rb3_smem_t> out;
        std::vector<int64_t> off(n_q + 1);
        for (int64_t sg : cands) {
            double best_ms = 1e300;
            for (int rep = 0; rep < 2; ++rep) {
                Ctx cc = call_ctx(idx->d);
                cc.smem_seg_fixed = sg;
                out.resize(ocap);
                int64_t exts[2] = {0, 0};
                const auto t0 = std::chrono::steady_clock::now();
                int r = run_smem(cc, idx->d.dev(), d_q, qlens, n_q, total, RB3_MEM_DEVICE, min_len, min_occ,
                                 out.data(), ocap, off.data(), exts);
                r = finish(cc, r);
                const auto t1 = std::chrono::steady_clock::now();
                if (r == RB3_ENOSPC) {
                    ocap = off[n_q];
                    --rep;
                    continue;
                }
                RB3_TRY(r);
                const double t = std::chrono::duration<double, std::milli>(t1 - t0).count();
                if (t < best_ms) best_ms = t;
            }
            res.push_back({sg, best_ms});
        }
        return RB3_OK;
    }();
    rc = finish(c, rc);
    if (rc != RB3_OK) return rc;
    size_t best = 0;
    for (size_t j = 0; j < res.size(); ++j)
        if (res[j].second < res[best].second) best = j;
    *segment = res[best].first;
    tune_store(smem_tune_key(idx->d.ctx.device, idx->d.n, total, n_q), res[best].first);
    for (int64_t j = 0; j < (int64_t)res.size() && j < cap; ++j) {
        cand[j] = res[j].first;
        ms[j] = res[j].second;
    }
    if (n_out) *n_out = (int64_t)res.size();
    return RB3_OK;
}

int rb3_test_fail_merge_after(int32_t stage) {
    if (stage < 0 || stage > 5) return fail(RB3_EINVAL, "stage must be 0 .. 5");
    g_fail_after.store(stage);
    return RB3_OK;
}

int rb3_prof_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return RB3_OK;
}

int rb3_prof_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_drain_locked();
    g_prof_agg.clear();
    return RB3_OK;
}

int rb3_prof_read(char *names, int64_t *launches, double *ms, int64_t cap, int64_t *n_out) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_drain_locked();
    int64_t i = 0;
    for (auto &kv : g_prof_agg) {
        if (i < cap) {
            if (names) {
                std::memset(names + i * 32, 0, 32);
                std::strncpy(names + i * 32, kv.first.c_str(), 31);
            }
            if (launches) launches[i] = kv.second.launches;
            if (ms) ms[i] = kv.second.ms;
        }
        ++i;
    }
    if (n_out) *n_out = i;
    return RB3_OK;
}

int rb3_merge_stats(const rb3_index *idx, char *keys, int64_t *vals, int64_t cap, int64_t *n_out) {
    if (!idx) return fail(RB3_EINVAL, "index is NULL");
    const MergeStats &s = idx->d.last;
    std::vector<std::pair<const char *, int64_t>> kv = {
        {"n1", s.n1}, {"m1", s.m1}, {"n2", s.n2}, {"m2", s.m2},
        {"chunks", s.chunks}, {"chunk_len", s.chunk_len}, {"chain_steps", s.chain_steps},
        {"fixup_steps", s.fixup_steps}, {"fixup_index_steps", s.fixup_index_steps}, {"fixup_segments", s.fixup_segments}, {"fixup_passes", s.fixup_passes}, {"fixup_run_max", s.fixup_run_max}, {"key_syms", s.key_syms},
        {"sort_bits", s.sort_bits}, {"sort_packed", s.sort_packed}, {"sort_passes", s.sort_passes}, {"tied_records", s.tied_records}, {"tie_groups", s.tie_groups}, {"tie_pairs", s.tie_pairs}, {"tie_small_reads", s.tie_small_reads}, {"tie_max_depth", s.tie_max_depth}, {"tie_deep_reads", s.tie_deep_reads},
        {"max_group", s.max_group}, {"tie_doubling", s.tie_doubling}, {"tie_rounds", s.tie_rounds},
        {"tie_work", s.tie_work}, {"tie_block_reads", s.tie_block_reads}};
    static const char *hist_names[32] = {
        "groups_log2_0", "groups_log2_1", "groups_log2_2", "groups_log2_3", "groups_log2_4",
        "groups_log2_5", "groups_log2_6", "groups_log2_7", "groups_log2_8", "groups_log2_9",
        "groups_log2_10", "groups_log2_11", "groups_log2_12", "groups_log2_13", "groups_log2_14",
        "groups_log2_15", "groups_log2_16", "groups_log2_17", "groups_log2_18", "groups_log2_19",
        "groups_log2_20", "groups_log2_21", "groups_log2_22", "groups_log2_23", "groups_log2_24",
        "groups_log2_25", "groups_log2_26", "groups_log2_27", "groups_log2_28", "groups_log2_29",
        "groups_log2_30", "groups_log2_31"};
    for (int b = 1; b < 32; ++b)
        if (s.group_hist[b]) kv.push_back({hist_names[b], (int64_t)s.group_hist[b]});
    int64_t i = 0;
    for (auto &p : kv) {
        if (i < cap) {
            if (keys) {
                std::memset(keys + i * 32, 0, 32);
                std::strncpy(keys + i * 32, p.first, 31);
            }
            if (vals) vals[i] = p.second;
        }
        ++i;
    }
    if (n_out) *n_out = i;
    return RB3_OK;
}

// ---------------------------------------------------------------------------
// run-length static index
// ---------------------------------------------------------------------------

static Ctx rle_ctx(const rb3_rle *r) {
    Ctx c;
    c.device = r->ctx.device;
    c.stream = r->ctx.stream;
    c.own_stream = false;
    c.alloc = r->ctx.alloc;
    c.free_fn = r->ctx.free_fn;
    c.alloc_ctx = r->ctx.alloc_ctx;
    c.both = r->both;
    c.smem_seg_fixed = r->ctx.smem_seg_fixed;
    return c;
}

static void rle_totals(rb3_rle *r, const int64_t tot[6]) {
    r->m = tot[0];
    int64_t acc = 0;
    for (int i = 0; i < 6; ++i) {
        r->C[i] = acc;
        acc += tot[i];
    }
}

void rb3_rle_free(rb3_rle *r) {
    if (!r) return;
    (void)hipSetDevice(r->ctx.device);
    if (r->ctx.stream) (void)hipStreamSynchronize(r->ctx.stream);
    Ctx c = rle_ctx(r);
    c.free_now(r->blk);
    c.free_now(r->seg);
    c.free_now(r->row);
    if (r->ctx.own_stream && r->ctx.stream) (void)hipStreamDestroy(r->ctx.stream);
    delete r;
}

static int rle_new(int device, const Ctx &like, rb3_rle **out) {
    rb3_rle *r = new (std::nothrow) rb3_rle();
    if (!r) return fail(RB3_ENOMEM, "host allocation failed");
    r->ctx.device = device;
    r->ctx.alloc = like.alloc;
    r->ctx.free_fn = like.free_fn;
    r->ctx.alloc_ctx = like.alloc_ctx;
    r->ctx.smem_seg_fixed = like.smem_seg_fixed;
    if (hipStreamCreateWithFlags(&r->ctx.stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete r;
        return fail(RB3_EDEVICE, "stream creation failed");
    }
    r->ctx.own_stream = true;
    *out = r;
    return RB3_OK;
}

int rb3_rle_build(const rb3_index *idx, int32_t row_shift, rb3_rle **out) {
    if (!idx || !out) return fail(RB3_EINVAL, "index or out is NULL");
    if (idx->d.n == 0) return fail(RB3_EINVAL, "run-length index of an empty BWT");
    RB3_HIP(hipSetDevice(idx->d.ctx.device));
    rb3_rle *r = nullptr;
    RB3_TRY(rle_new(idx->d.ctx.device, idx->d.ctx, &r));
    r->both = idx->d.ctx.both;
    // the build runs on the index's stream (it reads the index)
    Ctx c = call_ctx(idx->d);
    int rc = [&]() -> int {
        RleBuild b;
        RB3_TRY(rle_build(c, idx->d.dev(), row_shift, b));
        r->n = b.n;
        r->nseg = b.nseg;
        r->nblk = b.nblk;
        r->npieces = b.npieces;
        r->q = b.q;
        rle_totals(r, b.tot);
        r->blk = (uint64_t *)b.blk.release();
        r->seg = (int64_t *)b.seg.release();
        r->row = (uint16_t *)b.row.release();
        return RB3_OK;
    }();
    rc = finish(c, rc);
    if (rc != RB3_OK) {
        rb3_rle_free(r);
        return rc;
    }
    *out = r;
    return RB3_OK;
}

int rb3_rle_load(const rb3_opts *o, const uint64_t *blocks, int64_t nblocks, const int64_t *segs,
                 const uint16_t *row, int64_t n, int32_t row_shift, int32_t both, rb3_rle **out) {
    if (!out || !blocks || !segs || !row) return fail(RB3_EINVAL, "NULL argument");
    if (n <= 0 || nblocks <= 0) return fail(RB3_EINVAL, "empty run-length index");
    if (row_shift < 4 || row_shift > 20) return fail(RB3_EINVAL, "row shift must be in 4 .. 20");
    const int64_t nseg = (n + RLE_SEG - 1) >> RLE_SEG_SHIFT;
    // the segment table on the host: zero counts first, every segment's
    // counts adding up to its length, first blocks increasing to nblocks
    for (int k = 0; k < 7; ++k)
        if (segs[k] != 0) return fail(RB3_EINVAL, "run-length index: first table row is not zero");
    for (int64_t s = 0; s < nseg; ++s) {
        const int64_t len = (s + 1) * RLE_SEG < n ? RLE_SEG : n - s * RLE_SEG;
        int64_t sum = 0;
        for (int k = 0; k < 6; ++k) {
            const int64_t d = segs[(s + 1) * 8 + k] - segs[s * 8 + k];
            if (d < 0) return fail(RB3_EINVAL, "run-length index: decreasing counts");
            sum += d;
        }
        const int64_t nb = segs[(s + 1) * 8 + 6] - segs[s * 8 + 6];
        if (sum != len || nb < 1 || nb >= 65536)
            return fail(RB3_EINVAL, "run-length index: a segment's counts or blocks are out of range");
    }
    if (segs[nseg * 8 + 6] != nblocks) return fail(RB3_EINVAL, "run-length index: block count mismatch");
    rb3_opts d;
    rb3_opts_init(&d);
    if (!o) o = &d;
    Ctx like;
    RB3_TRY(ctx_from_opts(o, like));
    if (like.own_stream && like.stream) (void)hipStreamDestroy(like.stream);
    rb3_rle *r = nullptr;
    RB3_TRY(rle_new(o->device, like, &r));
    r->both = both ? 1 : 0;
    r->n = n;
    r->nseg = nseg;
    r->nblk = nblocks;
    r->q = row_shift;
    rle_totals(r, segs + nseg * 8);
    Ctx c = rle_ctx(r);
    int rc = [&]() -> int {
        const int64_t nrow = ((n - 1) >> row_shift) + 1;
        DBuf bb, sb, rb, bad;
        RB3_ALLOC(bb, &c, nblocks * RLE_WORDS * sizeof(uint64_t));
        RB3_ALLOC(sb, &c, (nseg + 1) * 8 * sizeof(int64_t));
        RB3_ALLOC(rb, &c, nrow * sizeof(uint16_t));
        RB3_ALLOC(bad, &c, sizeof(int32_t));
        RB3_HIP(hipMemcpyAsync(bb.p, blocks, nblocks * RLE_WORDS * sizeof(uint64_t), hipMemcpyHostToDevice,
                               c.stream));
        RB3_HIP(hipMemcpyAsync(sb.p, segs, (nseg + 1) * 8 * sizeof(int64_t), hipMemcpyHostToDevice, c.stream));
        RB3_HIP(hipMemcpyAsync(rb.p, row, nrow * sizeof(uint16_t), hipMemcpyHostToDevice, c.stream));
        RB3_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), c.stream));
        r->blk = (uint64_t *)bb.release();
        r->seg = (int64_t *)sb.release();
        r->row = (uint16_t *)rb.release();
        RB3_TRY(rle_check(c, r->view(), bad.as<int32_t>()));
        int32_t hbad = 0;
        RB3_TRY(read_flag(c, bad.as<int32_t>(), &hbad));
        if (hbad) return fail(RB3_EINVAL, "run-length index: blocks or index row fail the format checks");
        return RB3_OK;
    }();
    rc = finish(c, rc);
    if (rc != RB3_OK) {
        rb3_rle_free(r);
        return rc;
    }
    *out = r;
    return RB3_OK;
}

int rb3_rle_info(const rb3_rle *r, int64_t *n, int64_t *m, int64_t *runs, int64_t *blocks, int32_t *row_shift,
                 int64_t *bytes) {
    if (!r) return fail(RB3_EINVAL, "run-length index is NULL");
    if (n) *n = r->n;
    if (m) *m = r->m;
    if (runs) *runs = r->npieces;
    if (blocks) *blocks = r->nblk;
    if (row_shift) *row_shift = r->q;
    if (bytes)
        *bytes = r->nblk * RLE_WORDS * 8 + (r->nseg + 1) * 8 * 8 + ((((r->n - 1) >> r->q) + 1) * 2);
    return RB3_OK;
}

int rb3_rle_image(const rb3_rle *r, uint64_t *blocks, int64_t *segs, uint16_t *row) {
    if (!r || !blocks || !segs || !row) return fail(RB3_EINVAL, "NULL argument");
    RB3_HIP(hipSetDevice(r->ctx.device));
    Ctx c = rle_ctx(r);
    int rc = [&]() -> int {
        RB3_HIP(hipMemcpyAsync(blocks, r->blk, r->nblk * RLE_WORDS * sizeof(uint64_t), hipMemcpyDeviceToHost,
                               c.stream));
        RB3_HIP(hipMemcpyAsync(segs, r->seg, (r->nseg + 1) * 8 * sizeof(int64_t), hipMemcpyDeviceToHost,
                               c.stream));
        RB3_HIP(hipMemcpyAsync(row, r->row, ((((r->n - 1) >> r->q) + 1) * sizeof(uint16_t)), hipMemcpyDeviceToHost,
                               c.stream));
        return RB3_OK;
    }();
    return finish(c, rc);
}

int rb3_rle_export(const rb3_rle *r, uint8_t *codes) {
    if (!r || !codes) return fail(RB3_EINVAL, "NULL argument");
    RB3_HIP(hipSetDevice(r->ctx.device));
    Ctx c = rle_ctx(r);
    int rc = [&]() -> int {
        DBuf dc;
        RB3_ALLOC(dc, &c, r->n);
        RB3_TRY(rle_decode_all(c, r->view(), dc.as<uint8_t>()));
        RB3_HIP(hipMemcpyAsync(codes, dc.p, r->n, hipMemcpyDeviceToHost, c.stream));
        return RB3_OK;
    }();
    return finish(c, rc);
}

int rb3_rle_count(const rb3_rle *r, const uint8_t *q, const int64_t *qlens, int64_t n_q, int32_t mem, int64_t *lo,
                  int64_t *hi) {
    if (!r) return fail(RB3_EINVAL, "run-length index is NULL");
    if (n_q > 0 && (!lo || !hi)) return fail(RB3_EINVAL, "output arrays are NULL");
    int64_t total = 0;
    RB3_TRY(check_strings(q, qlens, n_q, mem, true, &total));
    if (n_q == 0) return RB3_OK;
    RB3_HIP(hipSetDevice(r->ctx.device));
    Ctx c = rle_ctx(r);
    const RleView v = r->view();
    int rc = run_count(c, DevIndex{}, q, qlens, n_q, total, mem, lo, hi, &v);
    return finish(c, rc);
}

int rb3_rle_smem(const rb3_rle *r, const uint8_t *q, const int64_t *qlens, int64_t n_q, int32_t mem,
                 int32_t min_len, int64_t min_occ, rb3_smem_t *out, int64_t out_cap, int64_t *out_off) {
    if (!r) return fail(RB3_EINVAL, "run-length index is NULL");
    if (!out_off) return fail(RB3_EINVAL, "out_off is NULL");
    if (min_len < 1 || min_occ < 1) return fail(RB3_EINVAL, "min_len and min_occ must be >= 1");
    if (out_cap < 0 || (out_cap > 0 && !out)) return fail(RB3_EINVAL, "bad output buffer");
    if (!r->both) return fail(RB3_EINVAL, "SMEM finding needs an index of both strands");
    if (n_q >= (int64_t)INT32_MAX) return fail(RB3_ELIMIT, "too many queries");
    int64_t total = 0;
    RB3_TRY(check_strings(q, qlens, n_q, mem, true, &total));
    out_off[0] = 0;
    if (n_q == 0) return RB3_OK;
    RB3_HIP(hipSetDevice(r->ctx.device));
    Ctx c = rle_ctx(r);
    const RleView v = r->view();
    int64_t exts[2] = {0, 0};
    int rc = run_smem(c, DevIndex{}, q, qlens, n_q, total, mem, min_len, min_occ, out, out_cap, out_off, exts, &v);
    if (rc == RB3_OK) {
        g_last_smem_exts[0] = exts[0];
        g_last_smem_exts[1] = exts[1];
    }
    return finish(c, rc);
}

int rb3_rle_hapl(const rb3_rle *r, const rb3_hapl_opts *o, const uint8_t *q, const int64_t *qlens, int64_t n_q,
                 int32_t mem, rb3_hapl_t *out, int64_t out_cap, int64_t *out_off) {
    if (!r) return fail(RB3_EINVAL, "run-length index is NULL");
    rb3_hapl_opts oo;
    int64_t total = 0;
    RB3_TRY(hapl_args(o, q, qlens, n_q, mem, out, out_cap, out_off, r->both, r->n, &oo, &total));
    if (n_q == 0) return RB3_OK;
    RB3_HIP(hipSetDevice(r->ctx.device));
    Ctx c = rle_ctx(r);
    const RleView v = r->view();
    int rc = run_hapl(c, DevIndex{}, q, qlens, n_q, total, mem, oo, out, out_cap, out_off, &v);
    return finish(c, rc);
}

}  // extern "C"
