// Continuous-batching query server over one index.
//
// Worker threads, each with its own HIP stream and its own caching device
// allocator, take every pending request up to a batch limit whenever they
// are free, so requests that arrive while other batches run on the GPU are
// admitted as soon as a worker (a stream slot) and the device-memory budget
// allow, and batches on different streams overlap on the device. A batch is
// split into its count requests and its SMEM requests (grouped by their
// min_len / min_occ) and each part goes through the same pipeline as
// rb3_count / rb3_smem.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "rb3_internal.h"

namespace rb3 {

// Device memory pool of one worker: blocks are kept per rounded size and
// reused, so steady-state batches allocate nothing from HIP.
struct Pool {
    int device = 0;
    std::multimap<size_t, void *> free_blocks;
    std::map<void *, size_t> size_of;
    static size_t round(size_t b) {
        size_t r = 256;
        while (r < b) r <<= 1;
        return r;
    }
    void *alloc(size_t bytes) {
        size_t r = round(bytes);
        auto it = free_blocks.find(r);
        if (it != free_blocks.end()) {
            void *p = it->second;
            free_blocks.erase(it);
            return p;
        }
        void *p = nullptr;
        if (hipMalloc(&p, r) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        size_of[p] = r;
        return p;
    }
    void release(void *p) {
        auto it = size_of.find(p);
        if (it != size_of.end()) free_blocks.emplace(it->second, p);
    }
    ~Pool() {
        for (auto &kv : size_of) (void)hipFree(kv.first);
    }
};

static void *pool_alloc(size_t bytes, void *ctx) { return ((Pool *)ctx)->alloc(bytes); }
static void pool_free(void *p, void *ctx) { ((Pool *)ctx)->release(p); }

struct Request {
    uint64_t ticket;
    int32_t kind;
    int32_t min_len;
    int64_t min_occ;
    std::vector<uint8_t> q;
};

struct Done {
    rb3_result r;
    std::vector<rb3_smem_t> recs;
};

}  // namespace rb3

using namespace rb3;

struct rb3_server {
    const rb3_index *idx = nullptr;
    rb3_server_opts so;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> pending;
    std::deque<Done> done;
    std::vector<std::thread> workers;
    bool stop = false;
    uint64_t next_ticket = 1;
    int64_t inflight_bytes = 0;
    int64_t inflight_batches = 0;
    int64_t batches = 0, served = 0, max_batch = 0;
    int64_t busy_us = 0;  // summed over workers: time spent running batches
};

namespace {

int64_t footprint(const Request &r) {
    // device bytes a request needs while in flight: codes, staging, per-base
    // worst-case SMEM records, segment tables
    int64_t L = (int64_t)r.q.size();
    return L * 2 + (r.kind == RB3_REQ_SMEM ? (L / 8 + 64) * (int64_t)sizeof(rb3_smem_t) * 2 : 64) + 4096;
}

bool valid_bytes(const uint8_t *q, int64_t len) {
    for (int64_t i = 0; i < len; ++i) {
        switch (q[i] | 0x20) {
        case 'a': case 'c': case 'g': case 't': case 'n': break;
        default: return false;
        }
    }
    return true;
}

void run_batch(rb3_server *s, Ctx &c, std::vector<Request> &batch) {
    const DevIndex ix = index_dev(s->idx);
    std::vector<Done> out(batch.size());
    for (size_t i = 0; i < batch.size(); ++i) {
        std::memset(&out[i].r, 0, sizeof(rb3_result));
        out[i].r.ticket = batch[i].ticket;
        out[i].r.kind = batch[i].kind;
    }
    // count requests together
    {
        std::vector<size_t> which;
        std::vector<uint8_t> buf;
        std::vector<int64_t> lens;
        for (size_t i = 0; i < batch.size(); ++i)
            if (batch[i].kind == RB3_REQ_COUNT) {
                which.push_back(i);
                buf.insert(buf.end(), batch[i].q.begin(), batch[i].q.end());
                lens.push_back((int64_t)batch[i].q.size());
            }
        if (!which.empty()) {
            std::vector<int64_t> lo(which.size()), hi(which.size());
            int rc = run_count(c, ix, buf.data(), lens.data(), (int64_t)which.size(), (int64_t)buf.size(),
                               RB3_MEM_HOST, lo.data(), hi.data());
            rc = rc != RB3_OK ? rc : c.flush();
            for (size_t k = 0; k < which.size(); ++k) {
                rb3_result &r = out[which[k]].r;
                r.status = rc;
                r.lo = rc == RB3_OK ? lo[k] : 0;
                r.hi = rc == RB3_OK ? hi[k] : 0;
            }
        }
    }
    // SMEM requests, grouped by parameters
    std::map<std::pair<int32_t, int64_t>, std::vector<size_t>> groups;
    for (size_t i = 0; i < batch.size(); ++i)
        if (batch[i].kind == RB3_REQ_SMEM) groups[{batch[i].min_len, batch[i].min_occ}].push_back(i);
    for (auto &g : groups) {
        std::vector<uint8_t> buf;
        std::vector<int64_t> lens;
        for (size_t i : g.second) {
            buf.insert(buf.end(), batch[i].q.begin(), batch[i].q.end());
            lens.push_back((int64_t)batch[i].q.size());
        }
        int64_t nq = (int64_t)g.second.size();
        int64_t cap = (int64_t)buf.size() / 16 + 16 * nq + 16;
        std::vector<rb3_smem_t> recs;
        std::vector<int64_t> off(nq + 1);
        int rc = RB3_OK;
        for (int attempt = 0; attempt < 2; ++attempt) {
            recs.resize(cap);
            int64_t exts[2] = {0, 0};
            rc = run_smem(c, ix, buf.data(), lens.data(), nq, (int64_t)buf.size(), RB3_MEM_HOST, g.first.first,
                          g.first.second, recs.data(), cap, off.data(), exts);
            int r2 = c.flush();
            if (rc == RB3_OK) rc = r2;
            if (rc != RB3_ENOSPC) break;
            cap = off[nq];
        }
        for (int64_t k = 0; k < nq; ++k) {
            Done &d = out[g.second[k]];
            d.r.status = rc;
            if (rc == RB3_OK) {
                d.recs.assign(recs.begin() + off[k], recs.begin() + off[k + 1]);
                for (auto &x : d.recs) x.qid = 0;
                d.r.n_smem = off[k + 1] - off[k];
            }
        }
    }
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto &d : out) s->done.push_back(std::move(d));
    s->served += (int64_t)batch.size();
    s->cv_done.notify_all();
}

void worker_main(rb3_server *s) {
    (void)hipSetDevice(index_device(s->idx));
    Pool pool;
    Ctx c;
    c.device = index_device(s->idx);
    c.alloc = pool_alloc;
    c.free_fn = pool_free;
    c.alloc_ctx = &pool;
    c.both = index_both(s->idx);
    if (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess) return;
    for (;;) {
        std::vector<Request> batch;
        int64_t bytes = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] {
                if (s->stop) return true;
                if (s->pending.empty()) return false;
                // admit when the first request fits the memory budget, or when
                // nothing else is in flight (a request larger than the budget
                // runs alone rather than waiting forever)
                return s->inflight_bytes + footprint(s->pending.front()) <= s->so.mem_budget ||
                       s->inflight_batches == 0;
            });
            if (s->stop) break;
            int64_t bases = 0;
            while (!s->pending.empty() && (int64_t)batch.size() < s->so.max_batch_queries) {
                const Request &r = s->pending.front();
                int64_t f = footprint(r);
                bool first = batch.empty();
                if (!first && (bases + (int64_t)r.q.size() > s->so.max_batch_bases ||
                               s->inflight_bytes + bytes + f > s->so.mem_budget))
                    break;
                bases += (int64_t)r.q.size();
                bytes += f;
                batch.push_back(std::move(s->pending.front()));
                s->pending.pop_front();
            }
            s->inflight_bytes += bytes;
            s->inflight_batches += 1;
            // batches running together share the GPU's lanes: each aims at
            // its share of the SMEM segments that fill the chip. A batch
            // alone on the GPU may cut its queries into the shortest
            // segments (lowest latency); when several run, segments keep at
            // least SMEM_SEG_BUSY positions, since each repeats some work at
            // its start and the server's throughput matters more then
            c.smem_segs = SMEM_TARGET_SEGS / s->inflight_batches;
            c.smem_seg_min = s->inflight_batches > 1 ? SMEM_SEG_BUSY : SMEM_SEG_MIN;
            s->batches += 1;
            if ((int64_t)batch.size() > s->max_batch) s->max_batch = (int64_t)batch.size();
        }
        const auto t0 = std::chrono::steady_clock::now();
        run_batch(s, c, batch);
        const auto us = std::chrono::duration_cast<std::chrono::microseconds>(std::chrono::steady_clock::now() - t0);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->inflight_bytes -= bytes;
            s->inflight_batches -= 1;
            s->busy_us += (int64_t)us.count();
        }
        s->cv_work.notify_all();
    }
    (void)c.flush();
    (void)hipStreamDestroy(c.stream);
}

}  // namespace

extern "C" {

void rb3_server_opts_init(rb3_server_opts *so) {
    if (!so) return;
    std::memset(so, 0, sizeof(*so));
    so->workers = 4;
    so->max_batch_queries = 4096;
    so->max_batch_bases = 8 << 20;
    so->mem_budget = 0;  // from the device's free memory at creation
    so->max_queued = 1 << 16;
}

int rb3_server_create(const rb3_index *idx, const rb3_server_opts *so, rb3_server **out) {
    if (!idx || !out) {
        set_error(RB3_EINVAL, "NULL argument");
        return RB3_EINVAL;
    }
    rb3_server_opts d;
    rb3_server_opts_init(&d);
    if (!so) so = &d;
    if (so->workers < 1 || so->workers > 64 || so->max_batch_queries < 1 || so->max_batch_bases < 1 ||
        so->mem_budget < 0 || so->max_queued < 1) {
        set_error(RB3_EINVAL, "bad server options");
        return RB3_EINVAL;
    }
    rb3_server_opts eff = *so;
    if (eff.mem_budget == 0) {
        // half of the device memory free now: the index and other users keep the rest
        size_t fr = 0, tot = 0;
        RB3_HIP(hipSetDevice(index_device(idx)));
        RB3_HIP(hipMemGetInfo(&fr, &tot));
        eff.mem_budget = (int64_t)(fr / 2);
        if (eff.mem_budget < ((int64_t)1 << 26)) eff.mem_budget = (int64_t)1 << 26;
    }
    rb3_server *s = new (std::nothrow) rb3_server();
    if (!s) {
        set_error(RB3_ENOMEM, "host allocation failed");
        return RB3_ENOMEM;
    }
    s->idx = idx;
    s->so = eff;
    for (int i = 0; i < so->workers; ++i) s->workers.emplace_back(worker_main, s);
    *out = s;
    return RB3_OK;
}

int rb3_server_submit(rb3_server *s, int32_t kind, const uint8_t *q, int64_t len, int32_t min_len, int64_t min_occ,
                      uint64_t *ticket) {
    if (!s || !ticket || len < 0 || (len > 0 && !q)) {
        set_error(RB3_EINVAL, "bad argument");
        return RB3_EINVAL;
    }
    if (kind != RB3_REQ_COUNT && kind != RB3_REQ_SMEM) {
        set_error(RB3_EINVAL, "unknown request kind");
        return RB3_EINVAL;
    }
    if (kind == RB3_REQ_SMEM && (min_len < 1 || min_occ < 1 || !index_both(s->idx))) {
        set_error(RB3_EINVAL, "SMEM request needs min_len, min_occ >= 1 and a both-strand index");
        return RB3_EINVAL;
    }
    if (len >= ((int64_t)1 << 31)) {
        set_error(RB3_ELIMIT, "query too long");
        return RB3_ELIMIT;
    }
    if (!valid_bytes(q, len)) {
        set_error(RB3_EINVAL, "byte outside ACGTNacgtn in the query");
        return RB3_EINVAL;
    }
    Request r;
    r.kind = kind;
    r.min_len = min_len;
    r.min_occ = min_occ;
    r.q.assign(q, q + len);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if ((int64_t)s->pending.size() >= s->so.max_queued) {
            set_error(RB3_EAGAIN, "server queue full: retry after polling results");
            return RB3_EAGAIN;
        }
        r.ticket = s->next_ticket++;
        *ticket = r.ticket;
        s->pending.push_back(std::move(r));
    }
    s->cv_work.notify_one();
    return RB3_OK;
}

int rb3_server_poll(rb3_server *s, int32_t wait_ms, rb3_result *res, int64_t res_cap, rb3_smem_t *recs,
                    int64_t rec_cap, int64_t *n_res, int64_t *n_recs) {
    if (!s || !n_res || !n_recs || res_cap < 0 || rec_cap < 0 || (res_cap > 0 && !res) || (rec_cap > 0 && !recs)) {
        set_error(RB3_EINVAL, "bad argument");
        return RB3_EINVAL;
    }
    *n_res = 0;
    *n_recs = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && wait_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty(); });
    int64_t nr = 0, nk = 0;
    while (!s->done.empty() && nr < res_cap) {
        Done &d = s->done.front();
        int64_t k = (int64_t)d.recs.size();
        if (nk + k > rec_cap) {
            if (nr == 0) {
                set_error(RB3_ENOSPC, "record buffer too small for the next result");
                *n_recs = k;  // the size needed
                return RB3_ENOSPC;
            }
            break;
        }
        d.r.smem_off = nk;
        res[nr++] = d.r;
        if (k) std::memcpy(recs + nk, d.recs.data(), k * sizeof(rb3_smem_t));
        nk += k;
        s->done.pop_front();
    }
    *n_res = nr;
    *n_recs = nk;
    return RB3_OK;
}

int rb3_server_stats(rb3_server *s, int64_t *queued, int64_t *inflight, int64_t *batches, int64_t *served,
                     int64_t *max_batch, int64_t *busy_us, int64_t *mem_budget) {
    if (!s) {
        set_error(RB3_EINVAL, "server is NULL");
        return RB3_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (queued) *queued = (int64_t)s->pending.size();
    if (mem_budget) *mem_budget = s->so.mem_budget;
    if (inflight) *inflight = s->inflight_batches;
    if (batches) *batches = s->batches;
    if (served) *served = s->served;
    if (max_batch) *max_batch = s->max_batch;
    if (busy_us) *busy_us = s->busy_us;
    return RB3_OK;
}

int rb3_server_replay(rb3_server *s, int32_t kind, const uint8_t *q, const int64_t *qlens, int64_t n,
                      int32_t min_len, int64_t min_occ, const double *arrival_s, double *latency_s,
                      double *wall_s) {
    if (!s || n < 0 || (n > 0 && (!qlens || !arrival_s || !latency_s))) {
        set_error(RB3_EINVAL, "bad argument");
        return RB3_EINVAL;
    }
    using clk = std::chrono::steady_clock;
    std::vector<int64_t> off(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + qlens[i];
    std::map<uint64_t, int64_t> who;
    std::mutex wmu;
    std::vector<int32_t> status(n, RB3_OK);
    std::atomic<int64_t> expected(n);  // results still to come; lowered by failed submissions
    const auto t0 = clk::now();
    auto since = [&](clk::time_point t) { return std::chrono::duration<double>(t - t0).count(); };
    // The poller takes out of the done queue only the results of this call's
    // own tickets; results of other clients' requests stay for their polls.
    std::thread poller([&] {
        int64_t got = 0;
        while (got < expected.load()) {
            std::vector<std::pair<uint64_t, int32_t>> mine;
            {
                std::unique_lock<std::mutex> lk(s->mu);
                s->cv_done.wait_for(lk, std::chrono::milliseconds(20), [&] { return !s->done.empty(); });
                std::lock_guard<std::mutex> lw(wmu);
                for (auto it = s->done.begin(); it != s->done.end();) {
                    if (who.count(it->r.ticket)) {
                        mine.emplace_back(it->r.ticket, it->r.status);
                        it = s->done.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            const double now = since(clk::now());
            std::lock_guard<std::mutex> lw(wmu);
            for (auto &tk : mine) {
                const int64_t i = who[tk.first];
                latency_s[i] = now - arrival_s[i];
                status[i] = tk.second;
                ++got;
            }
        }
    });
    for (int64_t i = 0; i < n; ++i) {
        while (since(clk::now()) < arrival_s[i]) std::this_thread::yield();
        uint64_t t = 0;
        int rc;
        // (wmu is never held across a submit: the poller takes s->mu, then wmu)
        while ((rc = rb3_server_submit(s, kind, q + off[i], qlens[i], min_len, min_occ, &t)) == RB3_EAGAIN)
            std::this_thread::yield();  // a full queue: the request waits, its latency counting from its arrival
        if (rc != RB3_OK) {
            std::lock_guard<std::mutex> lk(wmu);
            latency_s[i] = -1;
            status[i] = rc;
            expected.fetch_sub(1);
        } else {
            std::lock_guard<std::mutex> lk(wmu);
            who[t] = i;
        }
    }
    poller.join();
    if (wall_s) *wall_s = since(clk::now());
    for (int64_t i = 0; i < n; ++i)
        if (status[i] != RB3_OK) {
            set_error(status[i], "a request failed");
            return status[i];
        }
    return RB3_OK;
}

void rb3_server_free(rb3_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    delete s;
}

}  // extern "C"
