// The library's autotuner: picks the LF-chain chunk length of merges and the
// query segment length of SMEM calls by timing candidates on the caller's
// own data, and keeps the choice per (GPU architecture, size class) for
// later calls with the option left at 0. Results live in a process-wide
// table and, when the environment variable RB3_TUNE_CACHE names a file, in
// that file (one "key value" line per entry), read on first use.
//
// The occurrence-checkpoint interval is not a candidate: an index block of
// 128 symbols is 64 bytes, half of a 128-byte L2 line, and blocks of 64 or
// 256 symbols would cost the same one line per rank (with twice or the
// same index bytes), so there is nothing for a tuner to find there.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "rb3_internal.h"

namespace rb3 {

namespace {

std::mutex g_tune_mu;
std::map<std::string, int64_t> g_tune;
bool g_tune_loaded = false;

int ilog2(int64_t v) {
    int b = 0;
    while (v > 1) {
        v >>= 1;
        ++b;
    }
    return b;
}

std::string arch_of(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

void load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("RB3_TUNE_CACHE");
    if (!path || !*path) return;
    std::ifstream f(path);
    std::string key;
    int64_t v;
    while (f >> key >> v) g_tune[key] = v;
}

void store(const std::string &key, int64_t v) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_locked();
    g_tune[key] = v;
    const char *path = std::getenv("RB3_TUNE_CACHE");
    if (!path || !*path) return;
    std::ofstream f(path, std::ios::trunc);
    for (auto &kv : g_tune) f << kv.first << " " << kv.second << "\n";
}

int64_t lookup(const std::string &key) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_locked();
    auto it = g_tune.find(key);
    return it == g_tune.end() ? 0 : it->second;
}

}  // namespace

// Size classes: powers of two of the index size, the batch size and the
// mean string (query) length.
std::string merge_tune_key(int dev, int64_t n1, int64_t n2, int64_t m2) {
    std::ostringstream s;
    s << arch_of(dev) << "|merge|n1=" << ilog2(n1 > 0 ? n1 : 1) << "|n2=" << ilog2(n2 > 0 ? n2 : 1)
      << "|len=" << ilog2(m2 > 0 ? n2 / m2 : 1);
    return s.str();
}

std::string smem_tune_key(int dev, int64_t n, int64_t bases, int64_t nq) {
    std::ostringstream s;
    s << arch_of(dev) << "|smem|n=" << ilog2(n > 0 ? n : 1) << "|bases=" << ilog2(bases > 0 ? bases : 1)
      << "|qlen=" << ilog2(nq > 0 ? bases / nq : 1);
    return s.str();
}

int64_t tuned_chunk_len(int dev, int64_t n1, int64_t n2, int64_t m2) {
    return lookup(merge_tune_key(dev, n1, n2, m2));
}

// 0: not tuned; -1: tuned, the automatic rule won; > 0 the segment length.
int64_t tuned_smem_segment(int dev, int64_t n, int64_t bases, int64_t nq) {
    return lookup(smem_tune_key(dev, n, bases, nq));
}

void tune_store(const std::string &key, int64_t v) { store(key, v); }

}  // namespace rb3
