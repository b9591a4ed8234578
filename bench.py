#!/usr/bin/env python3
"""Benchmark: pangenome-shaped incremental BWT merge on one MI355X.

Workload (the pangenome merge configuration): a random 4 Mb base genome, 64
haplotypes derived with SNP rate 1e-3 and indel rate 1e-4; the index holds
haplotypes 0-31 on both strands (about 256 M symbols) and one step merges
haplotypes 32-63 on both strands (about 256 M new suffixes) into a copy of
it. The batch is resident in device memory before timing starts.

One JSON line on stdout; progress on stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BLOCK_BYTES = 64


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_2409_00613_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_2409_00613_amd", "csrc", f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def merge_method_bytes(st: dict) -> dict:
    """Bytes the method itself must move for one merge, per unit of work
    (the per-suffix figures of the measurement plan): for each non-sentinel
    new suffix one random index block for its rank, 1 B symbol read and 8 B
    rank written by the chain; one ideal sort pass over a 12-byte record,
    read and written (24 B); the emitted BWT symbol (1 B); and the
    interleave's streaming of the old and the merged BWT at 0.5 B per
    symbol."""
    n1, n2, m2 = st["n1"], st["n2"], st["m2"]
    rank = (n2 - m2) * BLOCK_BYTES
    chain_io = (n2 - m2) * 1 + n2 * 8
    sort = n2 * 24
    emit = n2 * 1
    interleave = n1 * 0.5 + (n1 + n2) * 0.5
    return {"rank": rank, "chain_io": chain_io, "sort": sort, "emit": emit, "interleave": interleave,
            "chain": rank + chain_io, "total": rank + chain_io + sort + emit + interleave}


def algorithmic_bytes(kernel: str, st: dict, steps: int) -> float | None:
    """Bytes moved by all launches of one kernel over the timed steps (per-unit
    figures times units, the units taken from the merge's own counters). For
    `chain` these are the method's bytes only (merge_method_bytes); what the
    implementation adds is in overhead_bytes."""
    n1, n2, m2 = st["n1"], st["n2"], st["m2"]
    per_step = {
        "chain": merge_method_bytes(st)["chain"],
        # fix-up steps over wide intervals: a block, the recorded low end, the
        # symbol, the key written
        "chain_fixup": st.get("fixup_index_steps", 0) * (BLOCK_BYTES + 8 + 1 + 8),
        # the other fix-up steps: the mask read to fold segments, then the
        # mask, low end and symbol read and the key written to replay them
        "fix_compose": (st["fixup_steps"] - st.get("fixup_index_steps", 0)) * 8,
        "fix_keys": (st["fixup_steps"] - st.get("fixup_index_steps", 0)) * (8 + 8 + 1 + 8),
        # per pass: key 8 B read for the histogram
        "sort_hist": n2 * 8 * st["sort_passes"],
        # per pass: key + value read and written (the first pass has no value
        # to read); packed 8-byte records between the first and last passes
        "sort_scatter": (n2 * (16 * (st["sort_passes"] - 1) + 20) if st.get("sort_packed")
                         else n2 * 24 * st["sort_passes"] - n2 * 4),
        # per active record per round: position, rank h further on, key written
        "tie_gather": st["tie_work"] * 12 if st.get("tie_doubling") else None,
        # per active record per round: its record and group (16 B), key (4 B),
        # rank update (4 B) and five 4-byte outputs
        "tie_rerank": st["tie_work"] * 44 if st.get("tie_doubling") else None,
        "tie_compact": st["tie_work"] * 40 if st.get("tie_doubling") else None,
        # sorted keys read once to find groups
        "tie_groups": n2 * 8,
        # key reads of the symbol walk (8 B each)
        "tie_walk": st["tie_work"] * 8 if not st.get("tie_doubling") else None,
        "tie_lanes": st["tie_small_reads"] * 8,
        "tie_deep": st["tie_deep_reads"] * 8,
        # sorted keys, old BWT read, merged BWT written (0.5 B per symbol)
        "interleave": n2 * 8 + n1 * 0.5 + (n1 + n2) * 0.5,
    }
    v = per_step.get(kernel)
    return None if v is None else float(v) * steps


def overhead_bytes(kernel: str, st: dict) -> float | None:
    """Per merge, what the implementation moves beyond the method's bytes:
    for `chain`, the second block of interval steps whose ends lie in
    different blocks and the 8-byte row mask recorded per unresolved step."""
    if kernel != "chain":
        return None
    return float((st["chain_steps"] - (st["n2"] - st["m2"])) * BLOCK_BYTES + st["fixup_steps"] * 8)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def read_traffic(kernel: str, workload: str, src_hash: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != src_hash:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(sample_len: int, threads: int):
    """The oracle timed on a bounded sample of the same workload: every
    haplotype cut to its first sample_len bases; the oracle builds the merged
    BWT by sorting all suffixes. Reported as new suffixes per second."""
    import oracle
    import synth
    w = synth.config_pangenome(genome_len=sample_len + 200, n_b1=32, n_new=32)
    cut = lambda s: synth.pack([x[:sample_len] for x in s.as_list()])
    b1, new = cut(w.b1), cut(w.new)
    allst = b1 + new
    codes, lens = oracle.expand(allst.data, allst.lens)
    n2 = 2 * (new.total + new.n)
    t0 = time.perf_counter()
    oracle.bwt(codes, lens, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": n2 / dt, "unit": "suffixes/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"naive-sort BWT of the merged list with every haplotype cut to its first "
                      f"{sample_len} bases ({int(lens.sum()) + lens.shape[0]} suffixes, {n2} of them new); "
                      f"{dt:.2f} s"}


def smem_bench(genome: int, n_index: int, n_queries: int, plain_queries: int, rates: list[float],
               served_queries: int, min_len: int = 31, steps: int = 2, batched_only: bool = False):
    """SMEM finding on a serving-shaped workload: closed-loop batched
    throughput, the plain one-query-per-call form, and served latency under
    Poisson arrivals at fractions of the batched saturation rate
    (batched_only: the batched calls alone, for counter runs)."""
    import synth
    from paper_2409_00613_amd import rb3
    t = time.perf_counter()
    w = synth.config_serving(genome_len=genome, n_index=n_index, n_unseen=8, n_queries=n_queries)
    log(f"serving workload: {n_index} haplotypes of ~{genome} bases, {n_queries} queries "
        f"({w.queries.total} bases) in {time.perf_counter() - t:.1f} s")
    t = time.perf_counter()
    # batches of 32 haplotypes keep every merge below the per-batch size limit;
    # device memory from torch's caching allocator, as a caller would pass it
    alloc = rb3.TorchAllocator(0)
    idx = rb3.rb3_build(w.index.slice(0, min(32, n_index)).data, w.index.slice(0, min(32, n_index)).lens,
                        allocator=alloc)
    for a in range(32, n_index, 32):
        part = w.index.slice(a, min(a + 32, n_index))
        idx.merge(part.data, part.lens)
        log(f"  merged haplotypes {a}..{min(a + 32, n_index) - 1}")
    n, m, _ = idx.info()
    log(f"query index: n={n} in {time.perf_counter() - t:.1f} s")
    bases = w.queries.total
    import torch
    qdev = torch.from_numpy(w.queries.data).cuda()  # queries resident in HBM before timing
    torch.cuda.synchronize()
    # the library's autotuner picks the segment length for this batch; the
    # timed calls (smem_segment 0) use its choice
    tuning = rb3.rb3_tune_smem(idx, qdev, w.queries.lens, min_len)
    log(f"tuned SMEM segment: {tuning['segment']} (-1: automatic rule; trial ms {tuning['trials']})")
    idx.smem(qdev, w.queries.lens, min_len)  # warm-up
    rb3.rb3_prof_reset()
    rb3.rb3_prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        recs, off = idx.smem(qdev, w.queries.lens, min_len)
    t1 = time.perf_counter()
    rb3.rb3_prof_enable(False)
    prof = rb3.rb3_prof_read()
    sst = rb3.rb3_last_smem_stats()
    exts, blocks = sst["extensions"], sst["blocks"]
    batched = bases * steps / (t1 - t0)
    qps = n_queries * steps / (t1 - t0)
    k_ms = prof.get("smem", (0, 0.0))[1] / steps
    roof = None
    if k_ms > 0:
        # the distinct index blocks the extensions read (one per extension
        # whose two rank positions share a block, else two), counted on the
        # device
        ab = blocks * BLOCK_BYTES
        ach = ab / (k_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "kernel": "smem", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": read_traffic("smem", f"serving{n_index}", kernel_source_hash()),
                "algorithmic_bytes_per_launch": ab,
                "avg_launch_ms": k_ms, "extensions_per_base": round(exts / bases, 3),
                "blocks_per_extension": round(blocks / max(exts, 1), 3)}
    log(f"SMEM batched: {batched / 1e9:.3f} G bases/s, {qps:.0f} queries/s, {len(recs)} SMEMs, "
        f"{exts} extensions, smem kernel {k_ms:.2f} ms")
    config = {"workload": "serving", "genome_len": genome, "haplotypes_indexed": n_index,
              "both_strands": True, "n": n, "queries": n_queries, "query_bases": bases,
              "min_len": min_len, "min_occ": 1, "query_lengths": "log-uniform 100-100000"}
    rle = rle_bench(idx, n, qdev, w.queries.lens, min_len, bases, steps, recs, off)
    hapl = hapl_bench(idx, n, w.queries, n_index, steps)
    if batched_only:
        idx.close()
        return {"metric": "SMEM query bases/s", "value": round(batched, 1), "unit": "bases/s",
                "config": config, "roofline": roof, "tuning": tuning, "run_length": rle, "hapl": hapl}
    # plain form: one query per call
    k = min(plain_queries, n_queries)
    pq = w.queries.slice(0, k)
    t0 = time.perf_counter()
    for i in range(k):
        one = pq.slice(i, i + 1)
        idx.smem(one.data, one.lens, min_len)
    t1 = time.perf_counter()
    plain = pq.total / (t1 - t0)
    log(f"SMEM plain (one query per call, {k} queries): {plain / 1e9:.4f} G bases/s")
    served = []
    srv = rb3.Server(idx, workers=4)
    m_served = min(served_queries, n_queries)
    sq = w.queries.slice(0, m_served)
    # warm-up: the workers' device pools fill on their first batches
    wq = w.queries.slice(0, min(1000, m_served))
    srv.replay(rb3.RB3_REQ_SMEM, wq.data, wq.lens, synth.poisson_arrivals(wq.n, rates[0] * qps), min_len, 1)
    for frac in rates:
        lam = frac * qps
        arr = synth.poisson_arrivals(m_served, lam)
        lat, wall = srv.replay(rb3.RB3_REQ_SMEM, sq.data, sq.lens, arr, min_len, 1)
        served.append({"load": frac, "qps": round(lam, 1), "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                       "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                       "bases_per_s": round(sq.total / wall, 1), "queries": m_served})
        log(f"SMEM served at {frac:.2f} x saturation ({lam:.0f} q/s): p50 {served[-1]['p50_ms']} ms, "
            f"p99 {served[-1]['p99_ms']} ms")
    st = srv.stats()
    srv.close()
    idx.close()
    return {"metric": "SMEM query bases/s", "value": round(batched, 1), "unit": "bases/s",
            "plain_one_query_per_call": round(plain, 1), "served": served, "server": st,
            "config": config, "roofline": roof, "tuning": tuning, "run_length": rle, "hapl": hapl}


def hapl_bench(idx, n, queries, n_index, steps, n_reads=200_000, read_len=125, bands=(10, 25),
               long_reads=3500, long_len=10_000):
    """Local haplotype enumeration (revised BWA-SW, semi-global) of short
    reads on the serving index: n_reads windows of read_len bases cut at
    seeded offsets from the serving queries (excerpts of unindexed
    haplotypes with 1% substitutions and 0.1% indels), device-resident, at
    the paper's bands (10 for short reads, 25 its default). Value: query
    bases/s of the batched call; the kernel's index-block bytes over its
    time give the roofline."""
    from paper_2409_00613_amd import rb3
    import torch
    g = np.random.default_rng(17)
    lens = queries.lens
    offs = np.concatenate([[0], np.cumsum(lens)])
    long_ = np.nonzero(lens >= read_len)[0]
    pick = long_[g.integers(0, long_.shape[0], n_reads)]
    st = offs[pick] + (g.random(n_reads) * (lens[pick] - read_len + 1)).astype(np.int64)
    data = queries.data[(st[:, None] + np.arange(read_len)[None, :]).ravel()]
    qlens = np.full(n_reads, read_len, np.int64)
    qdev = torch.from_numpy(np.ascontiguousarray(data)).cuda()
    torch.cuda.synchronize()
    bases = n_reads * read_len
    out = {"reads": n_reads, "read_len": read_len, "source": "windows of the serving queries", "bands": {}}
    for band in bands:
        _, off = idx.hapl(qdev, qlens, band=band)  # warm-up; sizes the output
        cap = int(off[-1])
        rb3.rb3_prof_reset()
        rb3.rb3_prof_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            recs, off = idx.hapl(qdev, qlens, cap=cap, band=band)
        t1 = time.perf_counter()
        rb3.rb3_prof_enable(False)
        prof = rb3.rb3_prof_read()
        hs = rb3.rb3_last_hapl_stats()
        # the LDS-table kernel, plus the device-memory one for the queries
        # that outgrew it
        k_ms = (prof.get("hapl_wave", (0, 0.0))[1] + prof.get("hapl", (0, 0.0))[1]) / steps
        rate = bases * steps / (t1 - t0)
        ab = hs["blocks"] * BLOCK_BYTES
        ach = ab / (k_ms / 1e3) / 1e9 if k_ms > 0 else 0.0
        out["bands"][str(band)] = {
            "bases_per_s": round(rate, 1), "ms_per_call": round((t1 - t0) / steps * 1e3, 3),
            "kernel_ms": round(k_ms, 3), "results": int(off[-1]),
            "reads_with_results": int(np.count_nonzero(np.diff(off))),
            "extensions_per_base": round(hs["extensions"] / bases, 3),
            "blocks_per_extension": round(hs["blocks"] / max(hs["extensions"], 1), 3),
            "cells_per_position": round(hs["cells"] / bases, 2),
            "reads_moved_to_device_tables": hs["moved"],
            "roofline": {"bound": "hbm", "kernel": "hapl_wave", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                         "traffic": read_traffic("hapl_wave", f"serving{n_index}_band{band}", kernel_source_hash()),
                         "algorithmic_bytes_per_launch": ab, "avg_launch_ms": k_ms}}
        log(f"haplotype enumeration, band {band}: {rate / 1e6:.2f} M bases/s ({n_reads} reads of {read_len}), "
            f"kernel {k_ms:.1f} ms, {hs['extensions'] / bases:.2f} extensions/base, {int(off[-1])} results")
    # long reads (the paper's long-read rows use band 25): windows of
    # long_len bases of the serving queries, one call
    if long_reads > 0:
        lq = np.nonzero(lens >= long_len)[0]
        pick = lq[g.integers(0, lq.shape[0], long_reads)]
        st = offs[pick] + (g.random(long_reads) * (lens[pick] - long_len + 1)).astype(np.int64)
        data = queries.data[(st[:, None] + np.arange(long_len)[None, :]).ravel()]
        ldev = torch.from_numpy(np.ascontiguousarray(data)).cuda()
        llens = np.full(long_reads, long_len, np.int64)
        torch.cuda.synchronize()
        _, off = idx.hapl(ldev, llens, band=25)  # warm-up; sizes the output
        cap = int(off[-1])
        t0 = time.perf_counter()
        recs, off = idx.hapl(ldev, llens, cap=cap, band=25)
        t1 = time.perf_counter()
        hs = rb3.rb3_last_hapl_stats()
        lb = long_reads * long_len
        out["long_reads"] = {"reads": long_reads, "read_len": long_len, "band": 25,
                             "bases_per_s": round(lb / (t1 - t0), 1), "ms_per_call": round((t1 - t0) * 1e3, 3),
                             "results": int(off[-1]), "reads_with_results": int(np.count_nonzero(np.diff(off))),
                             "extensions_per_base": round(hs["extensions"] / lb, 3),
                             "reads_moved_to_device_tables": hs["moved"]}
        log(f"haplotype enumeration of long reads, band 25: {lb / (t1 - t0) / 1e6:.2f} M bases/s "
            f"({long_reads} reads of {long_len}), {int(off[-1])} results, {hs['moved']} reads moved")
    return out


def hapl_only(args):
    """Haplotype enumeration alone: the serving index (320 haplotypes of a
    10 Mb genome, built by ten merges of 32), then hapl_bench. Value: query
    bases/s of 125 bp reads at band 10."""
    import synth
    from paper_2409_00613_amd import rb3
    w = synth.config_serving(genome_len=10_000_000, n_index=320, n_unseen=8, n_queries=10_000)
    alloc = rb3.TorchAllocator(0)
    idx = rb3.rb3_build(w.index.slice(0, 32).data, w.index.slice(0, 32).lens, allocator=alloc)
    for a in range(32, 320, 32):
        part = w.index.slice(a, a + 32)
        idx.merge(part.data, part.lens)
    n, m, _ = idx.info()
    log(f"serving index: n={n}")
    h = hapl_bench(idx, n, w.queries, 320, args.steps)
    idx.close()
    b10 = h["bands"]["10"]
    out = {"metric": "haplotype enumeration query bases/s", "value": b10["bases_per_s"], "unit": "bases/s",
           "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": b10["ms_per_call"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": "hapl", "genome_len": 10_000_000, "haplotypes_indexed": 320, "n": n,
                      "reads": h["reads"], "read_len": h["read_len"], "band": 10},
           "roofline": b10["roofline"], "hapl": h}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = hapl_cpu_baseline()
    return out


def hapl_cpu_baseline(n_reads: int = 40, read_len: int = 125):
    """The oracle's haplotype enumeration on a bounded sample: reads of the
    same shape against a 32-haplotype index of a 30 kb genome (the oracle
    holds a suffix array of the whole text, so the serving index is out of
    its reach), band 10. Reported as query bases/s."""
    import oracle
    import synth
    w = synth.config_pangenome(genome_len=30_000, n_b1=32, n_new=4)
    codes, lens = oracle.expand(w.b1.data, w.b1.lens)
    text = oracle.Text(codes, lens)
    enc = np.zeros(256, np.uint8)
    for i, c in enumerate(b"ACGTN"):
        enc[c] = i + 1
    g = np.random.default_rng(3)
    reads = []
    for j in range(n_reads):
        src = w.new.get(j % w.new.n)
        s = int(g.integers(0, len(src) - read_len))
        reads.append(enc[synth.mutate(np.frombuffer(src[s:s + read_len], np.uint8), 0.01, 0.001, g)])
    t0 = time.perf_counter()
    for r in reads:
        text.hapl(r, band=10)
    dt = time.perf_counter() - t0
    return {"value": round(n_reads * read_len / dt, 1), "unit": "bases/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_reads} reads of {read_len} bases (1% substitutions, 0.1% indels) against 32 "
                      f"haplotypes of a 30 kb genome ({codes.shape[0]} symbols), band 10; {dt:.2f} s"}


def rle_bench(idx, n, qdev, qlens, min_len, bases, steps, want_recs, want_off):
    """The same index in the run-length static form: its size against the
    3-bit-plane form, the build time, and the batched SMEM rate on it (the
    records must equal the plane index's)."""
    from paper_2409_00613_amd import rb3
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = rb3.rb3_rle_build(idx)
    build_s = time.perf_counter() - t
    info = r.info()
    plain_bytes = ((n >> 7) + 1) * 64 + ((n >> 24) + 1) * 64
    recs, off = r.smem(qdev, qlens, min_len)  # warm-up, and the parity check
    same = bool(np.array_equal(recs, want_recs) and np.array_equal(off, want_off))
    rb3.rb3_prof_reset()
    rb3.rb3_prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        r.smem(qdev, qlens, min_len)
    t1 = time.perf_counter()
    rb3.rb3_prof_enable(False)
    prof = rb3.rb3_prof_read()
    sst = rb3.rb3_last_smem_stats()
    k_ms = prof.get("smem_rle", (0, 0.0))[1] / steps
    rate = bases * steps / (t1 - t0)
    blk = sst["blocks"] * 128
    out = {"bytes": info["bytes"], "bytes_per_symbol": round(info["bytes"] / n, 4),
           "plane_form_bytes": plain_bytes, "compression": round(plain_bytes / info["bytes"], 2),
           "runs": info["runs"], "mean_run": round(n / max(info["runs"], 1), 2), "blocks": info["blocks"],
           "row_shift": info["row_shift"], "build_s": round(build_s, 3),
           "smem_bases_per_s": round(rate, 1), "smem_kernel_ms": round(k_ms, 3),
           "blocks_decoded": sst["blocks"], "block_GB_per_s": round(blk / (k_ms / 1e3) / 1e9, 1) if k_ms else None,
           "smem_equal_to_plane_form": same}
    log(f"run-length form: {info['bytes'] / 1e9:.3f} GB ({out['bytes_per_symbol']} B/symbol, "
        f"{out['compression']}x smaller than the plane form), {info['runs']} runs, built in {build_s:.2f} s; "
        f"SMEM {rate / 1e9:.3f} G bases/s (kernel {k_ms:.2f} ms), records equal: {same}")
    r.close()
    return out


def timed_merges(b1, new, steps: int, warmup: int):
    """Merge a device-resident batch into a fresh copy of b1, warmup + steps
    times; the timed region covers the steps only (copy + merge each)."""
    import torch
    from paper_2409_00613_amd import rb3
    new_dev = torch.from_numpy(new.data).cuda()
    new_lens = new.lens.copy()
    torch.cuda.synchronize()

    def step():
        idx = b1.clone()
        idx.merge(new_dev, new_lens)
        return idx

    for i in range(warmup):
        step().close()
        log(f"warmup {i + 1}/{warmup} done")
    torch.cuda.synchronize()
    rb3.rb3_prof_reset()
    rb3.rb3_prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for i in range(steps):
        if last is not None:
            last.close()
        last = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rb3.rb3_prof_enable(False)
    prof = rb3.rb3_prof_read()
    st = last.merge_stats()
    n_out, _, _ = last.info()
    last.close()
    # the same steps without the per-launch timing events, for their cost
    torch.cuda.synchronize()
    u0 = time.perf_counter()
    for i in range(steps):
        step().close()
    torch.cuda.synchronize()
    unprof_ms = (time.perf_counter() - u0) / steps * 1e3
    del new_dev
    log(f"timed {steps} steps in {t1 - t0:.3f} s; without kernel timing events {unprof_ms:.3f} ms/step")
    for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        log(f"  {k:24s} launches={v[0]:6d}  ms/step={v[1] / steps:9.3f}")
    return {"ms": (t1 - t0) / steps * 1e3, "prof": prof, "stats": st, "n_out": n_out, "unprofiled_ms": unprof_ms}


def host_input_merges(b1, new, steps: int):
    """The same merge fed from host memory (the batch in pinned host memory),
    every upload inside the timed region. Sequential: each step uploads its
    batch, then merges it. Overlapped: while a step merges (on the index's own
    stream), the next step's batch is uploaded on a side stream (default
    priority) into the other of two device buffers, so the PCIe transfer hides
    behind the merge."""
    import torch
    host = torch.from_numpy(new.data).pin_memory()
    lens = new.lens.copy()
    bufs = [torch.empty(host.numel(), dtype=torch.uint8, device="cuda") for _ in range(2)]
    side = torch.cuda.Stream()

    def merge_from(buf):
        idx = b1.clone()
        idx.merge(buf, lens)
        return idx

    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        bufs[0].copy_(host, non_blocking=True)
    torch.cuda.synchronize()
    up_ms = (time.perf_counter() - t) / steps * 1e3
    merge_from(bufs[0]).close()  # warm-up
    torch.cuda.synchronize()
    seq = []
    for _ in range(steps):
        t = time.perf_counter()
        bufs[0].copy_(host, non_blocking=True)
        torch.cuda.synchronize()
        merge_from(bufs[0]).close()
        torch.cuda.synchronize()
        seq.append((time.perf_counter() - t) * 1e3)
    # overlapped: step i's time runs from the end of step i - 1 (its batch
    # uploaded during that step) to the end of its own merge and the next
    # batch's upload
    ovl = []
    with torch.cuda.stream(side):
        bufs[0].copy_(host, non_blocking=True)
    side.synchronize()
    t = time.perf_counter()
    for i in range(steps):
        if i + 1 < steps:
            with torch.cuda.stream(side):
                bufs[(i + 1) % 2].copy_(host, non_blocking=True)
        merge_from(bufs[i % 2]).close()
        side.synchronize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ovl.append((t1 - t) * 1e3)
        t = t1
    n2 = 2 * (new.total + new.n)
    sq, ov = float(np.median(seq)), float(np.median(ovl))
    log(f"host input: upload {up_ms:.2f} ms; upload then merge median {sq:.2f} ms/step "
        f"({min(seq):.2f}-{max(seq):.2f}); upload beside the previous merge median {ov:.2f} ms/step "
        f"({min(ovl):.2f}-{max(ovl):.2f})")
    return {"batch_bytes": int(host.numel()), "upload_ms": round(up_ms, 3),
            "upload_gb_per_s": round(host.numel() / (up_ms / 1e3) / 1e9, 2),
            "sequential_ms_per_step": {"median": round(sq, 3), "min": round(min(seq), 3), "max": round(max(seq), 3)},
            "overlapped_ms_per_step": {"median": round(ov, 3), "min": round(min(ovl), 3), "max": round(max(ovl), 3)},
            "sequential_suffixes_per_s": round(n2 / (sq / 1e3), 1),
            "overlapped_suffixes_per_s": round(n2 / (ov / 1e3), 1), "steps": steps,
            "overlap_gain": round(sq / ov, 3)}


def roofline_of(prof: dict, st: dict, steps: int, workload: str, src_hash: str):
    """Roofline entry for the kernel with the largest total time among those
    that run alone: the tie kernels of the size classes run at the same time
    on side streams, so their event times overlap and are left out."""
    alone = {k: v for k, v in prof.items() if not k.startswith("tie_") or k == "tie_groups"}
    if not alone:
        return None
    dom = max(alone.items(), key=lambda kv: kv[1][1])[0]
    dom_ms_total = prof[dom][1]
    launches = prof[dom][0]
    ab = algorithmic_bytes(dom, st, steps)
    if ab is None or dom_ms_total <= 0:
        return None
    achieved = ab / (dom_ms_total / 1e3) / 1e9
    ov = overhead_bytes(dom, st)
    return {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": read_traffic(dom, workload, src_hash), "algorithmic_bytes_per_launch": ab / launches,
            "avg_launch_ms": dom_ms_total / launches,
            "implementation_overhead_bytes_per_launch": ov}


def merge_roofline(st: dict, ms_per_step: float):
    """The whole merge against the HBM roofline: the method's bytes for one
    merge (merge_method_bytes) over the measured time of a step (the step also
    copies the 0.5 B-per-symbol existing index first)."""
    mb = merge_method_bytes(st)
    achieved = mb["total"] / (ms_per_step / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "method_bytes_per_merge": mb,
            "method_bytes_per_new_suffix": round(mb["total"] / st["n2"], 2),
            "roofline_suffixes_per_s": round(st["n2"] / (mb["total"] / (HBM_PEAK_GBS * 1e9)), 1)}


def plain_vs_batched(b1_strings, new, chunk: int, k: int):
    """The same merge of the first k new strings in the batched form (one
    LF-chain launch over every chunk) and in the plain form (one launch per
    string); both results must be identical."""
    import torch
    from paper_2409_00613_amd import rb3
    sub = new.slice(0, min(k, new.n))
    sub_dev = torch.from_numpy(sub.data).cuda()
    out = {}
    exports = {}
    for form, per_string in (("batched", False), ("plain", True)):
        b1 = rb3.rb3_build(b1_strings.data, b1_strings.lens, chunk_len=chunk, launch_per_string=per_string)
        for rep in range(2):  # the first is a warm-up
            idx = b1.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            idx.merge(sub_dev, sub.lens)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if rep == 1:
                exports[form] = idx.export()
            idx.close()
        st_n2 = 2 * (sub.total + sub.n)
        out[form] = {"ms": round(dt * 1e3, 3), "suffixes_per_s": round(st_n2 / dt, 1)}
        b1.close()
        log(f"{form} form, {sub.n} strings ({st_n2} new suffixes): {dt * 1e3:.1f} ms")
    assert np.array_equal(exports["batched"], exports["plain"]), "plain and batched forms disagree"
    out["strings"] = sub.n
    out["strands"] = 2 * sub.n
    out["new_suffixes"] = 2 * (sub.total + sub.n)
    out["batched_over_plain"] = round(out["plain"]["ms"] / out["batched"]["ms"], 2)
    out["identical"] = True
    return out


def locate_bench(args):
    """Locate on the pangenome index of the default workload (32 + 32
    haplotypes of a 4 Mb genome, both strands, 512 M symbols) with
    suffix-array samples every 32 positions: the index is built from the
    first 32 haplotypes and the other 32 are merged in (the merge keeps the
    samples; its time with samples is reported), then rows drawn uniformly
    are located (value: located rows/s), and Locate1 returns one occurrence
    for the SA interval of each of 100,000 25-mers cut from the haplotypes.
    Inputs are device-resident before timing."""
    import torch
    import synth
    from paper_2409_00613_amd import rb3
    rate = args.ssa
    w = synth.config_pangenome(genome_len=args.genome)
    alloc = rb3.TorchAllocator(0)
    idx = rb3.rb3_build(w.b1.data, w.b1.lens, allocator=alloc, ssa_rate=rate)
    plain = rb3.rb3_build(w.b1.data, w.b1.lens, allocator=alloc)
    new_dev = torch.from_numpy(w.new.data).cuda()
    torch.cuda.synchronize()
    merge_ms = {}
    merge_kernels = {}
    for name, ix in (("with_samples", idx), ("without_samples", plain)):
        rb3.rb3_prof_reset()
        rb3.rb3_prof_enable(True)
        t0 = time.perf_counter()
        ix.merge(new_dev, w.new.lens)
        torch.cuda.synchronize()
        merge_ms[name] = round((time.perf_counter() - t0) * 1e3, 2)
        rb3.rb3_prof_enable(False)
        merge_kernels[name] = {k: round(v[1], 3) for k, v in rb3.rb3_prof_read().items() if v[1] >= 0.2}
    plain.close()
    for k in sorted(merge_kernels["with_samples"], key=lambda k: -merge_kernels["with_samples"][k])[:10]:
        log(f"  merge kernel {k:16s} {merge_kernels['with_samples'][k]:8.2f} ms with samples, "
            f"{merge_kernels['without_samples'].get(k, 0.0):8.2f} ms without")
    n, m, _ = idx.info()
    r_, nsmp = idx.ssa_info()
    log(f"index n={n}, {nsmp} samples (distance {rate}); merge of the second 32 haplotypes: "
        f"{merge_ms['with_samples']} ms with samples, {merge_ms['without_samples']} ms without")
    g = torch.Generator(device="cpu").manual_seed(7)
    nrows = args.locate_rows
    rows = torch.randint(0, n, (nrows,), generator=g, dtype=torch.int64).cuda()
    torch.cuda.synchronize()
    idx.locate(rows)  # warm-up
    rb3.rb3_prof_reset()
    rb3.rb3_prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        idx.locate(rows)
    t1 = time.perf_counter()
    rb3.rb3_prof_enable(False)
    prof = rb3.rb3_prof_read()
    steps_lf = rb3.rb3_last_locate_stats()["lf_steps"]
    k_ms = prof.get("locate", (0, 0.0))[1] / args.steps
    rate_rows = nrows * args.steps / (t1 - t0)
    # per LF step: the row's 64-byte block, its 16 bytes of sample words and
    # 4-byte block count; per row: its index in, the final sample test, the
    # 8-byte sample value and the 16-byte answer out
    ab = steps_lf * (BLOCK_BYTES + 16 + 4) + nrows * (8 + 20 + 8 + 16)
    ach = ab / (k_ms / 1e3) / 1e9 if k_ms > 0 else 0.0
    log(f"locate: {rate_rows / 1e6:.1f} M rows/s ({steps_lf / nrows:.2f} LF steps per row), "
        f"kernel {k_ms:.2f} ms per {nrows} rows")
    # Locate1 on the intervals of 25-mers cut from the haplotypes
    rnd = np.random.default_rng(11)
    allst = w.b1 + w.new
    pats = []
    for _ in range(args.locate1_queries):
        sidx = int(rnd.integers(0, allst.n))
        s_ = allst.get(sidx)
        a = int(rnd.integers(0, len(s_) - 25))
        pats.append(s_[a:a + 25])
    q = synth.pack(pats)
    lo, hi = idx.count(q.data, q.lens)
    lo_d, hi_d = torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda()
    torch.cuda.synchronize()
    idx.locate1(lo_d, hi_d)  # warm-up
    rb3.rb3_prof_reset()
    rb3.rb3_prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        idx.locate1(lo_d, hi_d)
    t1 = time.perf_counter()
    rb3.rb3_prof_enable(False)
    prof1 = rb3.rb3_prof_read()
    l1_steps = rb3.rb3_last_locate_stats()["lf_steps"]
    l1_ms = prof1.get("locate1", (0, 0.0))[1] / args.steps
    l1_rate = len(pats) * args.steps / (t1 - t0)
    occ = hi - lo
    log(f"locate1: {l1_rate / 1e6:.2f} M intervals/s, {l1_steps / len(pats):.2f} rank-all steps per interval "
        f"(mean occurrences {occ.mean():.1f}), kernel {l1_ms:.2f} ms per {len(pats)} intervals")
    idx.close()
    out = {"metric": "located rows/s", "value": round(rate_rows, 1), "unit": "rows/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 1, "ms_per_step": round((t1 - t0) / args.steps * 1e3, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
           "data": "synthetic",
           "config": {"workload": "locate", "genome_len": args.genome, "haplotypes": 64, "both_strands": True,
                      "n": n, "ssa_rate": rate, "samples": nsmp, "rows": nrows,
                      "locate1_intervals": len(pats), "locate1_pattern_len": 25},
           "roofline": {"bound": "hbm", "kernel": "locate", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                        "traffic": read_traffic("locate", "locate", kernel_source_hash()),
                        "algorithmic_bytes_per_launch": ab, "avg_launch_ms": k_ms,
                        "lf_steps_per_row": round(steps_lf / nrows, 3)},
           "locate1": {"intervals_per_s": round(l1_rate, 1), "kernel_ms": round(l1_ms, 3),
                       "rank_all_steps_per_interval": round(l1_steps / len(pats), 3),
                       "mean_occurrences": round(float(occ.mean()), 2)},
           "merge_ms": merge_ms, "merge_kernels_ms": merge_kernels, "source_hash": kernel_source_hash()}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = locate_cpu_baseline(args.cpu_sample)
    return out


def locate_cpu_baseline(sample_len: int):
    """The oracle on a bounded sample of the same workload: every haplotype
    cut to its first sample_len bases; the oracle sorts every suffix to get
    the suffix array and reads each row's position from it. Reported as
    located rows per second over the whole sample."""
    import oracle
    import synth
    w = synth.config_pangenome(genome_len=sample_len + 200, n_b1=32, n_new=32)
    cut = lambda s: synth.pack([x[:sample_len] for x in s.as_list()])
    allst = cut(w.b1) + cut(w.new)
    codes, lens = oracle.expand(allst.data, allst.lens)
    threads = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    _, S = oracle.bwt(codes, lens, nthreads=threads, want_sa=True)
    j, off = oracle.locate(S, lens, np.arange(S.shape[0]))
    dt = time.perf_counter() - t0
    return {"value": round(S.shape[0] / dt, 1), "unit": "rows/s", "cores": threads, "kind": "oracle",
            "sample": f"suffix sort of the 64 haplotypes cut to their first {sample_len} bases "
                      f"({S.shape[0]} rows), then every row located; {dt:.2f} s"}


def incremental_bench(args):
    """Large incremental build: 100 haplotypes of a 100 Mb genome with
    segmental duplications, merged 10 at a time (the first batch is a build
    into an empty index). Each batch is uploaded to the device before its
    merge is timed."""
    import torch
    import synth
    from paper_2409_00613_amd import rb3
    t = time.perf_counter()
    inc = synth.config_incremental()
    log(f"base genome with duplications: {inc.base.shape[0]} bases in {time.perf_counter() - t:.1f} s")
    alloc = rb3.TorchAllocator(0)
    per = inc.n_hap // args.batches
    idx = None
    batches = []
    total_new = 0
    total_s = 0.0
    rb3.rb3_prof_reset()
    rb3.rb3_prof_enable(True)
    torch.cuda.reset_peak_memory_stats()
    dev_free_min = None
    for b in range(args.batches):
        t = time.perf_counter()
        batch = inc.batch(b * per, per)
        gen_s = time.perf_counter() - t
        bdev = torch.from_numpy(batch.data).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if idx is None:
            idx = rb3.rb3_build(bdev, batch.lens, allocator=alloc, chunk_len=args.chunk)
        else:
            idx.merge(bdev, batch.lens)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        free, tot = torch.cuda.mem_get_info()
        dev_free_min = free if dev_free_min is None else min(dev_free_min, free)
        del bdev
        st = idx.merge_stats()
        n, m, _ = idx.info()
        new_suffixes = st["n2"]
        total_new += new_suffixes
        total_s += dt
        batches.append({"batch": b, "n1": st["n1"], "n2": new_suffixes, "n": n, "ms": round(dt * 1e3, 1),
                        "suffixes_per_s": round(new_suffixes / dt, 1), "tie_max_depth": st["tie_max_depth"],
                        "max_group": st["max_group"], "tie_doubling": st["tie_doubling"],
                        "fixup_steps": st["fixup_steps"], "fixup_index_steps": st["fixup_index_steps"]})
        log(f"batch {b}: {per} haplotypes generated in {gen_s:.1f} s; {new_suffixes} new suffixes merged "
            f"into n1={st['n1']} in {dt * 1e3:.1f} ms ({new_suffixes / dt / 1e9:.2f} G/s); n={n}")
    rb3.rb3_prof_enable(False)
    prof = rb3.rb3_prof_read()
    peak_alloc = torch.cuda.max_memory_allocated()
    kernels = {k: {"launches": v[0], "ms_total": v[1]} for k, v in prof.items()}
    for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])[:12]:
        log(f"  {k:24s} launches={v[0]:6d}  ms total={v[1]:9.1f}")
    if idx is not None:
        n, m, _ = idx.info()
        idx.close()
    return {"metric": "BWT-merge suffixes inserted/s", "value": round(total_new / total_s, 1),
            "unit": "suffixes/s", "n_gpus": 1, "steps": args.batches, "warmup": 0,
            "ms_per_step": round(total_s / args.batches * 1e3, 1), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
            "config": {"workload": "incremental", "genome_len": int(inc.base.shape[0]),
                       "haplotypes": inc.n_hap, "batches": args.batches, "haplotypes_per_batch": per,
                       "both_strands": True, "segmental_duplications": "0.1% of the base, 1-50 kb, half inverted",
                       "n_final": n},
            "batches": batches, "total_merge_s": round(total_s, 2),
            "peak_hbm_allocated_bytes": int(peak_alloc), "device_free_min_bytes": int(dev_free_min),
            "kernels": kernels, "source_hash": kernel_source_hash()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--genome", type=int, default=4_000_000, help="base genome length")
    ap.add_argument("--chunk", type=int, default=0, help="LF-chain chunk length (0 = library default)")
    ap.add_argument("--cpu-sample", type=int, default=120_000,
                    help="haplotype prefix length for the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-host-input", action="store_true",
                    help="skip the merges fed from pinned host memory (PCIe-inclusive rate)")
    ap.add_argument("--no-smem", action="store_true", help="skip the SMEM serving measurement")
    ap.add_argument("--no-incremental", action="store_true",
                    help="skip the large incremental build (10 batches of 10 haplotypes of 100 Mb)")
    ap.add_argument("--smem-haplotypes", type=int, default=320,
                    help="haplotypes in the SMEM serving index of the default run (320: the full serving "
                         "configuration)")
    ap.add_argument("--smem-batched-only", action="store_true",
                    help="SMEM: the batched calls only (no per-query calls, no served latency); for counter runs")
    ap.add_argument("--workload", default="pangenome_merge",
                    choices=["pangenome_merge", "uneven_merge", "incremental", "serving", "locate", "hapl"],
                    help="pangenome_merge: 32 haplotypes into 32 (default); uneven_merge: 10,000 "
                         "log-normal contigs and 2 chromosomes into the same index, plus the plain "
                         "one-launch-per-string form on a sample; incremental: 100 haplotypes of a "
                         "100 Mb genome merged in 10 batches; serving: the full serving configuration "
                         "(320 haplotypes) only; locate: rows located and Locate1 on the pangenome "
                         "index with suffix-array samples; hapl: haplotype enumeration alone on the "
                         "serving index")
    ap.add_argument("--plain-strings", type=int, default=200,
                    help="uneven_merge: input strings in the plain-vs-batched sample")
    ap.add_argument("--batches", type=int, default=10, help="incremental: number of batches")
    ap.add_argument("--ssa", type=int, default=32, help="locate: suffix-array sampling distance")
    ap.add_argument("--locate-rows", type=int, default=4_000_000, help="locate: rows per call")
    ap.add_argument("--locate1-queries", type=int, default=100_000, help="locate: Locate1 intervals per call")

    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES (three times) and exit; "
                         "used to scale hardware byte counters")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(args.copy_calibration, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_calibration, "copies": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2409_00613_amd import rb3

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload == "serving":
        res = smem_bench(10_000_000, 320, 10_000, 500, [0.25, 0.5, 0.8], 10_000)
        if not args.no_cpu_baseline:
            res["hapl"]["cpu_baseline"] = hapl_cpu_baseline()
        res.update({"n_gpus": 1, "steps": 2, "warmup": 1, "higher_is_better": True, "scaling": "weak",
                    "vs_baseline": None, "dtype": "int64", "data": "synthetic"})
        print(json.dumps(res), flush=True)
        return
    if args.workload == "incremental":
        res = incremental_bench(args)
        print(json.dumps(res), flush=True)
        return
    if args.workload == "locate":
        res = locate_bench(args)
        print(json.dumps(res), flush=True)
        return
    if args.workload == "hapl":
        res = hapl_only(args)
        print(json.dumps(res), flush=True)
        return
    workload = args.workload
    t = time.perf_counter()
    w = synth.config_pangenome(genome_len=args.genome)
    b1_strings, new_strings = w.b1, w.new
    if workload == "uneven_merge":
        u = synth.config_uneven(genome_len=args.genome)
        b1_strings, new_strings = u.b1, u.new
    log(f"generated {b1_strings.n} indexed + {new_strings.n} new strings ({new_strings.total} new bases) "
        f"in {time.perf_counter() - t:.1f} s")

    alloc = rb3.TorchAllocator(0)
    t = time.perf_counter()
    b1 = rb3.rb3_build(b1_strings.data, b1_strings.lens, allocator=alloc, chunk_len=args.chunk)
    torch.cuda.synchronize()
    n1, m1, _ = b1.info()
    log(f"built existing index: n1={n1} m1={m1} in {time.perf_counter() - t:.1f} s")
    tuning = None
    if args.chunk == 0:
        # the library's autotuner picks the chain chunk length on this batch;
        # the timed merges (chunk_len 0) use its choice
        nd = torch.from_numpy(new_strings.data).cuda()
        tuning = rb3.rb3_tune_merge(b1, nd, new_strings.lens)
        del nd
        log(f"tuned chunk length: {tuning['chunk_len']} (trial ms {tuning['trials']})")
    r = timed_merges(b1, new_strings, args.steps, args.warmup)
    st, ms, prof, n_out = r["stats"], r["ms"], r["prof"], r["n_out"]
    n2 = st["n2"]
    value = n2 / (ms / 1e3)
    kernels = {k: {"launches": v[0], "ms_per_step": v[1] / args.steps} for k, v in prof.items()}
    src_hash = kernel_source_hash()
    roofline = roofline_of(prof, st, args.steps, workload, src_hash)

    host_input = None
    if workload == "pangenome_merge" and not args.no_host_input:
        host_input = host_input_merges(b1, new_strings, 10)

    plain = None
    if workload == "uneven_merge" and args.plain_strings > 0:
        plain = plain_vs_batched(b1_strings, new_strings, args.chunk, args.plain_strings)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.host_threads()
        log(f"timing the oracle on {threads} host threads ...")
        cpu = cpu_baseline(args.cpu_sample, threads)
        log(f"oracle: {cpu['value']:.3g} suffixes/s ({cpu['sample']})")

    b1.close()
    torch.cuda.empty_cache()
    smem = None
    if not args.no_smem:
        rates = [0.25, 0.5, 0.8] if args.smem_haplotypes >= 320 else [0.5]
        smem = smem_bench(10_000_000, args.smem_haplotypes, 10_000, 200, rates, 10_000,
                          batched_only=args.smem_batched_only)
        if not args.no_cpu_baseline:
            smem["hapl"]["cpu_baseline"] = hapl_cpu_baseline()
        torch.cuda.empty_cache()
    incremental = None
    if workload == "pangenome_merge" and not args.no_incremental:
        ri = incremental_bench(args)
        incremental = {"value": ri["value"], "unit": ri["unit"], "config": ri["config"], "batches": ri["batches"],
                       "total_merge_s": ri["total_merge_s"], "peak_hbm_allocated_bytes": ri["peak_hbm_allocated_bytes"],
                       "device_free_min_bytes": ri["device_free_min_bytes"]}
        torch.cuda.empty_cache()

    out = {
        "metric": "BWT-merge suffixes inserted/s",
        "value": round(value, 1),
        "unit": "suffixes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "ms_per_step_without_timing_events": round(r["unprofiled_ms"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": workload, "genome_len": args.genome, "strings_indexed": b1_strings.n,
                   "strings_merged": new_strings.n, "both_strands": True, "n1": n1, "n2": n2,
                   "n_merged": n_out, "chunk_len": st["chunk_len"]},
        "roofline": roofline,
        "merge_roofline": merge_roofline(st, ms),
        "cpu_baseline": cpu,
        "smem": smem,
        "incremental": incremental,
        "plain_vs_batched": plain,
        "host_input": host_input,
        "tuning": {"merge": tuning, "smem": smem.get("tuning") if smem else None},
        "merge_stats": st,
        "kernels": kernels,
        "source_hash": src_hash,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
