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


def algorithmic_bytes(kernel: str, st: dict, steps: int) -> float | None:
    """Bytes the method must move in all launches of one kernel over the timed
    steps (per-unit figures times units, the units taken from the merge's own
    counters)."""
    n1, n2, m2 = st["n1"], st["n2"], st["m2"]
    per_step = {
        # one random 64-byte block per rank step, plus the symbol read and the
        # 8-byte key written per new suffix
        "chain": st["chain_steps"] * BLOCK_BYTES + (n2 - m2) * 1 + n2 * 8,
        "chain_fixup": st["fixup_steps"] * (BLOCK_BYTES + 1 + 8),
        # per pass: key 8 B read for the histogram
        "sort_hist": n2 * 8 * max(1, -(-st["sort_bits"] // 8)),
        # per pass: key + value read and written (the first pass has no value to read)
        "sort_scatter": n2 * 24 * max(1, -(-st["sort_bits"] // 8)) - n2 * 4,
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
            "sample": f"naive-sort BWT of the merged list with every haplotype cut to its first "
                      f"{sample_len} bases ({int(lens.sum()) + lens.shape[0]} suffixes, {n2} of them new); "
                      f"{dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--genome", type=int, default=4_000_000, help="base genome length")
    ap.add_argument("--chunk", type=int, default=0, help="LF-chain chunk length (0 = library default)")
    ap.add_argument("--cpu-sample", type=int, default=40_000,
                    help="haplotype prefix length for the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    workload = "pangenome_merge"
    t = time.perf_counter()
    w = synth.config_pangenome(genome_len=args.genome)
    log(f"generated {w.b1.n}+{w.new.n} haplotypes of ~{args.genome} bases in {time.perf_counter() - t:.1f} s")

    alloc = rb3.TorchAllocator(0)
    t = time.perf_counter()
    b1 = rb3.rb3_build(w.b1.data, w.b1.lens, allocator=alloc, chunk_len=args.chunk)
    torch.cuda.synchronize()
    n1, m1, _ = b1.info()
    log(f"built existing index: n1={n1} m1={m1} in {time.perf_counter() - t:.1f} s")
    new_dev = torch.from_numpy(w.new.data).cuda()
    new_lens = w.new.lens.copy()
    torch.cuda.synchronize()

    def step():
        idx = b1.clone()
        idx.merge(new_dev, new_lens)
        return idx

    for i in range(args.warmup):
        step().close()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    rb3.rb3_prof_reset()
    rb3.rb3_prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for i in range(args.steps):
        if last is not None:
            last.close()
        last = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rb3.rb3_prof_enable(False)
    prof = rb3.rb3_prof_read()
    st = last.merge_stats()
    n_out, m_out, _ = last.info()
    last.close()
    log(f"timed {args.steps} steps in {t1 - t0:.3f} s")

    ms = (t1 - t0) / args.steps * 1e3
    n2 = st["n2"]
    value = n2 / (ms / 1e3)
    kernels = {k: {"launches": v[0], "ms_per_step": v[1] / args.steps} for k, v in prof.items()}
    for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        log(f"  {k:24s} launches={v[0]:6d}  ms/step={v[1] / args.steps:9.3f}")
    dom = max(prof.items(), key=lambda kv: kv[1][1])[0]
    dom_ms_total = prof[dom][1]
    launches = prof[dom][0]
    ab = algorithmic_bytes(dom, st, args.steps)
    src_hash = kernel_source_hash()
    roofline = None
    if ab is not None and dom_ms_total > 0:
        achieved = ab / (dom_ms_total / 1e3) / 1e9
        traffic = read_traffic(dom, workload, src_hash)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic, "algorithmic_bytes_per_launch": ab / launches,
                    "avg_launch_ms": dom_ms_total / launches}

    cpu = None
    if not args.no_cpu_baseline:
        threads = max(1, min(16, os.cpu_count() or 1))
        log(f"timing the oracle on {threads} host threads ...")
        cpu = cpu_baseline(args.cpu_sample, threads)
        log(f"oracle: {cpu['value']:.3g} suffixes/s ({cpu['sample']})")

    out = {
        "metric": "BWT-merge suffixes inserted/s",
        "value": round(value, 1),
        "unit": "suffixes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": workload, "genome_len": args.genome, "haplotypes_indexed": w.b1.n,
                   "haplotypes_merged": w.new.n, "both_strands": True, "n1": n1, "n2": n2,
                   "n_merged": n_out, "chunk_len": st["chunk_len"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "merge_stats": st,
        "kernels": kernels,
        "source_hash": src_hash,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
