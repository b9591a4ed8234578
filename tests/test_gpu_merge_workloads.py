"""The batched-uneven and large-incremental merge workloads.

Batched uneven: thousands of strings of log-normal length (plus two long
chromosome-like ones) merged into the pangenome index in one call. The plain
form (one LF-chain launch per string) must give the identical BWT, and the
result must pass the oracle's inverse-BWT check. At full size (0.79 G new
suffixes into 256 M) the check is exact by the inverse-BWT argument: LF walks
from rows 0..m-1 recover every string only for the true BWT.

Large incremental: haplotypes of a genome with segmental duplications and
inversions, merged batch by batch (the first batch is a build into an empty
index). The bytes must not depend on how the haplotypes are split into
batches, and the final index must pass the inverse-BWT check. The full-size
run (100 haplotypes of 100 Mb, a 20 G-symbol index, positions beyond 2^32)
takes several minutes of host time and runs only when RB3_FULL_INCREMENTAL=1.
"""
import os
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2409_00613_amd import rb3

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def _expand(s):
    return oracle.expand(s.data, s.lens)


def _check_sentinel_rows(B, m1, new):
    # the sentinels of the new strands land on rows m1 .. m1 + m2 - 1
    nc, nl = _expand(new)
    ends = np.cumsum(nl) - 1
    assert np.array_equal(B[m1:m1 + nl.shape[0]], nc[ends])


def test_uneven_reduced_plain_equals_batched():
    say("case: uneven merge (reduced), plain one-launch-per-string form vs batched")
    u = synth.config_uneven(genome_len=300_000, n_b1=8, n_src=16, n_contigs=300, median=2000.0,
                            len_lo=50, len_hi=100_000, chrom_len=200_000, n_chrom=2)
    out = {}
    for per_string in (False, True):
        idx = rb3.rb3_build(u.b1.data, u.b1.lens, chunk_len=512, launch_per_string=per_string)
        n1, m1, _ = idx.info()
        idx.merge(u.new.data, u.new.lens)
        out[per_string] = idx.export()
        idx.close()
    assert np.array_equal(out[False], out[True])
    allst = u.b1 + u.new
    codes, lens = _expand(allst)
    assert oracle.verify(out[False], codes, lens) == 0
    _check_sentinel_rows(out[False], m1, u.new)


def test_uneven_full_size_verifies():
    say("case: uneven merge at full size (10,000 contigs + 2 chromosomes into 32 haplotypes)")
    u = synth.config_uneven()
    alloc = rb3.TorchAllocator(0)
    import torch
    idx = rb3.rb3_build(u.b1.data, u.b1.lens, allocator=alloc)
    n1, m1, _ = idx.info()
    idx.merge(torch.from_numpy(u.new.data).cuda(), u.new.lens)
    st = idx.merge_stats()
    B = idx.export()
    idx.close()
    say(f"  merged n2={st['n2']} new suffixes into n1={n1}; verifying on the host")
    assert st["m2"] == 2 * u.new.n and st["n2"] == 2 * (u.new.total + u.new.n)
    allst = u.b1 + u.new
    codes, lens = _expand(allst)
    assert oracle.verify(B, codes, lens) == 0
    _check_sentinel_rows(B, m1, u.new)


def _incremental(inc, sizes, alloc=None):
    idx = None
    first = 0
    for k in sizes:
        batch = inc.batch(first, k)
        first += k
        if idx is None:
            idx = rb3.rb3_build(batch.data, batch.lens, allocator=alloc)
        else:
            idx.merge(batch.data, batch.lens)
    return idx


def test_incremental_reduced_split_invariance():
    say("case: incremental merges (reduced): 5x2, 2x5 and 1x10 haplotypes give identical bytes")
    inc = synth.config_incremental(genome_len=600_000, n_hap=10, dup_frac=0.02, dup_lo=1000,
                                   dup_hi=20_000)
    outs = []
    for sizes in ([2] * 5, [5, 5], [10], [1, 3, 6]):
        idx = _incremental(inc, sizes)
        outs.append(idx.export())
        idx.close()
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)
    codes, lens = _expand(inc.batch(0, 10))
    assert oracle.verify(outs[0], codes, lens) == 0


@pytest.mark.skipif(os.environ.get("RB3_FULL_INCREMENTAL") != "1",
                    reason="full-size incremental build: several minutes of host time; "
                           "set RB3_FULL_INCREMENTAL=1")
def test_incremental_full_size_verifies():
    say("case: incremental build at full size (100 haplotypes of 100 Mb in 10 batches)")
    import torch
    inc = synth.config_incremental()
    alloc = rb3.TorchAllocator(0)
    idx = None
    codes_parts, lens_parts = [], []
    for b in range(10):
        t = time.time()
        batch = inc.batch(10 * b, 10)
        c_, l_ = _expand(batch)
        codes_parts.append(c_)
        lens_parts.append(l_)
        bdev = torch.from_numpy(batch.data).cuda()
        if idx is None:
            idx = rb3.rb3_build(bdev, batch.lens, allocator=alloc)
        else:
            idx.merge(bdev, batch.lens)
        torch.cuda.synchronize()
        del bdev, batch
        n, m, _ = idx.info()
        say(f"  batch {b}: n={n} m={m} ({time.time() - t:.1f} s with generation)")
    t = time.time()
    B = idx.export()
    idx.close()
    codes = np.concatenate(codes_parts)
    del codes_parts
    lens = np.concatenate(lens_parts)
    say(f"  exported {B.shape[0]} symbols in {time.time() - t:.1f} s")
    assert B.shape[0] > (1 << 32)
    t = time.time()
    v = oracle.Verifier(B, codes, lens)
    assert v.status == 0
    say(f"  symbol counts match; occurrence table built in {time.time() - t:.1f} s")
    m = lens.shape[0]
    for j0 in range(0, m, 16):
        t = time.time()
        r = v.walk(j0, min(m, j0 + 16), nthreads=16)
        say(f"  strings {j0}..{min(m, j0 + 16) - 1} walked in {time.time() - t:.1f} s")
        assert r == 0, f"string {r - 1} not recovered"
    v.close()
