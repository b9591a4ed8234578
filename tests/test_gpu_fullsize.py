"""Parity at the benchmark's full size: the pangenome merge (4 Mb genome,
32 + 32 haplotypes, both strands; 256 M new suffixes into a 256 M-symbol
index), called exactly as bench.py calls it.

The naive-sort oracle cannot sort 512 M suffixes in test time, so the merged
BWT is checked with the oracle's inverse-BWT verifier: LF walks from rows
0..m-1 must recover every input strand and the symbol counts must match,
which holds for exactly one string (the BWT). Counts are checked on a sample
of queries by brute force, and for all queries by strand symmetry.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2409_00613_amd import rb3

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def merged():
    say("case: full-size pangenome merge (4 Mb x 64 haplotypes)")
    w = synth.config_pangenome()
    alloc = rb3.TorchAllocator(0)
    b1 = rb3.rb3_build(w.b1.data, w.b1.lens, allocator=alloc)
    import torch
    idx = b1.clone()
    idx.merge(torch.from_numpy(w.new.data).cuda(), w.new.lens)
    st = idx.merge_stats()
    B = idx.export()
    n1, m1, _ = b1.info()
    b1.close()
    yield w, idx, B, st, n1, m1
    idx.close()


def test_fullsize_merge_inverse_bwt(merged):
    w, idx, B, st, n1, m1 = merged
    say("case: full-size merge, inverse-BWT verification on the host")
    allst = w.b1 + w.new
    codes, lens = oracle.expand(allst.data, allst.lens)
    assert B.shape[0] == int(lens.sum()) + lens.shape[0]
    assert st["n2"] == B.shape[0] - n1 and st["tie_doubling"] == 0
    assert oracle.verify(B, codes, lens) == 0
    # new sentinels land on rows m1 + j (Algorithm 1 starts every new chain at m1)
    nc, nl = oracle.expand(w.new.data, w.new.lens)
    ends = np.cumsum(nl) - 1
    assert np.array_equal(B[m1:m1 + nl.shape[0]], nc[ends])


def test_fullsize_counts(merged):
    w, idx, B, st, n1, m1 = merged
    say("case: full-size counts: brute force on a sample, strand symmetry on all")
    rng = np.random.default_rng(12)
    hap = w.new.get(3)
    qs = []
    for _ in range(400):
        L = int(rng.integers(12, 60))
        s = int(rng.integers(0, len(hap) - L))
        q = bytearray(hap[s:s + L])
        if rng.random() < 0.3:
            q[int(rng.integers(0, L))] = ord("ACGT"[int(rng.integers(0, 4))])
        qs.append(bytes(q))
    Q = synth.pack(qs)
    lo, hi = idx.count(Q.data, Q.lens)
    comp = bytes.maketrans(b"ACGT", b"TGCA")
    R = synth.pack([q.translate(comp)[::-1] for q in qs])
    lo2, hi2 = idx.count(R.data, R.lens)
    assert np.array_equal(hi - lo, hi2 - lo2)
    assert (hi > lo).sum() > 200
    allst = w.b1 + w.new
    codes, lens = oracle.expand(allst.data, allst.lens)
    sample = [0, 1, 2, 3, 4]
    S = synth.pack([qs[i] for i in sample])
    qc, ql = oracle.encode(S.data, S.lens)
    olo, ohi = oracle.count(codes, lens, qc, ql)
    assert np.array_equal(lo[sample], olo) and np.array_equal(hi[sample], ohi)
