"""Edge cases of the merge and query paths: empty batches, many tiny
strings, lower-case and N symbols, queries shorter than the SMEM minimum,
and the batch-size limit (rejected before any memory is read)."""
import random

import numpy as np
import pytest

import oracle
import synth
from paper_2409_00613_amd import rb3

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def _bwt(strings, both=True):
    codes, lens = oracle.expand(strings.data, strings.lens, both=both)
    return oracle.bwt(codes, lens)


def test_empty_batch_is_a_no_op():
    say("case: merging an empty batch")
    s = synth.pack([b"ACGTACGGT", b"TTGCA"])
    idx = rb3.rb3_build(s.data, s.lens)
    before = idx.export()
    idx.merge(np.zeros(0, np.uint8), np.zeros(0, np.int64))
    assert np.array_equal(idx.export(), before)
    assert idx.info()[:2] == (before.shape[0], 4)
    idx.close()


def test_many_tiny_strings():
    """20,000 strands of 1-4 symbols: thousands of sentinels per tie group,
    every new suffix within a few symbols of its sentinel."""
    say("case: 10,000 strings of 1-4 bases, built in one call and merged in two halves")
    rnd = random.Random(5)
    strs = [("".join(rnd.choice("ACGT") for _ in range(rnd.randint(1, 4)))).encode() for _ in range(10_000)]
    s = synth.pack(strs)
    want = _bwt(s)
    idx = rb3.rb3_build(s.data, s.lens)
    assert np.array_equal(idx.export(), want)
    idx.close()
    a, b = s.slice(0, 4_000), s.slice(4_000, 10_000)
    idx = rb3.rb3_build(a.data, a.lens, chunk_len=2)
    idx.merge(b.data, b.lens)
    assert np.array_equal(idx.export(), want)
    idx.close()


def test_lower_case_and_n():
    say("case: lower-case input and N symbols")
    up = [b"ACGTNNACGT", b"NNNN", b"GATTACA", b"N"]
    low = [x.lower() for x in up]
    su, sl = synth.pack(up), synth.pack(low)
    idx = rb3.rb3_build(sl.data, sl.lens)
    assert np.array_equal(idx.export(), _bwt(su))
    q = synth.pack([b"nn", b"acgtn", b"ACGTN"])
    lo, hi = idx.count(q.data, q.lens)
    codes, lens = oracle.expand(su.data, su.lens)
    qc, ql = oracle.encode(q.data, q.lens)
    olo, ohi = oracle.count(codes, lens, qc, ql)
    assert np.array_equal(lo, olo) and np.array_equal(hi, ohi)
    assert lo[1] == lo[2] and hi[1] == hi[2]
    idx.close()


def test_unstranded_merge():
    say("case: single-strand lists (both_strands off)")
    rnd = random.Random(9)
    old = synth.pack([("".join(rnd.choice("ACGT") for _ in range(rnd.randint(5, 200)))).encode() for _ in range(30)])
    new = synth.pack([("".join(rnd.choice("ACGT") for _ in range(rnd.randint(5, 200)))).encode() for _ in range(30)])
    idx = rb3.rb3_build(old.data, old.lens, both_strands=False, chunk_len=16)
    idx.merge(new.data, new.lens)
    assert np.array_equal(idx.export(), _bwt(old + new, both=False))
    assert idx.info()[1] == 60
    idx.close()


def test_smem_short_and_exact_queries():
    say("case: SMEM queries shorter than, equal to and just above min_len")
    w = synth.config_tiny()
    allst = w.b1 + w.new
    idx = rb3.rb3_build(allst.data, allst.lens)
    src = allst.get(5)
    qs = [src[:10], src[100:131], src[200:232], b"", b"ACGT" * 10, src[300:400]]
    q = synth.pack(qs)
    codes, lens = oracle.expand(allst.data, allst.lens)
    text = oracle.Text(codes, lens)
    recs, off = idx.smem(q.data, q.lens, 31, 1)
    for i in range(len(qs)):
        qc, _ = oracle.encode(np.frombuffer(qs[i], np.uint8), np.array([len(qs[i])]))
        exp = text.smem(qc, 31, 1)
        r = recs[off[i]:off[i + 1]]
        got = np.stack([r["start"], r["end"], r["occ"], r["k"], r["krc"]], 1) if len(r) else np.zeros((0, 5))
        assert np.array_equal(got, exp), i
    assert off[1] == off[0]            # 10 bases < min_len: nothing
    assert off[2] - off[1] == 1        # exactly min_len, present: one SMEM [0, 31)
    assert recs[off[1]]["end"] - recs[off[1]]["start"] == 31
    idx.close()


def test_batch_limit_is_rejected_before_reading():
    """Lengths summing past the per-batch limit are refused from the lengths
    alone: the (tiny) buffer is never read."""
    say("case: batch-size limit")
    s = synth.pack([b"ACGT"])
    idx = rb3.rb3_build(s.data, s.lens)
    before = idx.export()
    huge = np.array([1 << 31, 1 << 31], np.int64)
    with pytest.raises(rb3.RB3Error) as e:
        idx.merge(np.zeros(8, np.uint8), huge)
    assert e.value.code == rb3.RB3_ELIMIT
    assert np.array_equal(idx.export(), before)
    idx.close()


def test_run_of_n_longer_than_65536_merges():
    """A 70,000-symbol run of N in a new string: its suffixes share the
    insertion rank and the key for up to 70,000 symbols, so one tie group of
    about 70,000 members goes through the prefix-doubling rounds."""
    say("case: a string with a 70,000-base run of N merged into a small index (inverse-BWT check)")
    g = np.random.default_rng(70000)
    acgt = np.frombuffer(b"ACGT", np.uint8)
    flank = [acgt[g.integers(0, 4, 1500)].tobytes() for _ in range(3)]
    old = synth.pack([flank[0] + flank[1], flank[2]])
    new = synth.pack([flank[1][:700] + b"N" * 70000 + flank[2][:900], acgt[g.integers(0, 4, 400)].tobytes()])
    idx = rb3.rb3_build(old.data, old.lens)
    idx.merge(new.data, new.lens)
    st = idx.merge_stats()
    assert st["tie_doubling"] == 1 and st["max_group"] >= 65536, st
    B = idx.export()
    allst = synth.pack([old.get(i) for i in range(old.n)] + [new.get(i) for i in range(new.n)])
    codes, lens = oracle.expand(allst.data, allst.lens)
    assert B.shape[0] == codes.shape[0] + lens.shape[0]
    assert oracle.verify(B, codes, lens) == 0
    idx.close()


def test_70000_identical_reads_merge():
    """70,000 copies of one 25-base read (and its reverse complement): tie
    groups of 70,000 members at every offset, ordered in the end by the
    strands' sentinels."""
    say("case: 70,000 identical 25-base reads merged into an index holding the read once")
    read = b"ACGTTGCAAGGCTTACCGATAGCAT"
    old = synth.pack([b"GGGTACCA" + read + b"TTTAC", b"CCATG"])
    new = synth.pack([read] * 70000)
    idx = rb3.rb3_build(old.data, old.lens)
    idx.merge(new.data, new.lens)
    st = idx.merge_stats()
    assert st["tie_doubling"] == 1 and st["max_group"] >= 65536, st
    allst = synth.pack([old.get(i) for i in range(old.n)] + [read] * 70000)
    assert np.array_equal(idx.export(), _bwt(allst))
    idx.close()
