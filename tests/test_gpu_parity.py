"""GPU parity: the HIP library through its C ABI against the CPU oracle.

Every result is exact integer data, so parity is element-by-element
equality (BWT codes, SA intervals, SMEM records).
"""
import random

import numpy as np
import pytest

import oracle
import synth
from paper_2409_00613_amd import rb3

pytestmark = pytest.mark.gpu

SYM = "$ACGTN"


def say(msg):
    print(msg, flush=True)


def _expand(strs):
    return oracle.expand(strs.data, strs.lens)


def _rand_lists(rnd, n_lists):
    """Small pangenome-like lists: mutated copies of a short base string."""
    out = []
    for _ in range(n_lists):
        base = "".join(rnd.choice("ACGT") for _ in range(rnd.randint(5, 60)))

        def hap():
            return "".join(c if rnd.random() > 0.06 else rnd.choice("ACGT") for c in base)

        old = [hap() for _ in range(rnd.randint(1, 4))]
        new = [hap() if rnd.random() < 0.8 else "".join(rnd.choice("ACGTN") for _ in range(rnd.randint(1, 9)))
               for _ in range(rnd.randint(1, 4))]
        if rnd.random() < 0.15:
            new.append(old[0])  # exact duplicate of an indexed string
        out.append((synth.pack([s.encode() for s in old]), synth.pack([s.encode() for s in new])))
    return out


@pytest.fixture(scope="module")
def tiny():
    return synth.config_tiny()


def _codes_with_strands(rng, n, m):
    """n random codes 1..5 with exactly m sentinels, and m strand lengths >= 1
    summing to n - m."""
    codes = rng.integers(1, 6, n).astype(np.uint8)
    codes[rng.choice(n, m, replace=False)] = 0
    cuts = np.sort(rng.choice(np.arange(1, n - m), m - 1, replace=False)) if m > 1 else np.zeros(0, np.int64)
    lens = np.diff(np.concatenate([[0], cuts, [n - m]])).astype(np.int64)
    assert lens.min() >= 1 and int(lens.sum()) + m == n
    return codes, lens


def test_import_export_roundtrip():
    say("case: import/export round trip")
    rng = np.random.default_rng(5)
    for n, m in ((2, 1), (3, 1), (127, 2), (128, 3), (129, 64), (5000, 7), (300_001, 1000)):
        codes, lens = _codes_with_strands(rng, n, m)
        idx = rb3.rb3_import(codes, lens)
        assert np.array_equal(idx.export(), codes)
        nn, mm, C = idx.info()
        assert nn == n and mm == m
        cnt = np.bincount(codes, minlength=6)
        assert C == [int(x) for x in np.concatenate([[0], np.cumsum(cnt)[:-1]])]
        idx.close()


def test_import_rejects_failed_count_checks():
    say("case: import rejects bad codes and failed symbol-count checks")
    cases = [
        (np.array([1, 2, 7, 0], np.uint8), [3]),   # code 7
        (np.array([1, 2, 3], np.uint8), [2]),      # no sentinel, n != sum(L + 1)
        (np.array([1, 2, 3, 4], np.uint8), [3]),   # n = sum(L + 1) but no sentinel
        (np.array([0, 2, 0, 4], np.uint8), [3]),   # two sentinels for one strand
        (np.array([1, 0, 3, 4], np.uint8), [1, 1]),  # n != sum(L + 1)
        (np.array([1, 0, 0, 4], np.uint8), [2, 0]),  # an empty strand
    ]
    for codes, lens in cases:
        with pytest.raises(rb3.RB3Error) as e:
            rb3.rb3_import(codes, lens)
        assert e.value.code == rb3.RB3_EINVAL, (codes, lens)


def test_count_on_imported_oracle_bwt(tiny):
    say("case: count on an imported oracle BWT (tiny config)")
    allst = tiny.b1 + tiny.new
    codes, lens = _expand(allst)
    B = oracle.bwt(codes, lens)
    idx = rb3.rb3_import(B, lens)
    qc, ql = oracle.encode(tiny.queries.data, tiny.queries.lens)
    lo, hi = idx.count(tiny.queries.data, tiny.queries.lens)
    olo, ohi = oracle.count(codes, lens, qc, ql)
    assert np.array_equal(lo, olo) and np.array_equal(hi, ohi)
    assert (hi > lo).sum() > 100  # the workload has real hits
    idx.close()


def test_build_tiny_equals_oracle(tiny):
    say("case: build of the tiny config's first half")
    idx = rb3.rb3_build(tiny.b1.data, tiny.b1.lens)
    codes, lens = _expand(tiny.b1)
    assert np.array_equal(idx.export(), oracle.bwt(codes, lens))
    idx.close()


@pytest.mark.parametrize("chunk_len", [0, 97])
def test_merge_tiny_equals_oracle(tiny, chunk_len):
    say(f"case: tiny merge, chunk_len={chunk_len}")
    idx = rb3.rb3_build(tiny.b1.data, tiny.b1.lens, chunk_len=chunk_len)
    n1, m1, _ = idx.info()
    idx.merge(tiny.new.data, tiny.new.lens)
    got = idx.export()
    allst = tiny.b1 + tiny.new
    codes, lens = _expand(allst)
    want = oracle.bwt(codes, lens)
    assert np.array_equal(got, want)
    assert oracle.verify(got, codes, lens) == 0
    # Algorithm 1 starts every new sentinel at l = m1: new strand j sits on
    # row m1 + j, whose BWT symbol is the strand's last base
    _, nl = _expand(tiny.new)
    off = np.cumsum(lens)[m1 - 1:-1] if m1 else np.cumsum(lens)
    for j in range(nl.shape[0]):
        last = codes[int(off[j]) + int(nl[j]) - 1]
        assert got[m1 + j] == last
    st = idx.merge_stats()
    assert st["n2"] == got.shape[0] - n1
    idx.close()


def test_merge_random_small_lists():
    say("case: random small lists, tiny chunks")
    rnd = random.Random(41)
    for t, (old, new) in enumerate(_rand_lists(rnd, 60)):
        cl = rnd.choice([1, 2, 3, 5, 1000])
        idx = rb3.rb3_build(old.data, old.lens, chunk_len=cl)
        idx.merge(new.data, new.lens)
        codes, lens = _expand(old + new)
        assert np.array_equal(idx.export(), oracle.bwt(codes, lens)), (t, old.as_list(), new.as_list(), cl)
        idx.close()


def test_build_random_lists_equal_oracle():
    say("case: builds of random lists")
    rnd = random.Random(43)
    for t in range(40):
        strs = [("".join(rnd.choice("ACGTN" if rnd.random() < 0.2 else "ACGT")
                         for _ in range(rnd.randint(1, 50)))).encode() for _ in range(rnd.randint(1, 6))]
        if rnd.random() < 0.3:
            strs.append(strs[0])
        s = synth.pack(strs)
        for both in (True, False):
            idx = rb3.rb3_build(s.data, s.lens, both_strands=both)
            codes, lens = oracle.expand(s.data, s.lens, both=both)
            assert np.array_equal(idx.export(), oracle.bwt(codes, lens)), (t, both)
            idx.close()


@pytest.mark.parametrize("chunk_len", [1024, 40])
def test_merge_pangenome_small(chunk_len):
    """Haplotypes share long stretches with the index, so chain chunks
    converge late; with 40-position chunks whole runs of chunks stay
    unresolved after the chains, and one fix-up lane completes each run."""
    say(f"case: pangenome merge, 20 kb genome, 8 + 8 haplotypes, chunk_len={chunk_len}")
    w = synth.config_pangenome(genome_len=20_000, n_b1=8, n_new=8)
    idx = rb3.rb3_build(w.b1.data, w.b1.lens, chunk_len=chunk_len)
    idx.merge(w.new.data, w.new.lens)
    st = idx.merge_stats()
    codes, lens = _expand(w.b1 + w.new)
    got = idx.export()
    assert np.array_equal(got, oracle.bwt(codes, lens))
    assert st["tied_records"] > 0 and st["tie_groups"] > 0
    assert st["tie_work"] + st["tie_small_reads"] > 0
    if chunk_len == 40:
        assert st["fixup_steps"] > 0 and st["fixup_passes"] == 1 and st["fixup_run_max"] >= 2
    idx.close()


def test_fixup_segments_and_runs():
    """Unresolved ends longer than one 256-step segment of folded rank maps,
    and runs of several unresolved chunks: the fix-up's fold, run walk and
    segment replay against the oracle."""
    say("case: pangenome merge, 20 kb genome, 8 + 8 haplotypes, 700-position chunks")
    w = synth.config_pangenome(genome_len=20_000, n_b1=8, n_new=8)
    idx = rb3.rb3_build(w.b1.data, w.b1.lens, chunk_len=700)
    idx.merge(w.new.data, w.new.lens)
    st = idx.merge_stats()
    codes, lens = _expand(w.b1 + w.new)
    assert np.array_equal(idx.export(), oracle.bwt(codes, lens))
    # more segments than chunks: many unresolved ends span several segments
    assert st["fixup_segments"] > st["chunks"]
    assert st["fixup_passes"] == 1 and st["fixup_run_max"] >= 2
    idx.close()


def test_fixup_intervals_wider_than_64_rows():
    """An index holding 70 near-copies of one string: while a new copy's
    context matches more than 64 of them the chain interval spans more than
    64 rows, so the fix-up reads the index for those steps, then switches to
    the recorded row masks as copies drop out."""
    say("case: 70 near-copies of a 1000-base string in the index, 4 new copies merged")
    rnd = random.Random(21)
    base = [rnd.choice("ACGT") for _ in range(1000)]

    def mutated(k):
        s = list(base)
        for _ in range(k):
            i = rnd.randrange(len(s))
            s[i] = rnd.choice("ACGT".replace(s[i], ""))
        return "".join(s).encode()
    old = synth.pack([mutated(rnd.randint(0, 2)) for _ in range(70)])
    new = synth.pack([mutated(1) for _ in range(4)])
    idx = rb3.rb3_build(old.data, old.lens, chunk_len=300)
    idx.merge(new.data, new.lens)
    st = idx.merge_stats()
    codes, lens = _expand(old + new)
    assert np.array_equal(idx.export(), oracle.bwt(codes, lens))
    assert st["fixup_index_steps"] > 1000
    assert st["fixup_steps"] > st["fixup_index_steps"]
    idx.close()


def test_incremental_merges_equal_one_build():
    say("case: merge(build(X), Y, Z) == build(X ++ Y ++ Z)")
    w = synth.config_pangenome(genome_len=5_000, n_b1=6, n_new=6)
    allst = w.b1 + w.new
    idx = rb3.rb3_build(allst.slice(0, 2).data, allst.slice(0, 2).lens)
    for a, b in ((2, 5), (5, 6), (6, 12)):
        part = allst.slice(a, b)
        idx.merge(part.data, part.lens)
    one = rb3.rb3_build(allst.data, allst.lens)
    assert np.array_equal(idx.export(), one.export())
    codes, lens = _expand(allst)
    assert oracle.verify(idx.export(), codes, lens) == 0
    idx.close()
    one.close()


def test_merge_from_device_buffer(tiny):
    import torch
    say("case: merge with the batch already in device memory")
    idx = rb3.rb3_build(torch.from_numpy(tiny.b1.data).cuda(), tiny.b1.lens)
    idx.merge(torch.from_numpy(tiny.new.data).cuda(), tiny.new.lens)
    codes, lens = _expand(tiny.b1 + tiny.new)
    assert np.array_equal(idx.export(), oracle.bwt(codes, lens))
    idx.close()


def test_merge_with_torch_allocator(tiny):
    import torch
    say("case: torch caching allocator hooks")
    alloc = rb3.TorchAllocator(0)
    idx = rb3.rb3_build(tiny.b1.data, tiny.b1.lens, allocator=alloc)
    idx.merge(tiny.new.data, tiny.new.lens)
    codes, lens = _expand(tiny.b1 + tiny.new)
    assert np.array_equal(idx.export(), oracle.bwt(codes, lens))
    idx.close()
    torch.cuda.synchronize()


def test_failed_merge_leaves_index_unchanged(tiny):
    say("case: invalid input is rejected and the index is unchanged")
    idx = rb3.rb3_build(tiny.b1.data, tiny.b1.lens)
    before = idx.export()
    bad = tiny.new.data.copy()
    bad[100] = ord("X")
    with pytest.raises(rb3.RB3Error) as e:
        idx.merge(bad, tiny.new.lens)
    assert e.value.code == rb3.RB3_EINVAL
    with pytest.raises(rb3.RB3Error):
        idx.merge(tiny.new.data, np.array([0] * tiny.new.n))
    assert np.array_equal(idx.export(), before)
    idx.merge(tiny.new.data, tiny.new.lens)  # a retry succeeds
    codes, lens = _expand(tiny.b1 + tiny.new)
    assert np.array_equal(idx.export(), oracle.bwt(codes, lens))
    idx.close()


def test_count_edges(tiny):
    say("case: count edge cases")
    idx = rb3.rb3_build(tiny.b1.data, tiny.b1.lens)
    n, _, _ = idx.info()
    qs = synth.pack([b"", b"A", b"N", b"ACGTNNNN", tiny.b1.get(0)[:500], tiny.b1.get(3)])
    lo, hi = idx.count(qs.data, qs.lens)
    codes, lens = _expand(tiny.b1)
    qc, ql = oracle.encode(qs.data, qs.lens)
    olo, ohi = oracle.count(codes, lens, qc, ql)
    assert lo[0] == 0 and hi[0] == n
    assert np.array_equal(lo, olo) and np.array_equal(hi, ohi)
    assert hi[4] - lo[4] == 1 and hi[5] - lo[5] == 1
    idx.close()


@pytest.mark.parametrize("min_len,min_occ", [(1, 1), (5, 1), (11, 1), (31, 1), (8, 2)])
def test_smem_tiny(tiny, min_len, min_occ):
    say(f"case: SMEM on the tiny config, min_len={min_len} min_occ={min_occ}")
    allst = tiny.b1 + tiny.new
    idx = rb3.rb3_build(allst.data, allst.lens)
    q = tiny.queries.slice(0, 200)
    recs, off = idx.smem(q.data, q.lens, min_len, min_occ)
    codes, lens = _expand(allst)
    text = oracle.Text(codes, lens)
    qc, ql = oracle.encode(q.data, q.lens)
    qoff = np.concatenate([[0], np.cumsum(ql)])
    total = 0
    for i in range(q.n):
        exp = text.smem(qc[qoff[i]:qoff[i + 1]], min_len, min_occ)
        r = recs[off[i]:off[i + 1]]
        got = np.stack([r["start"], r["end"], r["occ"], r["k"], r["krc"]], 1) if len(r) else np.zeros((0, 5), np.int64)
        assert np.array_equal(got, exp), i
        assert (r["qid"] == i).all()
        total += len(r)
    assert total > 0
    idx.close()


def test_smem_pangenome_queries():
    say("case: SMEM of mutated haplotype excerpts on a small pangenome index")
    w = synth.config_serving(genome_len=30_000, n_index=6, n_unseen=3, n_queries=30, log_lo=2.0, log_hi=3.8)
    idx = rb3.rb3_build(w.index.data, w.index.lens)
    recs, off = idx.smem(w.queries.data, w.queries.lens, 31, 1)
    codes, lens = _expand(w.index)
    text = oracle.Text(codes, lens)
    qc, ql = oracle.encode(w.queries.data, w.queries.lens)
    qoff = np.concatenate([[0], np.cumsum(ql)])
    for i in range(w.queries.n):
        exp = text.smem(qc[qoff[i]:qoff[i + 1]], 31, 1)
        r = recs[off[i]:off[i + 1]]
        got = np.stack([r["start"], r["end"], r["occ"], r["k"], r["krc"]], 1) if len(r) else np.zeros((0, 5), np.int64)
        assert np.array_equal(got, exp), i
    idx.close()


def test_smem_small_capacity_reports_sizes(tiny):
    say("case: SMEM output capacity too small")
    allst = tiny.b1 + tiny.new
    idx = rb3.rb3_build(allst.data, allst.lens)
    q = tiny.queries.slice(0, 50)
    full, off = idx.smem(q.data, q.lens, 5, 1)
    small, off2 = idx.smem(q.data, q.lens, 5, 1, cap=3)  # retried internally after ENOSPC
    assert np.array_equal(off, off2) and np.array_equal(full, small)
    idx.close()


@pytest.mark.parametrize("copies,tail_len,muts", [(6, 300, 0), (40, 300, 0), (70, 300, 0), (70, 300, 2),
                                                  (200, 300, 2), (1000, 200, 3), (5000, 120, 2), (9000, 40, 0)])
def test_large_mixed_symbol_groups(copies, tail_len, muts):
    """Many new strings sharing a long tail after different first bases:
    one tied group per position of the shared part, with mixed BWT symbols
    right after the differing base. Up to ``muts`` substitutions per copy
    make the big groups split at many depths. The group sizes cover every
    tie kernel: a wave per group (up to 64 members), a workgroup per group
    (65..128, 129..256, 257..8192), and prefix doubling (more than 8192)."""
    say(f"case: {copies} strings with a shared {tail_len}-base tail, {muts} substitutions each")
    rnd = random.Random(copies * 7 + muts)
    tail = "".join(rnd.choice("ACGT") for _ in range(tail_len))
    strs = []
    for _ in range(copies):
        t = list(tail)
        for _ in range(rnd.randint(0, muts)):
            i = rnd.randrange(tail_len)
            t[i] = rnd.choice("ACGT")
        strs.append("".join(rnd.choice("ACGT") for _ in range(rnd.randint(1, 3))) + "".join(t))
    old = synth.pack([("".join(rnd.choice("ACGT") for _ in range(150)) + tail[:100]).encode()])
    new = synth.pack([s.encode() for s in strs])
    for start in ("empty", "index"):
        if start == "empty":
            idx = rb3.rb3_build(new.data, new.lens)
            codes, lens = _expand(new)
        else:
            idx = rb3.rb3_build(old.data, old.lens)
            idx.merge(new.data, new.lens)
            codes, lens = _expand(old + new)
        assert np.array_equal(idx.export(), oracle.bwt(codes, lens)), start
        st = idx.merge_stats()
        assert st["tie_groups"] > 0
        assert st["tie_doubling"] == (1 if st["max_group"] > 8192 else 0)
        idx.close()


def test_clone_outlives_source(tiny):
    say("case: a clone stays usable after its source is freed")
    src = rb3.rb3_build(tiny.b1.data, tiny.b1.lens)
    cp = src.clone()
    src.close()
    cp.merge(tiny.new.data, tiny.new.lens)
    lo, hi = cp.count(tiny.queries.data, tiny.queries.lens)
    codes, lens = _expand(tiny.b1 + tiny.new)
    assert np.array_equal(cp.export(), oracle.bwt(codes, lens))
    qc, ql = oracle.encode(tiny.queries.data, tiny.queries.lens)
    olo, ohi = oracle.count(codes, lens, qc, ql)
    assert np.array_equal(lo, olo) and np.array_equal(hi, ohi)
    cp.close()


@pytest.mark.parametrize("min_len,min_occ", [(31, 1), (51, 1), (19, 3)])
def test_smem_long_queries_across_segments(min_len, min_occ):
    """Queries of several kilobases are cut into segments inside the library;
    exact excerpts give one SMEM spanning every segment."""
    say(f"case: long SMEM queries, min_len={min_len} min_occ={min_occ}")
    w = synth.config_serving(genome_len=40_000, n_index=5, n_unseen=2, n_queries=12, log_lo=3.3, log_hi=4.3)
    hap = w.index.get(2)
    extra = synth.pack([hap[1000:9000], hap[20000:23100] + b"ACGTTGCA" + hap[23100:27000]])
    qs = w.queries + extra
    idx = rb3.rb3_build(w.index.data, w.index.lens)
    recs, off = idx.smem(qs.data, qs.lens, min_len, min_occ)
    codes, lens = _expand(w.index)
    text = oracle.Text(codes, lens)
    qc, ql = oracle.encode(qs.data, qs.lens)
    qoff = np.concatenate([[0], np.cumsum(ql)])
    for i in range(qs.n):
        exp = text.smem(qc[qoff[i]:qoff[i + 1]], min_len, min_occ)
        r = recs[off[i]:off[i + 1]]
        got = np.stack([r["start"], r["end"], r["occ"], r["k"], r["krc"]], 1) if len(r) else np.zeros((0, 5), np.int64)
        assert np.array_equal(got, exp), i
    # the exact 8 kb excerpt is one SMEM covering the whole query
    r = recs[off[qs.n - 2]:off[qs.n - 1]]
    if min_occ == 1:
        assert len(r) == 1 and r["start"][0] == 0 and r["end"][0] == 8000
    assert rb3.rb3_last_smem_stats()["extensions"] > 0
    idx.close()
