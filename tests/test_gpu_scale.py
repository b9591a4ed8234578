"""Parity past one superblock and past 2^32 symbols, against the oracle's
suffix-sort-free checks (a naive sort of these texts does not fit test time).

* Reduced serving index: 32 haplotypes of a 1 Mb genome on both strands
  (64 M symbols, four 2^24-symbol superblocks), built by a build and three
  merges. The BWT is checked by the oracle's inverse-BWT walk. SMEMs of 240
  queries (log-uniform 100 bp - 20 kb, excerpts of unseen haplotypes with
  1% substitutions and 0.1% indels) at min_len 31 and min_occ 1 and 2, with
  query segments of 32, 553 (the length the batched serving benchmark uses)
  and 4096 positions, are compared record by record with the oracle's seeded
  scan; counts of SMEM strings and of short excerpts with the oracle's
  one-pass intervals; Locate1 of every SMEM interval must return a position
  whose text starts with the SMEM.
* Merge past 2^32 symbols: 22 haplotypes of the 100 Mb genome with
  segmental duplications (the large incremental build's genome), merged as
  8 + 7 + 7 haplotypes into a 4.4 G-symbol BWT; checked by the inverse-BWT
  walk of every strand.
* Full serving index: 320 haplotypes of a 10 Mb genome (6.4 G symbols),
  built by ten merges of 32 as the serving benchmark builds it, with the
  benchmark's 553-position segments; SMEMs of 200 queries stratified by
  length (50 per quarter of the log-length range) against the seeded scan;
  haplotype enumeration of 125 bp reads at bands 10 and 25 checked by the
  properties that hold at any size.
"""
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2409_00613_amd import rb3

pytestmark = pytest.mark.gpu

BENCH_SEGMENT = 553  # 145 Mb of queries over 262,144 segments


def say(msg):
    print(msg, flush=True)


def _haplotypes(base, seed, first, count):
    return synth.haplotypes(base, seed, range(first, first + count))


def _queries(sources, seed, n, log_lo, log_hi):
    qs = []
    for q in range(n):
        g = synth.rng(seed, synth.STREAM_QUERY + q)
        L = int(10 ** g.uniform(log_lo, log_hi))
        src = sources[int(g.integers(0, len(sources)))]
        L = max(1, min(L, src.shape[0]))
        st = int(g.integers(0, src.shape[0] - L + 1))
        qs.append(synth.mutate(src[st:st + L], 0.01, 0.001, g))
    return qs


def _build(batches, **kw):
    idx = None
    for b in batches:
        if idx is None:
            idx = rb3.rb3_build(b.data, b.lens, **kw)
        else:
            idx.merge(b.data, b.lens)
    return idx


def _smem_rows(recs, off, i):
    r = recs[off[i]:off[i + 1]]
    if not len(r):
        return np.zeros((0, 5), np.int64)
    return np.stack([r["start"], r["end"], r["occ"], r["k"], r["krc"]], 1)


def _compare_smems(idx, Q, qc, ql, codes, lens, min_len, min_occ, label):
    t = time.time()
    want, woff = oracle.smem_scan(codes, lens, qc, ql, min_len, min_occ)
    t_or = time.time() - t
    recs, off = idx.smem(Q.data, Q.lens, min_len, min_occ)
    for i in range(Q.n):
        got = _smem_rows(recs, off, i)
        exp = want[woff[i]:woff[i + 1]]
        assert np.array_equal(got, exp), f"{label}: SMEMs of query {i} differ (len {Q.lens[i]})"
    say(f"  {label}: {len(want)} SMEMs equal (oracle scan {t_or:.1f} s)")
    return want, woff


@pytest.fixture(scope="module")
def reduced():
    say("case: reduced serving index (32 haplotypes x 1 Mb, 64 M symbols), build + 3 merges, samples every 32")
    seed = synth.SEED + 14
    base = synth.random_genome(1_000_000, synth.rng(seed, synth.STREAM_BASE))
    haps = _haplotypes(base, seed, 0, 32)
    unseen = _haplotypes(base, seed, 32, 8)
    batches = [synth.pack(haps[8 * b:8 * b + 8]) for b in range(4)]
    idx = _build(batches, ssa_rate=32)
    allst = synth.pack(haps)
    codes, lens = oracle.expand(allst.data, allst.lens)
    qs = _queries(unseen, seed, 240, 2.0, np.log10(20_000))
    Q = synth.pack(qs)
    qc, ql = oracle.encode(Q.data, Q.lens)
    yield idx, codes, lens, Q, qc, ql
    idx.close()


def test_reduced_index_inverse_bwt(reduced):
    idx, codes, lens, *_ = reduced
    say("case: reduced serving index, inverse-BWT check")
    B = idx.export()
    n, m, _ = idx.info()
    assert n > 4 * (1 << 24) - (1 << 22) and n == B.shape[0] and m == 64
    assert oracle.verify(B, codes, lens) == 0


@pytest.mark.parametrize("segment", [32, BENCH_SEGMENT, 4096])
def test_reduced_index_smem(reduced, segment):
    idx, codes, lens, Q, qc, ql = reduced
    say(f"case: reduced serving index, SMEMs with {segment}-position segments vs the seeded scan")
    B = idx.export()
    seg = rb3.rb3_import(B, lens, smem_segment=segment)
    try:
        for min_occ in (1, 2):
            _compare_smems(seg, Q, qc, ql, codes, lens, 31, min_occ, f"segment {segment}, min_occ {min_occ}")
    finally:
        seg.close()


def test_reduced_index_counts_and_locate1(reduced):
    idx, codes, lens, Q, qc, ql = reduced
    say("case: reduced serving index, counts of SMEM strings and excerpts; Locate1 of SMEM intervals")
    want, woff = oracle.smem_scan(codes, lens, qc, ql, 31, 1)
    qo = np.concatenate([[0], np.cumsum(ql)])
    pats = []
    for i in range(Q.n):
        for a, b, occ, k, krc in want[woff[i]:woff[i + 1]]:
            pats.append(Q.data[qo[i] + a:qo[i] + b])
    g = np.random.default_rng(5)
    for _ in range(3000):  # short excerpts of the queries (with their errors)
        i = int(g.integers(0, Q.n))
        L = int(g.integers(12, 120))
        if ql[i] < L:
            continue
        s = int(g.integers(0, ql[i] - L + 1))
        pats.append(Q.data[qo[i] + s:qo[i] + s + L])
    P = synth.pack(pats)
    pc, pl = oracle.encode(P.data, P.lens)
    olo, ohi = oracle.scan_intervals(codes, lens, pc, pl)
    lo, hi = idx.count(P.data, P.lens)
    assert np.array_equal(lo, olo) and np.array_equal(hi, ohi)
    assert (hi - lo > 0).sum() > len(pats) // 2
    # Locate1 of every SMEM interval [k, k + occ): the located suffix starts with the SMEM
    nsm = len(want)
    st, off = idx.locate1(want[:, 3], want[:, 3] + want[:, 2])
    starts = np.concatenate([[0], np.cumsum(lens)])
    pstart = np.concatenate([[0], np.cumsum(pl[:nsm])])
    for s in range(nsm):
        L = int(pl[s])
        j, o = int(st[s]), int(off[s])
        assert 0 <= j < lens.shape[0] and 0 <= o and o + L <= lens[j], f"Locate1 of SMEM {s} out of range"
        a = starts[j] + o
        assert np.array_equal(codes[a:a + L], pc[pstart[s]:pstart[s] + L]), f"Locate1 of SMEM {s}"


def test_reduced_index_run_length_form(reduced):
    idx, codes, lens, Q, qc, ql = reduced
    say("case: reduced serving index in the run-length static form: image, counts, SMEMs vs the seeded scan")
    B = idx.export()
    r = rb3.rb3_rle_build(idx)
    info = r.info()
    blocks, segs, row = r.image()
    want = oracle.rle_encode(B, info["row_shift"])
    assert np.array_equal(blocks, want.blocks) and np.array_equal(segs, want.seg) and np.array_equal(row, want.row)
    say(f"  {info['n']} symbols, {info['runs']} runs, {info['blocks']} blocks, {info['bytes'] / info['n']:.3f} B/symbol")
    g = np.random.default_rng(17)
    pos = np.concatenate([g.integers(0, B.shape[0] + 1, 20000), np.arange(0, B.shape[0], 1 << 20)])
    cum = [np.concatenate([[0], np.cumsum(B == c)]) for c in range(6)]
    assert np.array_equal(oracle.rle_rank(want, pos), np.stack([cum[c][pos] for c in range(6)], 1))
    # SMEMs on the run-length form against the oracle's seeded scan
    _compare_smems(r, Q, qc, ql, codes, lens, 31, 1, "run-length form, min_occ 1")
    lo, hi = r.count(Q.data, Q.lens)
    plo, phi = idx.count(Q.data, Q.lens)
    assert np.array_equal(lo, plo) and np.array_equal(hi, phi)
    # haplotype enumeration of 125 bp windows of the queries: the same
    # records on both forms, past the first superblock
    qo = np.concatenate([[0], np.cumsum(ql)])
    wins = [bytes(Q.data[qo[i]:qo[i] + 125]) for i in range(Q.n) if ql[i] >= 125]
    W = synth.pack(wins)
    for band in (10, 25):
        hr, ho = r.hapl(W.data, W.lens, band=band)
        hp, hpo = idx.hapl(W.data, W.lens, band=band)
        assert np.array_equal(ho, hpo) and np.array_equal(hr, hp), band
        assert hr.shape[0] > 0 and (hr["k"] > (1 << 24)).any()
    r.close()


def test_merge_past_2_32_symbols():
    say("case: merge past 2^32 symbols: 22 haplotypes of the 100 Mb genome as 8 + 7 + 7")
    import torch
    inc = synth.config_incremental()
    alloc = rb3.TorchAllocator(0)
    idx = None
    codes_parts, lens_parts = [], []
    t0 = time.time()
    for first, count in ((0, 8), (8, 7), (15, 7)):
        batch = inc.batch(first, count)
        c_, l_ = oracle.expand(batch.data, batch.lens)
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
        say(f"  after haplotypes {first}..{first + count - 1}: n={n} m={m} ({time.time() - t0:.1f} s)")
    n, m, C = idx.info()
    assert n > (1 << 32) and m == 44
    B = idx.export()
    idx.close()
    codes = np.concatenate(codes_parts)
    del codes_parts
    lens = np.concatenate(lens_parts)
    t = time.time()
    v = oracle.Verifier(B, codes, lens)
    assert v.status == 0
    bad = v.walk(0, lens.shape[0])
    say(f"  inverse-BWT check of {n} symbols: {time.time() - t:.1f} s")
    assert bad == 0
    cnt = np.bincount(B, minlength=6)
    assert C == [int(x) for x in np.concatenate([[0], np.cumsum(cnt)[:-1]])]
    v.close()


def _hapl_properties(idx, qs, n, band, exact):
    """Haplotype enumeration at any size: valid bi-intervals, scores in
    (0, |P|] by decreasing value, no result inside an earlier one (either
    interval), and an exact read's first result its own bi-interval with the
    full score."""
    P = synth.pack(qs)
    recs, off = idx.hapl(P.data, P.lens, band=band)
    assert off.shape[0] == len(qs) + 1 and np.all(np.diff(off) <= band)
    for i, q in enumerate(qs):
        got = recs[off[i]:off[i + 1]]
        assert np.all(got["qid"] == i)
        assert np.all(got["s"] > 0) and np.all(got["k"] + got["s"] <= n) and np.all(got["krc"] + got["s"] <= n)
        sc = got["score"].astype(np.int64)
        assert np.all(sc > 0) and np.all(sc <= len(q)) and np.all(np.diff(sc) <= 0)
        for a in range(got.shape[0]):
            for b in range(a):
                x, y = got[a], got[b]
                assert not (y["k"] <= x["k"] and x["k"] + x["s"] <= y["k"] + y["s"])
                assert not (y["krc"] <= x["krc"] and x["krc"] + x["s"] <= y["krc"] + y["s"])
    if exact:
        lo, hi = idx.count(P.data, P.lens)
        comp = bytes.maketrans(b"ACGT", b"TGCA")
        R = synth.pack([q.translate(comp)[::-1] for q in qs])
        rlo, _ = idx.count(R.data, R.lens)
        for i, q in enumerate(qs):
            top = recs[off[i]]
            assert (int(top["k"]), int(top["krc"]), int(top["s"]), int(top["score"])) == \
                (int(lo[i]), int(rlo[i]), int(hi[i] - lo[i]), len(q)), i


def test_full_serving_index_smem_stratified():
    say("case: full serving index (320 haplotypes x 10 Mb, 6.4 G symbols), 200 stratified queries vs the seeded scan; "
        "haplotype enumeration properties")
    import torch
    seed = synth.SEED + 4  # the serving workload's seed
    t0 = time.time()
    base = synth.random_genome(10_000_000, synth.rng(seed, synth.STREAM_BASE))
    haps = _haplotypes(base, seed, 0, 320)
    unseen = _haplotypes(base, seed, 320, 64)
    say(f"  haplotypes generated ({time.time() - t0:.1f} s)")
    alloc = rb3.TorchAllocator(0)
    idx = None
    for b in range(10):
        batch = synth.pack(haps[32 * b:32 * b + 32])
        bdev = torch.from_numpy(batch.data).cuda()
        if idx is None:
            idx = rb3.rb3_build(bdev, batch.lens, allocator=alloc, smem_segment=BENCH_SEGMENT)
        else:
            idx.merge(bdev, batch.lens)
        torch.cuda.synchronize()
        del bdev
    n, m, _ = idx.info()
    assert n > 6_000_000_000 and m == 640
    say(f"  index built ({time.time() - t0:.1f} s)")
    # the serving workload's queries (same recipe and streams), 50 from each
    # quarter of the log-length range 2 .. 5
    pool = _queries(unseen, seed, 2000, 2.0, 5.0)
    loglen = np.log10(np.array([len(q) for q in pool]))
    pick = []
    for k in range(4):
        inq = [i for i in range(len(pool)) if 2.0 + 0.75 * k <= loglen[i] < 2.0 + 0.75 * (k + 1)]
        pick += inq[:50]
    assert len(pick) == 200
    Q = synth.pack([pool[i] for i in pick])
    qc, ql = oracle.encode(Q.data, Q.lens)
    # haplotype enumeration at full size, in the bench's configuration: 125 bp
    # windows of indexed haplotypes (exact) and of the queries (1% / 0.1%)
    g = np.random.default_rng(29)
    exact = []
    for _ in range(1000):
        h = haps[int(g.integers(0, len(haps)))]
        a = int(g.integers(0, len(h) - 125))
        exact.append(bytes(h[a:a + 125]))
    longq = [q for q in pool if len(q) >= 125]
    mutated = []
    for _ in range(1000):
        q = longq[int(g.integers(0, len(longq)))]
        a = int(g.integers(0, len(q) - 124))
        mutated.append(bytes(q[a:a + 125]))
    for band in (10, 25):
        _hapl_properties(idx, exact, n, band, exact=True)
        _hapl_properties(idx, mutated, n, band, exact=False)
    say("  haplotype enumeration properties hold at bands 10 and 25")
    allst = synth.pack(haps)
    del haps
    codes, lens = oracle.expand(allst.data, allst.lens)
    del allst
    want, _ = _compare_smems(idx, Q, qc, ql, codes, lens, 31, 1, "full serving index, min_occ 1")
    assert len(want) > 1000 and want[:, 3].max() > (1 << 32)
    idx.close()
