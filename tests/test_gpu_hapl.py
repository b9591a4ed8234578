"""GPU parity of local haplotype enumeration (Sec. 2.7-2.8, Algorithm 5 and
the bi-interval filter) through the C ABI: every result (bi-interval and
score, in order) against the oracle on small pangenome indices, with and
without a band, on both index forms; at larger sizes the properties that
hold at any size; and the argument checks."""
import numpy as np
import pytest

import oracle
import synth
from paper_2409_00613_amd import rb3

pytestmark = pytest.mark.gpu

ENC = np.zeros(256, np.uint8)
for _i, _c in enumerate(b"ACGTN"):
    ENC[_c] = _i + 1
    ENC[_c | 0x20] = _i + 1


def say(msg):
    print(msg, flush=True)


def _reads(w, k, lmin, lmax, sub=0.02, indel=0.002, stream=0):
    qs = []
    for j in range(k):
        g = synth.rng(synth.SEED, synth.STREAM_QUERY + stream + j)
        src = w.new.get(j % w.new.n)
        L = int(g.integers(lmin, lmax + 1))
        s = int(g.integers(0, len(src) - L))
        qs.append(bytes(synth.mutate(np.frombuffer(src[s:s + L], np.uint8), sub, indel, g)))
    return qs


def _compare(text, qs, recs, off, **kw):
    assert off.shape[0] == len(qs) + 1
    for i, q in enumerate(qs):
        want = text.hapl(ENC[np.frombuffer(q, np.uint8)], **kw)
        got = recs[off[i]:off[i + 1]]
        assert [tuple(int(v) for v in x) for x in want] == \
            [(int(a["k"]), int(a["krc"]), int(a["s"]), int(a["score"])) for a in got], (i, q)
        assert np.all(got["qid"] == i)


@pytest.fixture(scope="module")
def small():
    w = synth.config_pangenome(genome_len=3000, n_b1=6, n_new=2)
    codes, lens = oracle.expand(w.b1.data, w.b1.lens)
    idx = rb3.rb3_build(w.b1.data, w.b1.lens)
    text = oracle.Text(codes, lens)
    yield w, idx, text, codes
    idx.close()


@pytest.mark.parametrize("dev", [False, True])
@pytest.mark.parametrize("band", [40, 25, 10, 1])
def test_hapl_matches_oracle_banded(small, band, dev):
    say(f"case: haplotype enumeration, 3 kb x 6 haplotypes, reads 8-100 bp, band {band}, device tables {dev}")
    w, idx, text, codes = small
    qs = _reads(w, 120, 8, 100)
    # exact substrings of indexed haplotypes, reads with N, the empty query
    g = np.random.default_rng(band)
    letters = np.frombuffer(b"$ACGTN", np.uint8)
    for _ in range(20):
        L = int(g.integers(1, 60))
        s = int(g.integers(0, 3000 - L))
        qs.append(w.b1.get(int(g.integers(0, w.b1.n)))[s:s + L])
    qs.append(b"")
    qs.append(b"N" * 5)
    q = bytearray(w.new.get(1)[100:160])
    q[30] = ord("N")
    qs.append(bytes(q))
    qs.append(letters[codes[500:540]].tobytes())
    qs.append(b"ACGT")  # an odd number of queries: the last wavefront of two holds one
    assert len(qs) % 2 == 1
    P = synth.pack(qs)
    recs, off = idx.hapl(P.data, P.lens, band=band, device_tables=dev)
    _compare(text, qs, recs, off, band=band)
    st = rb3.rb3_last_hapl_stats()
    assert st["extensions"] > 0


@pytest.mark.parametrize("band", [12, 13, 32, 33])
def test_hapl_kernel_boundaries(small, band):
    # the LDS tables change at these bands: 12 is the last on 64 cells and
    # 16 previous ones, 13 the first on 128 cells, 32 fills the 32 previous
    # cells exactly, 33 the first on 256 cells (one query a wavefront);
    # cheap gaps and mismatches fill the band at most positions
    say(f"case: haplotype enumeration at band {band} (a boundary between LDS table sizes)")
    w, idx, text, _ = small
    qs = _reads(w, 60, 20, 90, sub=0.03, indel=0.005, stream=15000)
    P = synth.pack(qs)
    for scores in ((1, 4, 6, 1), (2, 1, 1, 1)):
        m, x, o, e = scores
        recs, off = idx.hapl(P.data, P.lens, match=m, mismatch=x, gap_open=o, gap_ext=e, band=band)
        _compare(text, qs, recs, off, match=m, mismatch=x, gap_open=o, gap_ext=e, band=band)


def test_hapl_random_configurations(small):
    # seeded draws of scores (match 1-3, mismatch 0-4, gap open 0-6, gap
    # extension 1-3), bands across the LDS table sizes and both kernels
    say("case: haplotype enumeration, 16 seeded configurations of scores, band and tables")
    w, idx, text, _ = small
    g = np.random.default_rng(2024)
    for t in range(16):
        m, x, o, e = int(g.integers(1, 4)), int(g.integers(0, 5)), int(g.integers(0, 7)), int(g.integers(1, 4))
        band = int(g.choice([0, 1, 3, 7, 10, 12, 13, 16, 25, 31, 32, 33, 40]))
        dev = bool(g.integers(0, 2))
        qs = _reads(w, 16, 6, 14 if band == 0 else 70, sub=0.03, indel=0.005, stream=21000 + 100 * t)
        P = synth.pack(qs)
        kw = dict(match=m, mismatch=x, gap_open=o, gap_ext=e, band=band)
        say(f"  {kw} device tables {dev}")
        recs, off = idx.hapl(P.data, P.lens, device_tables=dev, max_cells=65535, **kw)
        _compare(text, qs, recs, off, **kw)


def test_hapl_repeatable(small):
    # lanes race to create cells; no result may depend on which one wins
    say("case: haplotype enumeration twice on the same reads (band 25, cheap gaps): equal records")
    w, idx, _, _ = small
    qs = _reads(w, 200, 20, 90, sub=0.03, indel=0.005, stream=16000)
    P = synth.pack(qs)
    kw = dict(match=2, mismatch=1, gap_open=1, gap_ext=1, band=25)
    r1, o1 = idx.hapl(P.data, P.lens, **kw)
    r2, o2 = idx.hapl(P.data, P.lens, **kw)
    assert np.array_equal(o1, o2) and np.array_equal(r1, r2)


@pytest.mark.parametrize("scores", [(1, 4, 6, 1), (2, 1, 1, 1)])
@pytest.mark.parametrize("dev", [False, True])
def test_hapl_matches_oracle_unbanded(small, dev, scores):
    m, x, o, e = scores
    say(f"case: haplotype enumeration without a band, reads 4-14 bp, device tables {dev}, scores {scores}")
    w, idx, text, _ = small
    # cheap gaps keep many more cells without a band: fewer reads for the oracle
    qs = _reads(w, 80 if scores == (1, 4, 6, 1) else 30, 4, 14, stream=5000)
    P = synth.pack(qs)
    recs, off = idx.hapl(P.data, P.lens, match=m, mismatch=x, gap_open=o, gap_ext=e, band=0, max_cells=65535,
                         device_tables=dev)
    _compare(text, qs, recs, off, match=m, mismatch=x, gap_open=o, gap_ext=e, band=0)


def test_hapl_queries_moved_to_device_tables(small):
    say("case: haplotype enumeration without a band, reads of 10-20 and of 80-100 bp: the queries whose cells "
        "outgrow the LDS tables are finished in device memory")
    w, idx, text, _ = small
    qs = _reads(w, 30, 10, 20, stream=7000) + _reads(w, 30, 80, 100, sub=0.0, indel=0.0, stream=7100)
    P = synth.pack(qs)
    recs, off = idx.hapl(P.data, P.lens, band=0, max_cells=65535)
    st = rb3.rb3_last_hapl_stats()
    say(f"moved {st['moved']} of {len(qs)}")
    assert 0 < st["moved"] < len(qs)
    _compare(text, qs, recs, off, band=0)


@pytest.mark.parametrize("scores", [(1, 4, 6, 1), (2, 3, 5, 2), (1, 2, 3, 2), (3, 1, 2, 3)])
def test_hapl_other_scores(small, scores):
    m, x, o, e = scores
    say(f"case: haplotype enumeration with match {m}, mismatch {x}, gap open {o}, gap extension {e}")
    w, idx, text, _ = small
    qs = _reads(w, 40, 10, 50, sub=0.04, indel=0.01, stream=9000)
    P = synth.pack(qs)
    recs, off = idx.hapl(P.data, P.lens, match=m, mismatch=x, gap_open=o, gap_ext=e, band=25, max_cells=16384)
    _compare(text, qs, recs, off, match=m, mismatch=x, gap_open=o, gap_ext=e, band=25)


@pytest.mark.parametrize("band", [10, 12])
@pytest.mark.parametrize("scores", [(2, 1, 1, 1), (3, 1, 2, 3)])
def test_hapl_many_tied_cells_small_band(small, band, scores):
    # with cheap mismatches and gaps, more than 16 cells tie at the band's
    # threshold at some positions (the oracle counts 80 such cuts for
    # (2, 1, 1, 1) at band 10 on these reads), so the ranking of the tied
    # cells counts over all cells instead of its 16-entry list
    m, x, o, e = scores
    say(f"case: haplotype enumeration at band {band} with match {m}, mismatch {x}, gap open {o}, gap extension {e}: "
        "more tied cells than the tie list holds")
    w, idx, text, _ = small
    qs = _reads(w, 40, 10, 50, sub=0.04, indel=0.01, stream=9000)
    P = synth.pack(qs)
    recs, off = idx.hapl(P.data, P.lens, match=m, mismatch=x, gap_open=o, gap_ext=e, band=band)
    _compare(text, qs, recs, off, match=m, mismatch=x, gap_open=o, gap_ext=e, band=band)


@pytest.mark.parametrize("band", [0, 1, 2, 20, 40])
def test_hapl_band_tie_break_worked_case(band):
    # AC and GC (both strands) against the query TC with a free mismatch:
    # the cells AC and GC tie at score 1, and a band of one keeps AC, whose
    # suffix-array interval starts first; each band runs a different kernel
    say(f"case: haplotype enumeration tie at the band's edge, band {band}")
    strs = [b"AC", b"GC"]
    P0 = synth.pack(strs)
    idx = rb3.rb3_build(P0.data, P0.lens)
    codes, lens = oracle.expand(P0.data, P0.lens)
    text = oracle.Text(codes, lens)
    enc = lambda s: np.array([ENC[c] for c in s], np.uint8)
    ac, _ = text.interval(enc(b"AC"))
    gc, _ = text.interval(enc(b"GC"))
    gt, _ = text.interval(enc(b"GT"))
    Q = synth.pack([b"TC"])
    recs, off = idx.hapl(Q.data, Q.lens, mismatch=0, band=band)
    got = [(int(a["k"]), int(a["krc"]), int(a["s"]), int(a["score"])) for a in recs]
    assert got == ([(ac, gt, 1, 1)] if band == 1 else [(ac, gt, 1, 1), (gc, gc, 2, 1)])
    _compare(text, [b"TC"], recs, off, mismatch=0, band=band)
    idx.close()


@pytest.mark.parametrize("band", [10, 25, 40, 0])
def test_hapl_run_length_index_and_output_retry(small, band):
    say(f"case: haplotype enumeration on the run-length index at band {band}; output sized by a retry")
    w, idx, text, _ = small
    # without a band, short reads (every cell is kept)
    qs = _reads(w, 60, 20, 80, stream=12000) if band else _reads(w, 40, 4, 14, stream=12500)
    P = synth.pack(qs)
    r = rb3.rb3_rle_build(idx, 0)
    recs, off = r.hapl(P.data, P.lens, cap=1, band=band)
    precs, poff = idx.hapl(P.data, P.lens, band=band)
    assert np.array_equal(off, poff) and np.array_equal(recs, precs)
    _compare(text, qs, recs, off, band=band)
    r.close()


def test_hapl_argument_checks(small):
    say("case: haplotype enumeration argument checks")
    w, idx, _, _ = small
    P = synth.pack(_reads(w, 4, 30, 40))
    for kw in ({"match": 0}, {"gap_ext": 0}, {"mismatch": -1}, {"band": -1}, {"max_cells": -1},
               {"max_cells": 65536}):
        with pytest.raises(rb3.RB3Error) as e:
            idx.hapl(P.data, P.lens, **kw)
        assert e.value.code == rb3.RB3_EINVAL, kw
    with pytest.raises(rb3.RB3Error) as e:
        idx.hapl(P.data, P.lens, max_cells=2)
    assert e.value.code == rb3.RB3_ELIMIT
    with pytest.raises(rb3.RB3Error) as e:
        idx.hapl(b"ACGTX", [5])
    assert e.value.code == rb3.RB3_EINVAL
    one = rb3.rb3_build(w.b1.data, w.b1.lens, both_strands=False)
    with pytest.raises(rb3.RB3Error) as e:
        one.hapl(P.data, P.lens)
    assert e.value.code == rb3.RB3_EINVAL
    one.close()
    recs, off = idx.hapl(b"", np.zeros(0, np.int64))
    assert recs.shape[0] == 0 and off.tolist() == [0]


def _properties(idx, qs, recs, off, n, exact):
    """What holds at any size: valid intervals, order by score, no result
    inside an earlier one, scores at most the query length, and an exact
    read's best result its own bi-interval with the full score."""
    for i, q in enumerate(qs):
        got = recs[off[i]:off[i + 1]]
        assert np.all(got["s"] > 0) and np.all(got["k"] + got["s"] <= n) and np.all(got["krc"] + got["s"] <= n)
        sc = got["score"].astype(np.int64)
        assert np.all(sc > 0) and np.all(sc <= len(q))
        assert np.all(np.diff(sc) <= 0)
        for a in range(got.shape[0]):
            for b in range(a):
                x, y = got[a], got[b]
                assert not (y["k"] <= x["k"] and x["k"] + x["s"] <= y["k"] + y["s"])
                assert not (y["krc"] <= x["krc"] and x["krc"] + x["s"] <= y["krc"] + y["s"])
    if exact:
        P = synth.pack(qs)
        lo, hi = idx.count(P.data, P.lens)
        comp = bytes.maketrans(b"ACGT", b"TGCA")
        R = synth.pack([q.translate(comp)[::-1] for q in qs])
        rlo, _ = idx.count(R.data, R.lens)
        for i, q in enumerate(qs):
            top = recs[off[i]]
            assert (int(top["k"]), int(top["krc"]), int(top["s"]), int(top["score"])) == \
                (int(lo[i]), int(rlo[i]), int(hi[i] - lo[i]), len(q)), i


def test_hapl_bench_shape_properties():
    say("case: haplotype enumeration of 125 bp reads on 32 haplotypes x 200 kb, band 10: properties")
    w = synth.config_pangenome(genome_len=200_000, n_b1=32, n_new=4)
    idx = rb3.rb3_build(w.b1.data, w.b1.lens)
    n = idx.info()[0]
    qs = _reads(w, 3000, 125, 125, sub=0.01, indel=0.001, stream=20000)
    P = synth.pack(qs)
    recs, off = idx.hapl(P.data, P.lens, band=10)
    _properties(idx, qs, recs, off, n, exact=False)
    g = np.random.default_rng(4)
    ex = []
    for _ in range(300):
        h = w.b1.get(int(g.integers(0, w.b1.n)))
        s = int(g.integers(0, len(h) - 125))
        ex.append(h[s:s + 125])
    E = synth.pack(ex)
    erecs, eoff = idx.hapl(E.data, E.lens, band=10)
    _properties(idx, ex, erecs, eoff, n, exact=True)
    idx.close()


@pytest.mark.parametrize("scores", [(1, 4, 6, 1), (2, 1, 1, 1)])
@pytest.mark.parametrize("band", [10, 25])
def test_hapl_lds_and_device_tables_agree_at_scale(band, scores):
    # the two kernels take the same steps independently (wavefronts with LDS
    # tables, one thread per query with device-memory tables): every record
    # equal on 3,000 reads of 125 bp against 32 haplotypes x 200 kb
    m, x, o, e = scores
    say(f"case: haplotype enumeration, LDS against device-memory tables, 3,000 reads of 125 bp, band {band}, "
        f"scores {scores}")
    w = synth.config_pangenome(genome_len=200_000, n_b1=32, n_new=4)
    idx = rb3.rb3_build(w.b1.data, w.b1.lens)
    qs = _reads(w, 3000, 125, 125, sub=0.01, indel=0.001, stream=40000)
    P = synth.pack(qs)
    kw = dict(match=m, mismatch=x, gap_open=o, gap_ext=e, band=band, max_cells=4096)
    a, ao = idx.hapl(P.data, P.lens, **kw)
    b, bo = idx.hapl(P.data, P.lens, device_tables=True, **kw)
    assert np.array_equal(ao, bo) and np.array_equal(a, b)
    idx.close()


@pytest.mark.parametrize("band", [10, 25])
def test_hapl_125bp_sample_against_oracle(band):
    say(f"case: haplotype enumeration of 125 bp reads on 32 haplotypes x 30 kb, band {band}: a sample against the "
        "oracle")
    w = synth.config_pangenome(genome_len=30_000, n_b1=32, n_new=4)
    idx = rb3.rb3_build(w.b1.data, w.b1.lens)
    qs = _reads(w, 2000, 125, 125, sub=0.01, indel=0.001, stream=30000)
    P = synth.pack(qs)
    recs, off = idx.hapl(P.data, P.lens, band=band)
    _properties(idx, qs, recs, off, idx.info()[0], exact=False)
    codes, lens = oracle.expand(w.b1.data, w.b1.lens)
    text = oracle.Text(codes, lens)
    pick = list(range(0, 2000, 100))
    _compare(text, [qs[i] for i in pick], *_subset(recs, off, pick), band=band)
    idx.close()


def _subset(recs, off, pick):
    parts, o = [], [0]
    for j, i in enumerate(pick):
        r = recs[off[i]:off[i + 1]].copy()
        r["qid"] = j
        parts.append(r)
        o.append(o[-1] + r.shape[0])
    return np.concatenate(parts), np.array(o, np.int64)


@pytest.mark.parametrize("dev", [False, True])
def test_hapl_query_longer_than_65535(dev):
    say(f"case: haplotype enumeration of a 70,000 bp exact query, band 1, device tables {dev} (their 16-bit hash "
        "generations wrap)")
    g = np.random.default_rng(11)
    acgt = np.frombuffer(b"ACGT", np.uint8)
    s = acgt[g.integers(0, 4, 80_000)].tobytes()
    idx = rb3.rb3_build(np.frombuffer(s, np.uint8), np.array([len(s)], np.int64))
    q = s[5000:75_000]
    # gap extension so costly that no gap cell is ever positive
    recs, off = idx.hapl(np.frombuffer(q, np.uint8), np.array([len(q)], np.int64), band=1, max_cells=16,
                         gap_ext=1 << 20, device_tables=dev)
    _properties(idx, [q], recs, off, idx.info()[0], exact=True)
    assert off.tolist() == [0, 1]
    idx.close()
