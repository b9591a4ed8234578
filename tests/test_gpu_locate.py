"""Suffix-array samples and locate: every row's position after builds and
merges against the oracle's suffix array, the number of samples against its
definition, Locate1 hits checked through the oracle's inverse suffix array,
and the error paths."""
import random

import numpy as np
import pytest

import oracle
import synth
from paper_2409_00613_amd import rb3

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def _sa(strings, both=True):
    codes, lens = oracle.expand(strings.data, strings.lens, both=both)
    B, S = oracle.bwt(codes, lens, want_sa=True)
    return B, S, lens


def _expected_samples(batches, rate, both=True):
    """Samples of an index built from these batches: per batch, the positions
    of the batch's strands laid end to end (each with its sentinel) that are
    multiples of rate, plus every strand's first position."""
    total = 0
    for b in batches:
        k = 2 if both else 1
        lens = np.repeat(b.lens, k)
        starts = np.concatenate([[0], np.cumsum(lens + 1)])[:-1]
        n2 = int((lens + 1).sum())
        total += len(set(range(0, n2, rate)) | set(starts.tolist()))
    return total


def _check_all_rows(idx, strings, both=True):
    B, S, lens = _sa(strings, both)
    n = S.shape[0]
    assert idx.info()[0] == n
    rows = np.arange(n, dtype=np.int64)
    st, off = idx.locate(rows)
    wj, woff = oracle.locate(S, lens, rows)
    assert np.array_equal(st, wj)
    assert np.array_equal(off, woff)


@pytest.mark.parametrize("rate", [1, 3, 8, 32])
def test_locate_every_row_after_build(rate):
    say(f"case: build with sampling distance {rate}, locate every row")
    w = synth.config_tiny(n_str=12, length=300)
    idx = rb3.rb3_build(w.b1.data, w.b1.lens, ssa_rate=rate)
    assert idx.ssa_info() == (rate, _expected_samples([w.b1], rate))
    _check_all_rows(idx, w.b1)
    idx.close()


@pytest.mark.parametrize("both", [True, False])
def test_locate_every_row_after_merges(both):
    say(f"case: build + three merges with sampling distance 8, both strands {both}")
    w = synth.config_tiny(n_str=24, length=400)
    allst = w.b1 + w.new
    parts = [allst.slice(0, 5), allst.slice(5, 6), allst.slice(6, 20), allst.slice(20, allst.n)]
    idx = rb3.rb3_build(parts[0].data, parts[0].lens, both_strands=both, ssa_rate=8, chunk_len=64)
    for p in parts[1:]:
        idx.merge(p.data, p.lens)
    assert idx.ssa_info() == (8, _expected_samples(parts, 8, both))
    _check_all_rows(idx, allst, both)
    idx.close()


def test_samples_do_not_change_the_bwt():
    say("case: pangenome merge with and without samples give the same BWT")
    w = synth.config_pangenome(genome_len=20_000, n_b1=8, n_new=8)
    out = []
    for rate in (0, 16):
        idx = rb3.rb3_build(w.b1.data, w.b1.lens, ssa_rate=rate, chunk_len=256)
        idx.merge(w.new.data, w.new.lens)
        out.append(idx.export())
        if rate:
            _check_all_rows(idx, w.b1 + w.new)
        idx.close()
    assert np.array_equal(out[0], out[1])


def test_locate_sampled_rows_large_groups():
    """Many copies of a few strings: tie groups of every size class whose
    members share their BWT symbols, so only the samples force their order."""
    say("case: repeated strings, groups up to 300 members, sampling distance 5")
    rnd = random.Random(3)
    base = ["".join(rnd.choice("ACGT") for _ in range(rnd.randint(30, 90))) for _ in range(4)]
    strs = [base[i % 4].encode() for i in range(300)] + [base[0][:40].encode()] * 20
    s = synth.pack(strs)
    a, b = s.slice(0, 150), s.slice(150, s.n)
    idx = rb3.rb3_build(a.data, a.lens, ssa_rate=5)
    idx.merge(b.data, b.lens)
    _check_all_rows(idx, s)
    st = idx.merge_stats()
    assert st["max_group"] >= 65
    idx.close()


def test_locate1_hits_lie_in_their_intervals():
    say("case: Locate1 on intervals of substrings and random patterns")
    w = synth.config_tiny(n_str=16, length=500)
    allst = w.b1 + w.new
    idx = rb3.rb3_build(allst.data, allst.lens, ssa_rate=16)
    codes, lens = oracle.expand(allst.data, allst.lens)
    B, S = oracle.bwt(codes, lens, want_sa=True)
    rnd = random.Random(9)
    pats = []
    for _ in range(400):
        src = allst.get(rnd.randrange(allst.n))
        L = rnd.randint(1, 12)
        if rnd.random() < 0.8 and len(src) > L:
            st0 = rnd.randrange(len(src) - L)
            pats.append(src[st0:st0 + L])
        else:
            pats.append("".join(rnd.choice("ACGT") for _ in range(L)).encode())
    q = synth.pack(pats)
    lo, hi = idx.count(q.data, q.lens)
    st, off = idx.locate1(lo, hi)
    nonempty = hi > lo
    assert nonempty.sum() > 300
    assert np.all(st[~nonempty] == -1) and np.all(off[~nonempty] == -1)
    rows = oracle.rows_of(S, lens, st[nonempty], off[nonempty])
    assert np.all(rows >= lo[nonempty]) and np.all(rows < hi[nonempty])
    # the located text matches the pattern
    starts = np.concatenate([[0], np.cumsum(lens)])
    for i in np.flatnonzero(nonempty)[:100]:
        j, o = int(st[i]), int(off[i])
        got = codes[starts[j] + o: starts[j] + o + len(pats[i])]
        assert np.array_equal(got, oracle.encode(np.frombuffer(pats[i], np.uint8),
                                                  np.array([len(pats[i])]))[0])
    # the whole index as one interval, and single rows
    st, off = idx.locate1(np.array([0, 5]), np.array([S.shape[0], 6]))
    r = oracle.rows_of(S, lens, st, off)
    assert 0 <= r[0] < S.shape[0] and r[1] == 5
    idx.close()


def test_locate_device_rows_and_errors():
    say("case: rows in device memory; rows out of range; index without samples")
    import torch
    w = synth.config_tiny(n_str=6, length=200)
    idx = rb3.rb3_build(w.b1.data, w.b1.lens, ssa_rate=4)
    n = idx.info()[0]
    rows = np.array([0, n - 1, n // 2, 7], np.int64)
    st_h, off_h = idx.locate(rows)
    st_d, off_d = idx.locate(torch.from_numpy(rows).cuda())
    assert st_d.is_cuda and off_d.is_cuda
    assert np.array_equal(st_h, st_d.cpu().numpy()) and np.array_equal(off_h, off_d.cpu().numpy())
    lo_d = torch.tensor([0, 5], dtype=torch.int64, device="cuda")
    hi_d = torch.tensor([n, 6], dtype=torch.int64, device="cuda")
    st1, off1 = idx.locate1(lo_d, hi_d)
    st1h, off1h = idx.locate1(np.array([0, 5]), np.array([n, 6]))
    assert np.array_equal(st1.cpu().numpy(), st1h) and np.array_equal(off1.cpu().numpy(), off1h)
    for bad in ([-1], [n]):
        with pytest.raises(rb3.RB3Error) as e:
            idx.locate(np.array(bad, np.int64))
        assert e.value.code == rb3.RB3_EINVAL
    with pytest.raises(rb3.RB3Error):
        idx.locate1(np.array([3]), np.array([2]))
    with pytest.raises(rb3.RB3Error) as e:
        idx.locate1(np.array([0]), np.array([n + 1]))
    assert e.value.code == rb3.RB3_EINVAL
    # a clone keeps the samples
    c = idx.clone()
    assert c.ssa_info() == idx.ssa_info()
    st_c, off_c = c.locate(rows)
    assert np.array_equal(st_c, st_h) and np.array_equal(off_c, off_h)
    c.close()
    idx.close()
    plain = rb3.rb3_build(w.b1.data, w.b1.lens)
    assert plain.ssa_info() == (0, 0)
    with pytest.raises(rb3.RB3Error) as e:
        plain.locate(np.array([0], np.int64))
    assert e.value.code == rb3.RB3_EINVAL
    plain.close()


def test_locate_pangenome_sampled_rows():
    say("case: pangenome merge (60 kb genome, 8 + 8 haplotypes), 20,000 random rows, distance 32")
    w = synth.config_pangenome(genome_len=60_000, n_b1=8, n_new=8)
    idx = rb3.rb3_build(w.b1.data, w.b1.lens, ssa_rate=32)
    idx.merge(w.new.data, w.new.lens)
    allst = w.b1 + w.new
    codes, lens = oracle.expand(allst.data, allst.lens)
    B, S = oracle.bwt(codes, lens, want_sa=True)
    assert np.array_equal(idx.export(), B)
    rnd = np.random.default_rng(5)
    rows = rnd.integers(0, S.shape[0], 20_000)
    st, off = idx.locate(rows)
    wj, woff = oracle.locate(S, lens, rows)
    assert np.array_equal(st, wj) and np.array_equal(off, woff)
    steps = rb3.rb3_last_locate_stats()["lf_steps"]
    assert steps < 20_000 * 32
    idx.close()
