"""Failure handling, forced from the host so that every kernel still runs to
completion: device allocations that fail (an allocator hook that returns
NULL at the N-th call) and merges stopped after each stage (the library's
test hook). The merge's strong guarantee: after a failed merge the index
holds exactly the BWT it held before, and a retry gives the bytes a clean
merge gives. Also the server's bounded queue (RB3_EAGAIN)."""
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2409_00613_amd import rb3

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def work():
    # a small pangenome-shaped merge with short chunks, so that the fix-up,
    # the tie kernels and several sort passes all run
    w = synth.config_pangenome(genome_len=20_000, n_b1=6, n_new=6)
    allst = w.b1 + w.new
    codes, lens = oracle.expand(allst.data, allst.lens)
    want = oracle.bwt(codes, lens)
    return w, want


@pytest.mark.parametrize("ssa", [0, 8])
def test_allocation_failure_at_every_allocation(work, ssa):
    w, want = work
    say(f"case: a merge whose N-th device allocation fails, every N (samples every {ssa})")
    alloc = rb3.CountingAllocator(0)
    idx = rb3.rb3_build(w.b1.data, w.b1.lens, allocator=alloc, chunk_len=97, ssa_rate=ssa)
    before = idx.export()
    info = idx.info()
    # allocations of one clean merge, on a copy
    probe = idx.clone()
    alloc.reset()
    probe.merge(w.new.data, w.new.lens)
    total = alloc.calls
    assert np.array_equal(probe.export(), want)
    probe.close()
    assert total > 20
    for n in range(1, total + 1):
        alloc.reset(fail_at=n)
        with pytest.raises(rb3.RB3Error) as e:
            idx.merge(w.new.data, w.new.lens)
        assert e.value.code == rb3.RB3_ENOMEM, (n, e.value)
        alloc.reset()
        assert idx.info() == info, n
        assert np.array_equal(idx.export(), before), n
    alloc.reset()
    idx.merge(w.new.data, w.new.lens)
    assert np.array_equal(idx.export(), want)
    idx.close()


def test_merge_stopped_after_each_stage(work):
    w, want = work
    say("case: merges stopped after each stage leave the index unchanged; a retry is byte-identical")
    idx = rb3.rb3_build(w.b1.data, w.b1.lens, chunk_len=97, ssa_rate=8)
    before = idx.export()
    info = idx.info()
    try:
        for stage in (1, 2, 3, 4, 5):
            rb3.rb3_test_fail_merge_after(stage)
            with pytest.raises(rb3.RB3Error) as e:
                idx.merge(w.new.data, w.new.lens)
            assert e.value.code == rb3.RB3_EDEVICE and "stage" in str(e.value), stage
            rb3.rb3_test_fail_merge_after(0)
            assert idx.info() == info and np.array_equal(idx.export(), before), stage
    finally:
        rb3.rb3_test_fail_merge_after(0)
    idx.merge(w.new.data, w.new.lens)
    assert np.array_equal(idx.export(), want)
    # the located positions are those of a clean merge too
    ref = rb3.rb3_build(w.b1.data, w.b1.lens, chunk_len=97, ssa_rate=8)
    ref.merge(w.new.data, w.new.lens)
    rows = np.arange(0, len(want), 7, dtype=np.int64)
    a, b = idx.locate(rows), ref.locate(rows)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    ref.close()
    idx.close()


def test_build_stopped_returns_no_index(work):
    w, _ = work
    say("case: a build stopped after a stage returns an error and no index")
    try:
        rb3.rb3_test_fail_merge_after(2)
        with pytest.raises(rb3.RB3Error) as e:
            rb3.rb3_build(w.b1.data, w.b1.lens)
        assert e.value.code == rb3.RB3_EDEVICE
    finally:
        rb3.rb3_test_fail_merge_after(0)
    with pytest.raises(rb3.RB3Error):
        rb3.rb3_test_fail_merge_after(6)


def test_server_queue_full_gives_eagain():
    say("case: a server with a short queue refuses submissions with RB3_EAGAIN, then serves them")
    w = synth.config_serving(genome_len=200_000, n_index=8, n_unseen=2, n_queries=40, log_lo=3.0, log_hi=4.0)
    idx = rb3.rb3_build(w.index.data, w.index.lens)
    srv = rb3.Server(idx, workers=1, max_batch_queries=1, max_queued=2)
    assert srv.stats()["mem_budget"] > 0  # taken from the device's free memory
    tickets, refused = {}, 0
    for i in range(w.queries.n):
        q = w.queries.get(i)
        while True:
            try:
                tickets[srv.submit(rb3.RB3_REQ_SMEM, q, 31, 1)] = i
                break
            except rb3.RB3Error as e:
                assert e.code == rb3.RB3_EAGAIN
                refused += 1
                time.sleep(0.001)
    got = {}
    t0 = time.time()
    while len(got) < len(tickets):
        for r in srv.poll(wait_ms=50):
            got[r["ticket"]] = r
        assert time.time() - t0 < 60
    srv.close()
    assert refused > 0
    recs, off = idx.smem(w.queries.data, w.queries.lens, 31, 1)
    fields = ["start", "end", "occ", "k", "krc"]
    for t, i in tickets.items():
        mine = np.stack([got[t]["records"][f] for f in fields], 1) if len(got[t]["records"]) else np.zeros((0, 5))
        r = recs[off[i]:off[i + 1]]
        ref = np.stack([r[f] for f in fields], 1) if len(r) else np.zeros((0, 5))
        assert np.array_equal(mine, ref), i
    idx.close()


def test_replay_leaves_other_results_queued():
    say("case: an open-loop replay takes only its own results")
    w = synth.config_serving(genome_len=100_000, n_index=4, n_unseen=2, n_queries=30, log_lo=2.0, log_hi=3.0)
    idx = rb3.rb3_build(w.index.data, w.index.lens)
    srv = rb3.Server(idx, workers=2)
    other = srv.submit(rb3.RB3_REQ_COUNT, w.queries.get(0))
    time.sleep(0.2)  # let it finish before the replay starts
    lat, wall = srv.replay(rb3.RB3_REQ_SMEM, w.queries.data, w.queries.lens,
                           np.linspace(0, 0.01, w.queries.n), 31, 1)
    assert (lat >= 0).all() and wall > 0
    res = srv.poll(wait_ms=100)
    assert [r["ticket"] for r in res] == [other]
    lo, hi = idx.count(w.queries.slice(0, 1).data, w.queries.slice(0, 1).lens)
    assert (res[0]["lo"], res[0]["hi"]) == (int(lo[0]), int(hi[0]))
    srv.close()
    idx.close()
