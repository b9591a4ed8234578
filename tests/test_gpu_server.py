"""The continuous-batching server: every result is the same alone and in a
concurrent mix, and equal to the direct calls and to the oracle."""
import random
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2409_00613_amd import rb3

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def _drain(srv, n, timeout=60.0):
    got = {}
    t0 = time.time()
    while len(got) < n:
        for r in srv.poll(wait_ms=50):
            got[r["ticket"]] = r
        assert time.time() - t0 < timeout, "server did not answer in time"
    return got


def _key(r):
    if r["kind"] == rb3.RB3_REQ_COUNT:
        return ("c", r["status"], r["lo"], r["hi"])
    rec = r["records"]
    return ("s", r["status"], rec[["start", "end", "occ", "k", "krc"]].tobytes())


@pytest.fixture(scope="module")
def setup():
    w = synth.config_serving(genome_len=60_000, n_index=6, n_unseen=3, n_queries=60, log_lo=1.5, log_hi=3.9)
    idx = rb3.rb3_build(w.index.data, w.index.lens)
    rnd = random.Random(3)
    reqs = []
    for i in range(w.queries.n):
        q = w.queries.get(i)
        kind = rb3.RB3_REQ_SMEM if i % 3 else rb3.RB3_REQ_COUNT
        ml = rnd.choice([19, 31, 51])
        mo = rnd.choice([1, 1, 2])
        reqs.append((kind, q, ml, mo))
    yield w, idx, reqs
    idx.close()


def test_server_alone_equals_mix_equals_direct(setup):
    w, idx, reqs = setup
    say("case: server results alone vs in a mix vs direct calls")
    srv = rb3.Server(idx, workers=4, max_batch_queries=16)
    alone = []
    for kind, q, ml, mo in reqs:
        t = srv.submit(kind, q, ml, mo)
        alone.append(_key(_drain(srv, 1)[t]))
    tickets = [srv.submit(kind, q, ml, mo) for kind, q, ml, mo in reqs]
    mixed = _drain(srv, len(reqs))
    st = srv.stats()
    srv.close()
    assert st["max_batch"] > 1  # requests really were batched together
    for i, t in enumerate(tickets):
        assert _key(mixed[t]) == alone[i], i
    # direct calls
    for i, (kind, q, ml, mo) in enumerate(reqs):
        s = synth.pack([q])
        if kind == rb3.RB3_REQ_COUNT:
            lo, hi = idx.count(s.data, s.lens)
            assert alone[i] == ("c", 0, int(lo[0]), int(hi[0]))
        else:
            recs, off = idx.smem(s.data, s.lens, ml, mo)
            assert alone[i] == ("s", 0, recs[["start", "end", "occ", "k", "krc"]].tobytes())


def test_server_matches_oracle(setup):
    w, idx, reqs = setup
    say("case: server SMEM results against the oracle")
    codes, lens = oracle.expand(w.index.data, w.index.lens)
    text = oracle.Text(codes, lens)
    srv = rb3.Server(idx, workers=3, max_batch_queries=8, max_batch_bases=20_000, mem_budget=1 << 22)
    tickets = [srv.submit(kind, q, ml, mo) for kind, q, ml, mo in reqs]
    got = _drain(srv, len(reqs))
    srv.close()
    for t, (kind, q, ml, mo) in zip(tickets, reqs):
        qc, ql = oracle.encode(np.frombuffer(q, np.uint8), np.array([len(q)]))
        r = got[t]
        assert r["status"] == 0
        if kind == rb3.RB3_REQ_COUNT:
            assert (r["lo"], r["hi"]) == text.interval(qc)
        else:
            exp = text.smem(qc, ml, mo)
            rec = r["records"]
            g = np.stack([rec["start"], rec["end"], rec["occ"], rec["k"], rec["krc"]], 1) if len(rec) else np.zeros((0, 5))
            assert np.array_equal(g, exp)


def test_server_rejects_bad_input(setup):
    w, idx, reqs = setup
    say("case: server input validation")
    srv = rb3.Server(idx, workers=1)
    with pytest.raises(rb3.RB3Error):
        srv.submit(rb3.RB3_REQ_SMEM, b"ACGTXACGT", 5, 1)
    with pytest.raises(rb3.RB3Error):
        srv.submit(rb3.RB3_REQ_SMEM, b"ACGT", 0, 1)
    t = srv.submit(rb3.RB3_REQ_COUNT, b"", 0, 1)
    r = _drain(srv, 1)[t]
    n, _, _ = idx.info()
    assert (r["lo"], r["hi"]) == (0, n)
    srv.close()
