"""The autotuner: it picks one of its candidates, later calls with the option
at 0 use the choice, results do not depend on it, and the table is written
to the file RB3_TUNE_CACHE names."""
import os

import numpy as np
import pytest

import oracle
import synth
from paper_2409_00613_amd import rb3

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def test_tune_merge_and_use(tmp_path, monkeypatch):
    say("case: merge chunk length tuned on a batch, then used by a merge with chunk_len 0")
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("RB3_TUNE_CACHE", str(cache))
    w = synth.config_pangenome(genome_len=300_000, n_b1=8, n_new=8)
    idx = rb3.rb3_build(w.b1.data, w.b1.lens)
    before = idx.export()
    t = rb3.rb3_tune_merge(idx, w.new.data, w.new.lens)
    assert t["chunk_len"] in t["trials"] and set(t["trials"]) <= {1024, 2048, 4096, 8192}
    assert np.array_equal(idx.export(), before)  # the trials merged into copies
    idx.merge(w.new.data, w.new.lens)
    assert idx.merge_stats()["chunk_len"] == t["chunk_len"]
    allst = w.b1 + w.new
    codes, lens = oracle.expand(allst.data, allst.lens)
    assert oracle.verify(idx.export(), codes, lens) == 0
    assert cache.exists() and str(t["chunk_len"]) in cache.read_text()
    idx.close()


def test_tune_smem_and_use():
    say("case: SMEM segment length tuned on a query batch; results do not depend on it")
    w = synth.config_serving(genome_len=300_000, n_index=8, n_unseen=2, n_queries=200, log_lo=2.0, log_hi=4.0)
    idx = rb3.rb3_build(w.index.data, w.index.lens)
    ref, roff = idx.smem(w.queries.data, w.queries.lens, 31, 1)
    t = rb3.rb3_tune_smem(idx, w.queries.data, w.queries.lens, 31, 1)
    assert t["segment"] in t["trials"] and -1 in t["trials"]
    got, goff = idx.smem(w.queries.data, w.queries.lens, 31, 1)
    assert np.array_equal(goff, roff)
    fields = ["start", "end", "occ", "k", "krc", "qid"]
    for f in fields:
        assert np.array_equal(got[f], ref[f])
    idx.close()
