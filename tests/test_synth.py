"""The seeded input generator: reproducible, right shapes and rates."""
import numpy as np

import synth


def test_tiny_config_shapes_and_determinism():
    a = synth.config_tiny()
    b = synth.config_tiny()
    assert a.b1.n == 32 and a.new.n == 32 and a.queries.n == 1000
    assert set(np.unique(a.b1.data).tobytes()) <= set(b"ACGT")
    assert (a.b1.lens == 2000).all()
    assert np.array_equal(a.new.data, b.new.data) and np.array_equal(a.queries.data, b.queries.data)
    assert 20 <= a.queries.lens.min() and a.queries.lens.max() <= 100


def test_haplotype_rates():
    g = synth.rng(1, 0)
    base = synth.random_genome(400_000, g)
    hap = synth.haplotype(base, 1e-3, 1e-4, synth.rng(1, 1))
    # indels shift the length by a few hundred bases at most
    assert abs(hap.shape[0] - base.shape[0]) < 400
    snp_only = synth.haplotype(base, 1e-3, 0.0, synth.rng(1, 1))
    diff = int((snp_only != base).sum())
    assert 300 < diff < 500


def test_pangenome_small():
    w = synth.config_pangenome(genome_len=20_000, n_b1=4, n_new=4)
    assert w.b1.n == 4 and w.new.n == 4
    assert abs(int(w.b1.lens[0]) - 20_000) < 100


def test_mutate_and_segdups():
    g = synth.rng(2, 0)
    s = synth.random_genome(10_000, g)
    m = synth.mutate(s, 0.01, 0.0, synth.rng(2, 1))
    assert m.shape == s.shape and 40 < int((m != s).sum()) < 200
    d = synth.segmental_duplications(s, 0.05, 100, 300, synth.rng(2, 2))
    assert d.shape == s.shape and (d != s).any()
