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


def test_uneven_lengths_follow_the_log_normal_reading():
    """Contig lengths: log-normal around a 10 kb median with sigma = ln(100)/3
    (so +-3 sigma spans 100 bp..1 Mb), redrawn outside [100, 10^6]; the
    mean of that distribution is about 30 kb."""
    u = synth.config_uneven(genome_len=200_000, n_b1=2, n_src=4, n_contigs=3000, chrom_len=1000,
                            n_chrom=0, len_hi=1_000_000)
    L = u.new.lens.astype(np.float64)
    # contigs are cut to their 200 kb source haplotype here, so compare the
    # median and the spread of the log-lengths, which the cut barely moves
    assert 8_000 < np.median(L) < 12_500
    assert 1.35 < np.std(np.log(L[L < 150_000])) < 1.6
    assert L.min() >= 100


def test_incremental_duplications_shared_by_haplotypes():
    inc = synth.config_incremental(genome_len=300_000, n_hap=3, dup_frac=0.01, dup_lo=1000, dup_hi=5000)
    base = synth.random_genome(300_000, synth.rng(inc.seed, synth.STREAM_BASE))
    changed = int((inc.base != base).sum())
    # about 1% of the genome overwritten (copies may overlap or copy equal bases)
    assert 1_000 < changed < 9_000
    h0, h0b = inc.haplotype(0), inc.haplotype(0)
    assert np.array_equal(h0, h0b) and abs(h0.shape[0] - 300_000) < 300
