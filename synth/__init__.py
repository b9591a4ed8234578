"""Seeded synthetic DNA inputs shaped like pangenome workloads.

This module only produces raw input strings: ASCII bytes over ``ACGT``
concatenated into one ``uint8`` array, plus an ``int64`` array of lengths.
It holds none of the indexing method's arithmetic (no symbol codes, no reverse
complements, no suffix order). Both the CPU oracle and the GPU library read
what it produces, each doing its own encoding.

Random numbers come from numpy's PCG64 seeded with ``SeedSequence([seed,
stream])``, so each object (base genome, haplotype h, query q, ...) has its
own reproducible stream independent of how many others are drawn.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import math
import os

import numpy as np

SEED = 240900613
_BASES = np.frombuffer(b"ACGT", dtype=np.uint8)
_IDX = np.full(256, 255, dtype=np.uint8)
for _i, _c in enumerate(b"ACGT"):
    _IDX[_c] = _i

# stream ids inside one config's seed
STREAM_BASE = 0
STREAM_HAP = 1            # haplotype h uses STREAM_HAP + h
STREAM_QUERY = 1_000_000  # query q uses STREAM_QUERY + q
STREAM_ARRIVAL = 2_000_000
STREAM_CONTIG = 3_000_000  # contig c uses STREAM_CONTIG + c
STREAM_SECOND_BASE = 999


@dataclasses.dataclass
class Strings:
    """An ordered list of strings: concatenated ASCII bytes plus lengths."""

    data: np.ndarray  # uint8, sum(lens) bytes
    lens: np.ndarray  # int64

    @property
    def n(self) -> int:
        return int(self.lens.shape[0])

    @property
    def total(self) -> int:
        return int(self.lens.sum()) if self.lens.size else 0

    def offsets(self) -> np.ndarray:
        off = np.zeros(self.n + 1, dtype=np.int64)
        np.cumsum(self.lens, out=off[1:])
        return off

    def get(self, i: int) -> bytes:
        off = self.offsets()
        return self.data[off[i]:off[i + 1]].tobytes()

    def as_list(self) -> list[bytes]:
        off = self.offsets()
        return [self.data[off[i]:off[i + 1]].tobytes() for i in range(self.n)]

    def slice(self, a: int, b: int) -> "Strings":
        off = self.offsets()
        return Strings(self.data[off[a]:off[b]].copy(), self.lens[a:b].copy())

    def __add__(self, other: "Strings") -> "Strings":
        return Strings(np.concatenate([self.data, other.data]),
                       np.concatenate([self.lens, other.lens]))


def pack(items) -> Strings:
    arrs = [np.frombuffer(x, dtype=np.uint8) if isinstance(x, (bytes, bytearray))
            else np.asarray(x, dtype=np.uint8) for x in items]
    lens = np.array([len(a) for a in arrs], dtype=np.int64)
    data = np.concatenate(arrs) if arrs else np.zeros(0, dtype=np.uint8)
    return Strings(np.ascontiguousarray(data), lens)


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream])))


def random_genome(n: int, g: np.random.Generator) -> np.ndarray:
    """n iid uniform bases over ACGT."""
    return _BASES[g.integers(0, 4, n)]


def _substitute(seq: np.ndarray, pos: np.ndarray, g: np.random.Generator) -> None:
    """Replace seq[pos] by a uniformly chosen *different* base, in place."""
    if pos.size == 0:
        return
    shift = g.integers(1, 4, pos.size).astype(np.uint8)
    seq[pos] = _BASES[(_IDX[seq[pos]] + shift) % 4]


def _geometric_capped(g: np.random.Generator, p: float, cap: int) -> int:
    while True:
        v = int(g.geometric(p))
        if v <= cap:
            return v


def haplotype(base: np.ndarray, snp: float, indel: float, g: np.random.Generator,
              indel_p: float = 1.0 / 3.0, indel_max: int = 10) -> np.ndarray:
    """Derive one haplotype from ``base``.

    Walking the base position by position: with probability ``snp`` the base
    is replaced by a different one; otherwise, with probability ``indel``, an
    event happens after it: an insertion (p=1/2) of L iid bases or a deletion
    (p=1/2) of the next L bases, L ~ Geometric(indel_p) redrawn while > indel_max
    (mean about 3, max 10).
    """
    n = base.shape[0]
    u = g.random(n)
    snp_mask = u < snp
    del u
    v = g.random(n)
    ev = np.flatnonzero((~snp_mask) & (v < indel))
    del v
    hap = base.copy()
    _substitute(hap, np.flatnonzero(snp_mask), g)
    del snp_mask
    pieces = []
    cur = 0
    for p in ev.tolist():
        if p < cur:
            continue  # inside an earlier deletion
        ins = g.random() < 0.5
        L = _geometric_capped(g, indel_p, indel_max)
        pieces.append(hap[cur:p + 1])
        if ins:
            pieces.append(random_genome(L, g))
            cur = p + 1
        else:
            cur = min(n, p + 1 + L)
    pieces.append(hap[cur:])
    return np.concatenate(pieces)


def mutate(seq: np.ndarray, sub: float, indel: float, g: np.random.Generator,
           indel_lo: int = 1, indel_hi: int = 5) -> np.ndarray:
    """Query-style mutation: substitutions at rate ``sub``; otherwise indels at
    rate ``indel`` with length uniform in [indel_lo, indel_hi], ins:del = 1:1."""
    n = seq.shape[0]
    out = seq.copy()
    u = g.random(n)
    sub_mask = u < sub
    _substitute(out, np.flatnonzero(sub_mask), g)
    if indel <= 0:
        return out
    v = g.random(n)
    ev = np.flatnonzero((~sub_mask) & (v < indel))
    pieces = []
    cur = 0
    for p in ev.tolist():
        if p < cur:
            continue
        ins = g.random() < 0.5
        L = int(g.integers(indel_lo, indel_hi + 1))
        pieces.append(out[cur:p + 1])
        if ins:
            pieces.append(random_genome(L, g))
            cur = p + 1
        else:
            cur = min(n, p + 1 + L)
    pieces.append(out[cur:])
    res = np.concatenate(pieces)
    return res if res.size else out[:1].copy()


def segmental_duplications(base: np.ndarray, frac: float, lo: int, hi: int,
                           g: np.random.Generator) -> np.ndarray:
    """Copy segments of length U{lo..hi} to uniform targets (overwriting) until
    their total reaches ``frac`` of the genome; with p=1/2 a copy is reversed
    and complemented (an inversion)."""
    out = base.copy()
    n = out.shape[0]
    total = 0
    comp = np.zeros(256, dtype=np.uint8)
    for a, b in zip(b"ACGT", b"TGCA"):
        comp[a] = b
    while total < frac * n:
        L = int(g.integers(lo, hi + 1))
        L = min(L, n)
        src = int(g.integers(0, n - L + 1))
        dst = int(g.integers(0, n - L + 1))
        seg = out[src:src + L].copy()
        if g.random() < 0.5:
            seg = comp[seg[::-1]]
        out[dst:dst + L] = seg
        total += L
    return out


# ---------------------------------------------------------------------------
# Workload configurations
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class MergeWorkload:
    name: str
    b1: Strings          # strings already in the index (one strand each)
    new: Strings         # strings to merge (one strand each)
    queries: Strings | None = None


def config_tiny(seed: int = SEED + 1, n_str: int = 64, length: int = 2000,
                n_queries: int = 1000, qmin: int = 20, qmax: int = 100,
                sub: float = 0.01) -> MergeWorkload:
    """Plain merge, tiny: iid uniform ACGT strings of equal length; the first
    half forms the existing index, the second half is merged; count queries
    are excerpts of the strings with substitutions."""
    strs = [random_genome(length, rng(seed, STREAM_HAP + i)) for i in range(n_str)]
    half = n_str // 2
    qs = []
    for q in range(n_queries):
        g = rng(seed, STREAM_QUERY + q)
        src = strs[int(g.integers(0, n_str))]
        L = int(g.integers(qmin, qmax + 1))
        L = min(L, src.shape[0])
        st = int(g.integers(0, src.shape[0] - L + 1))
        qs.append(mutate(src[st:st + L], sub, 0.0, g))
    return MergeWorkload("tiny", pack(strs[:half]), pack(strs[half:]), pack(qs))


def _workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, min(n, 16))


def haplotypes(base: np.ndarray, seed: int, hs, snp: float = 1e-3, indel: float = 1e-4) -> list[np.ndarray]:
    """Haplotypes h in ``hs`` of ``base``, each from its own stream
    (STREAM_HAP + h), drawn on a pool of threads; the result does not depend
    on the number of threads."""
    hs = list(hs)
    if len(hs) <= 1:
        return [haplotype(base, snp, indel, rng(seed, STREAM_HAP + h)) for h in hs]
    with concurrent.futures.ThreadPoolExecutor(min(_workers(), len(hs))) as ex:
        return list(ex.map(lambda h: haplotype(base, snp, indel, rng(seed, STREAM_HAP + h)), hs))


def pangenome_haplotypes(seed: int, genome_len: int, n_hap: int, snp: float = 1e-3,
                         indel: float = 1e-4, first: int = 0,
                         base: np.ndarray | None = None) -> list[np.ndarray]:
    if base is None:
        base = random_genome(genome_len, rng(seed, STREAM_BASE))
    return haplotypes(base, seed, range(first, first + n_hap), snp, indel)


def config_pangenome(seed: int = SEED + 2, genome_len: int = 4_000_000,
                     n_b1: int = 32, n_new: int = 32) -> MergeWorkload:
    """Pangenome-shaped merge: haplotypes of one random base genome (SNP 1e-3,
    indel 1e-4); the first ``n_b1`` form the existing index, the next
    ``n_new`` are merged."""
    haps = pangenome_haplotypes(seed, genome_len, n_b1 + n_new)
    return MergeWorkload("pangenome", pack(haps[:n_b1]), pack(haps[n_b1:]))


def config_uneven(seed: int = SEED + 3, genome_len: int = 4_000_000, n_b1: int = 32,
                  n_src: int = 64, n_contigs: int = 10_000, len_lo: int = 100,
                  len_hi: int = 1_000_000, median: float = 1e4,
                  chrom_len: int = 50_000_000, n_chrom: int = 2,
                  contig_snp: float = 0.005) -> MergeWorkload:
    """Batched uneven merge: the existing index is the pangenome index; the new
    batch is ``n_contigs`` log-normal-length excerpts of haplotypes (each with
    fresh SNPs) plus ``n_chrom`` chromosome-like haplotypes of a second base
    genome. Log-lengths are normal around ln(median) with sigma chosen so that
    +-3 sigma spans [median / 100, median * 100] (1.535 for the defaults, mean
    about 30 kb), redrawn outside [len_lo, len_hi]."""
    haps = pangenome_haplotypes(SEED + 2, genome_len, n_src)
    sigma = math.log(100.0) / 3.0
    contigs = []
    for c in range(n_contigs):
        g = rng(seed, STREAM_CONTIG + c)
        while True:
            L = int(round(math.exp(g.normal(math.log(median), sigma))))
            if len_lo <= L <= len_hi:
                break
        src = haps[int(g.integers(0, n_src))]
        L = min(L, src.shape[0])
        st = int(g.integers(0, src.shape[0] - L + 1))
        contigs.append(mutate(src[st:st + L], contig_snp, 0.0, g))
    chroms = []
    if n_chrom:
        base2 = random_genome(chrom_len, rng(seed, STREAM_SECOND_BASE))
        for h in range(n_chrom):
            chroms.append(haplotype(base2, 1e-3, 1e-4, rng(seed, STREAM_HAP + h)))
    return MergeWorkload("uneven", pack(haps[:n_b1]), pack(contigs + chroms))


@dataclasses.dataclass
class QueryWorkload:
    name: str
    index: Strings
    queries: Strings
    arrivals: np.ndarray | None = None


def config_serving(seed: int = SEED + 4, genome_len: int = 10_000_000,
                   n_index: int = 320, n_unseen: int = 64, n_queries: int = 10_000,
                   log_lo: float = 2.0, log_hi: float = 5.0, sub: float = 0.01,
                   indel: float = 0.001) -> QueryWorkload:
    """Serving: index = ``n_index`` haplotypes; queries are log-uniform-length
    excerpts of ``n_unseen`` other haplotypes with 1% substitutions and 0.1%
    1-5 bp indels."""
    base = random_genome(genome_len, rng(seed, STREAM_BASE))
    idx = haplotypes(base, seed, range(n_index))
    unseen = haplotypes(base, seed, range(n_index, n_index + n_unseen))
    qs = []
    for q in range(n_queries):
        g = rng(seed, STREAM_QUERY + q)
        L = int(10 ** g.uniform(log_lo, log_hi))
        src = unseen[int(g.integers(0, n_unseen))]
        L = max(1, min(L, src.shape[0]))
        st = int(g.integers(0, src.shape[0] - L + 1))
        qs.append(mutate(src[st:st + L], sub, indel, g))
    return QueryWorkload("serving", pack(idx), pack(qs))


def poisson_arrivals(n: int, rate_per_s: float, seed: int = SEED + 4) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    g = rng(seed, STREAM_ARRIVAL)
    return np.cumsum(g.exponential(1.0 / rate_per_s, n))


class IncrementalWorkload:
    """Large incremental build: a base genome with segmental duplications and
    inversions, and ``n_hap`` haplotypes of it, drawn on demand (haplotype h
    always from its own stream) so that batches need not all be in memory."""

    def __init__(self, seed: int, genome_len: int, n_hap: int, dup_frac: float, dup_lo: int,
                 dup_hi: int):
        self.seed = seed
        self.n_hap = n_hap
        base = random_genome(genome_len, rng(seed, STREAM_BASE))
        self.base = segmental_duplications(base, dup_frac, dup_lo, dup_hi, rng(seed, STREAM_BASE + 7))

    def haplotype(self, h: int) -> np.ndarray:
        return haplotype(self.base, 1e-3, 1e-4, rng(self.seed, STREAM_HAP + h))

    def batch(self, first: int, count: int) -> Strings:
        return pack(haplotypes(self.base, self.seed, range(first, first + count)))


def config_incremental(seed: int = SEED + 5, genome_len: int = 100_000_000,
                       n_hap: int = 100, dup_frac: float = 0.001, dup_lo: int = 1000,
                       dup_hi: int = 50_000) -> IncrementalWorkload:
    """Large incremental build (see IncrementalWorkload); merged in batches."""
    return IncrementalWorkload(seed, genome_len, n_hap, dup_frac, dup_lo, dup_hi)
