"""Pins of the oracle's local haplotype enumeration (hapl.c; Sec. 2.7-2.8):
the DAWG recurrences of Algorithm 5 against a brute force over every
substring of the text (a plain string-against-string dynamic program with
the same scores and the same rule that only positive cells are kept, whose
best score per SA interval must equal the DAWG cell's), exact and mutated
queries against hand-derived scores, the band as a restriction, and the
redundancy filter against its definition."""
import numpy as np
import pytest

import oracle
import synth

MATCH, MIS, GO, GE = 1, 4, 6, 1
DEFAULT = (MATCH, MIS, GO, GE)
NEG = -10 ** 9


def _string_score(P, S, sc=DEFAULT):
    """Best score of P (whole) against S (whole), P and S read from their
    ends, keeping only positive cells (the start cell has score 0)."""
    MATCH, MIS, GO, GE = sc
    m, L = len(P), len(S)
    H = [[NEG] * (L + 1) for _ in range(m + 1)]
    E = [[NEG] * (L + 1) for _ in range(m + 1)]
    F = [[NEG] * (L + 1) for _ in range(m + 1)]
    H[m][L] = 0

    def ok(i, j):
        return (i == m and j == L) or H[i][j] > 0

    for i in range(m - 1, -1, -1):
        for j in range(L, -1, -1):
            g = e = f = NEG
            if j < L and ok(i + 1, j + 1):
                g = H[i + 1][j + 1] + (MATCH if P[i] == S[j] else -MIS)
            if ok(i + 1, j):
                e = max(H[i + 1][j] - GO, E[i + 1][j]) - GE
            if j < L and ok(i, j + 1):
                f = max(H[i][j + 1] - GO, F[i][j + 1]) - GE
            E[i][j], F[i][j] = e, f
            H[i][j] = max(g, e, f)
    return H[0][0] if H[0][0] > 0 else None


COMP = np.array([0, 4, 3, 2, 1, 5], np.uint8)


def _brute(text, codes, lens, P, sc=DEFAULT, with_rc=False):
    """{(k, s): best score} over every substring S of every strand; with_rc:
    {(k, s): (best score, the smallest and the largest start of the reverse
    complement's SA interval among the strings S of the node attaining it)}."""
    MATCH, MIS, GO, GE = sc
    best = {}
    # a deletion run of length d costs GO + d * GE and the best score is
    # len(P) * MATCH, so no positive alignment holds more text symbols
    maxlen = len(P) + max(0, len(P) * MATCH - GO) // GE + 1
    seen = set()
    starts = np.concatenate([[0], np.cumsum(lens)])
    for st in range(len(lens)):
        a0, a1 = int(starts[st]), int(starts[st + 1])
        for a in range(a0, a1):
            for L in range(1, min(maxlen, a1 - a) + 1):
                S = bytes(codes[a:a + L])
                if S in seen:
                    continue
                seen.add(S)
                v = _string_score(P, S, sc)
                if v is None:
                    continue
                arr = np.frombuffer(S, np.uint8)
                k, hi = text.interval(arr)
                key = (k, hi - k)
                if with_rc:
                    krc, _ = text.interval(COMP[arr[::-1]])
                    krc = int(krc)
                    old = best.get(key)
                    if old is None or v > old[0]:
                        best[key] = (v, krc, krc)
                    elif v == old[0]:
                        best[key] = (v, min(old[1], krc), max(old[2], krc))
                else:
                    best[key] = max(best.get(key, NEG), v)
    return best


def _text(seed, nstr=3, length=40):
    g = np.random.default_rng(seed)
    acgt = np.frombuffer(b"ACGT", np.uint8)
    base = acgt[g.integers(0, 4, length)]
    strs = []
    for _ in range(nstr):
        s = base.copy()
        s[g.integers(0, length, 2)] = acgt[g.integers(0, 4, 2)]
        strs.append(s.tobytes())
    w = synth.pack(strs)
    codes, lens = oracle.expand(w.data, w.lens)
    return oracle.Text(codes, lens), codes, lens


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_hapl_dawg_equals_brute_force(seed):
    text, codes, lens = _text(seed)
    g = np.random.default_rng(100 + seed)
    for trial in range(6):
        L = int(g.integers(5, 9))
        a = int(g.integers(0, codes.shape[0] - L))
        P = codes[a:a + L].copy()
        P[P == 0] = 1
        if trial % 3 == 1:
            P[int(g.integers(0, L))] = int(g.integers(1, 5))  # a substitution
        elif trial % 3 == 2:
            P = np.delete(P, int(g.integers(1, L - 1)))  # an indel relative to the text
        want = _brute(text, codes, lens, P)
        got = text.hapl(P, MATCH, MIS, GO, GE, band=0, raw=True)
        gotd = {(int(r[0]), int(r[2])): int(r[3]) for r in got}
        assert gotd == want, (seed, trial, P)
        # every reverse-complement interval is the one of the string's reverse complement
        for r in got:
            assert r[1] >= 0 and r[1] + r[2] <= text.n


@pytest.mark.parametrize("scores", [(2, 3, 5, 2), (3, 1, 2, 3), (2, 1, 1, 1)])
def test_hapl_dawg_equals_brute_force_other_scores(scores):
    # the score sets of the GPU parity tests: cheap gaps and mismatches make
    # deletion chains, insertions and ties that the default scores rarely do
    text, codes, lens = _text(21, nstr=3, length=24)
    g = np.random.default_rng(31)
    for trial in range(4):
        L = int(g.integers(4, 7))
        a = int(g.integers(0, codes.shape[0] - L))
        P = codes[a:a + L].copy()
        P[P == 0] = 1
        if trial % 2 == 1:
            P[int(g.integers(0, L))] = int(g.integers(1, 5))
        want = _brute(text, codes, lens, P, scores)
        got = text.hapl(P, *scores, band=0, raw=True)
        assert {(int(r[0]), int(r[2])): int(r[3]) for r in got} == want, (scores, trial, P)


@pytest.mark.parametrize("scores", [(2, 1, 1, 1), (3, 1, 2, 3)])
def test_hapl_representative_brute_force(scores):
    # a node holds several strings (X and XZ when every X is followed by Z),
    # whose reverse complements have intervals of one size but different
    # starts: the reported k' is that of the string with the smallest start
    # among the node's strings whose own alignment attains the node's score
    text, codes, lens = _text(41, nstr=3, length=24)
    g = np.random.default_rng(43)
    chosen = 0
    for trial in range(5):
        L = int(g.integers(4, 8))
        a = int(g.integers(0, codes.shape[0] - L))
        P = codes[a:a + L].copy()
        P[P == 0] = 2
        if trial % 2 == 1:
            P[int(g.integers(0, L))] = int(g.integers(1, 5))
        want = _brute(text, codes, lens, P, scores, with_rc=True)
        got = text.hapl(P, *scores, band=0, raw=True)
        assert {(int(r[0]), int(r[2])): (int(r[3]), int(r[1])) for r in got} == \
            {key: (v[0], v[1]) for key, v in want.items()}, (scores, trial, P)
        chosen += sum(1 for v in want.values() if v[1] != v[2])
    # nodes whose optimal strings' reverse complements start at different
    # rows, where the choice is made
    assert chosen > 0


@pytest.mark.parametrize("seed,scores,query", [(40, (2, 1, 1, 1), [2, 1, 2, 3, 3, 4]),
                                               (41, (4, 2, 3, 1), [1, 2, 1, 3])])
def test_hapl_gap_representative_brute_force(seed, scores, query):
    # inputs where a cell's best score comes from an insertion or deletion
    # run whose own string is not the representative of the score it left:
    # the gap passes on the run's representative (a gap that passed on H's
    # representative fails here)
    text, codes, lens = _text(seed, nstr=3, length=24)
    P = np.array(query, np.uint8)
    want = _brute(text, codes, lens, P, scores, with_rc=True)
    got = text.hapl(P, *scores, band=0, raw=True)
    assert {(int(r[0]), int(r[2])): (int(r[3]), int(r[1])) for r in got} == \
        {key: (v[0], v[1]) for key, v in want.items()}


def test_hapl_band_tie_break():
    # AC and GC both align to the query TC with one match and one mismatch
    # that costs nothing (mismatch score 0): their cells tie at score 1. A
    # band of one keeps the cell whose suffix-array interval starts first
    # (AC before GC), the band's order being score, then smaller k, then
    # smaller s.
    enc = {c: i + 1 for i, c in enumerate(b"ACGTN")}
    w = synth.pack([b"AC", b"GC"])
    codes, lens = oracle.expand(w.data, w.lens)
    text = oracle.Text(codes, lens)

    def iv(s):
        return text.interval(np.array([enc[c] for c in s], np.uint8))

    ac, gc, gt = iv(b"AC"), iv(b"GC"), iv(b"GT")
    assert ac[0] < gc[0]
    P = np.array([enc[c] for c in b"TC"], np.uint8)
    rows = lambda r: [tuple(int(v) for v in x) for x in r]
    # GC is its own reverse complement: it occurs once on each strand
    assert rows(text.hapl(P, 1, 0, 6, 1, band=0)) == [(ac[0], gt[0], 1, 1), (gc[0], gc[0], 2, 1)]
    assert rows(text.hapl(P, 1, 0, 6, 1, band=1)) == [(ac[0], gt[0], 1, 1)]


def test_hapl_hand_scores():
    text, codes, _ = _text(7, nstr=2, length=60)
    P = codes[10:40].copy()
    k, hi = text.interval(P)
    res = text.hapl(P, MATCH, MIS, GO, GE, band=25)
    assert (int(res[0, 0]), int(res[0, 2]), int(res[0, 3])) == (k, hi - k, 30)
    # one substitution: 29 matches and a mismatch
    Q = P.copy()
    Q[15] = Q[15] % 4 + 1
    res = text.hapl(Q, MATCH, MIS, GO, GE, band=25)
    assert int(res[0, 3]) == 29 - MIS
    # a deleted query symbol: 29 matches and one text symbol deleted
    D = np.delete(P, 15)
    res = text.hapl(D, MATCH, MIS, GO, GE, band=25)
    assert int(res[0, 3]) == 29 - GO - GE
    # an empty query matches nothing
    assert text.hapl(np.zeros(0, np.uint8), band=25).shape[0] == 0


def test_hapl_band_restricts():
    text, codes, _ = _text(11, nstr=4, length=50)
    g = np.random.default_rng(5)
    for _ in range(8):
        a = int(g.integers(0, codes.shape[0] - 12))
        P = codes[a:a + 12].copy()
        P[P == 0] = 2
        P[int(g.integers(0, 12))] = int(g.integers(1, 5))
        full = {(int(r[0]), int(r[2])): int(r[3]) for r in text.hapl(P, band=0, raw=True)}
        # a wide band changes nothing; a narrow one keeps a subset with scores no higher
        wide = {(int(r[0]), int(r[2])): int(r[3]) for r in text.hapl(P, band=100000, raw=True)}
        assert wide == full
        for band in (1, 2, 5):
            res = text.hapl(P, band=band, raw=True)
            assert len(res) <= band
            for r in res:
                key = (int(r[0]), int(r[2]))
                assert key in full and int(r[3]) <= full[key]
        # raw rows come by decreasing score, then smaller k, then smaller s
        raw = text.hapl(P, band=0, raw=True)
        order = sorted(range(len(raw)), key=lambda x: (-raw[x, 3], raw[x, 0], raw[x, 2]))
        assert order == list(range(len(raw)))


def test_hapl_filter_definition():
    text, codes, _ = _text(13, nstr=5, length=45)
    g = np.random.default_rng(9)
    for _ in range(8):
        a = int(g.integers(0, codes.shape[0] - 10))
        P = codes[a:a + 10].copy()
        P[P == 0] = 3
        raw = text.hapl(P, band=0, raw=True)
        kept = []
        for r in raw:
            inside = any((r[0] >= q[0] and r[0] + r[2] <= q[0] + q[2]) or
                         (r[1] >= q[1] and r[1] + r[2] <= q[1] + q[2]) for q in kept)
            if not inside:
                kept.append(r)
        got = text.hapl(P, band=0)
        assert np.array_equal(got, np.array(kept, np.int64).reshape(-1, 4))
