"""Pins for the CPU oracle: checks it against hand-worked values, the paper's
worked example, textbook routines, invariants and brute force on tiny inputs.

None of these tests needs a GPU. The brute-force helpers here are written
independently of ``oracle/oracle.c`` (pure Python over explicit tuples), so a
mistake in the oracle's sentinel order, symbol order, complement, interval
bounds or SMEM filter fails at least one of them.
"""
import itertools
import os
import random

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SYM = "$ACGTN"
CODE = {c: i for i, c in enumerate(SYM)}
COMP = {"A": "T", "C": "G", "G": "C", "T": "A", "N": "N"}


def _rc(s):
    return "".join(COMP[c] for c in reversed(s))


def _codes(strands):
    """Concatenate already-expanded strands into (codes, lens) directly."""
    data = np.array([CODE[c] for s in strands for c in s], dtype=np.uint8)
    lens = np.array([len(s) for s in strands], dtype=np.int64)
    return data, lens


def _bwt_str(B):
    return "".join(SYM[int(c)] for c in B)


# --- independent brute force (pure Python) --------------------------------

def _suffixes(strands):
    """Every suffix as a tuple of (kind, value): sentinel j -> (0, j), base c ->
    (1, rank of c in ACGTN). Returns list of (tuple, string index, offset)."""
    out = []
    for j, s in enumerate(strands):
        full = [(1, "ACGTN".index(c)) for c in s] + [(0, j)]
        for t in range(len(s) + 1):
            out.append((tuple(full[t:]), j, t))
    return out


def _brute_bwt(strands):
    suf = sorted(_suffixes(strands))
    m = len(strands)
    res = []
    for _, j, t in suf:
        if t == 0:
            res.append("$")          # preceded by the previous sentinel (T[-1] = T[n-1])
        else:
            res.append(strands[j][t - 1])
    assert len(res) == sum(len(s) + 1 for s in strands) and res.count("$") == m
    return "".join(res)


def _rotation_bwt(s):
    """Textbook Burrows-Wheeler transform of one string: sort every rotation of
    s + '$' ('$' smallest) and take the last column."""
    order = {c: i for i, c in enumerate("$ACGTN")}
    t = s + "$"
    rots = sorted((t[i:] + t[:i] for i in range(len(t))),
                  key=lambda r: [order[c] for c in r])
    return "".join(r[-1] for r in rots)


def _lf_decode(B, m):
    """Recover every string from a multi-string BWT by LF walks (Retrieve)."""
    cnt = {c: B.count(c) for c in SYM}
    C, acc = {}, 0
    for c in SYM:
        C[c] = acc
        acc += cnt[c]
    out = []
    for j in range(m):
        k, s = j, []
        while B[k] != "$":
            a = B[k]
            s.append(a)
            k = C[a] + B[:k].count(a)
        out.append("".join(reversed(s)))
    return out


def _brute_interval(strands, P):
    key = [(1, "ACGTN".index(c)) for c in P]
    suf = sorted(x[0] for x in _suffixes(strands))
    lo = sum(1 for s in suf if list(s[:len(key)]) < key and list(s[:len(key)]) != key)
    occ = sum(1 for s in suf if list(s[:len(key)]) == key)
    return lo, lo + occ


def _brute_smem(strands, P, min_len):
    """SMEMs from the MEM-containment definition (Sec. 2.6): enumerate every
    maximal exact match (text offset, pattern offset, length) over all strands,
    keep pattern intervals not contained in another MEM's interval."""
    mems = set()
    for s in strands:
        for t in range(len(s)):
            for p in range(len(P)):
                if s[t] != P[p]:
                    continue
                if t > 0 and p > 0 and s[t - 1] == P[p - 1]:
                    continue  # extendable to the left
                L = 0
                while t + L < len(s) and p + L < len(P) and s[t + L] == P[p + L]:
                    L += 1
                mems.add((p, p + L))
    smems = [iv for iv in mems
             if not any(o != iv and o[0] <= iv[0] and iv[1] <= o[1] for o in mems)]
    smems = sorted(iv for iv in smems if iv[1] - iv[0] >= min_len)
    res = []
    for a, b in smems:
        sub = P[a:b]
        occ = sum(1 for s in strands for t in range(len(s) - len(sub) + 1) if s[t:t + len(sub)] == sub)
        res.append((a, b, occ))
    return res


def _occ(strands, sub):
    """Occurrences of sub over every strand (overlaps counted; a match never
    crosses a strand's end)."""
    return sum(1 for s in strands for t in range(len(s) - len(sub) + 1) if s[t:t + len(sub)] == sub)


def _brute_smem_occ(strands, P, min_len, smin):
    """SMEMs with a minimum occurrence count, from the containment definition
    (Sec. 2.6 with the min-occurrence threshold): among all pattern intervals
    [a, b) whose substring occurs at least smin times, keep those that no
    other such interval contains. No e(i) recurrence is used."""
    freq = [(a, b) for a in range(len(P)) for b in range(a + 1, len(P) + 1) if _occ(strands, P[a:b]) >= smin]
    keep = [iv for iv in freq
            if not any(o != iv and o[0] <= iv[0] and iv[1] <= o[1] for o in freq)]
    return sorted((a, b, _occ(strands, P[a:b])) for a, b in keep if b - a >= min_len)


def _pangenome_strands(rnd, n_hap, length, sub, with_n=False):
    base = "".join(rnd.choice("ACGT") for _ in range(length))
    haps = ["".join(c if rnd.random() > sub else rnd.choice("ACGT") for c in base) for _ in range(n_hap)]
    if with_n:
        haps = ["".join(c if rnd.random() > 0.03 else "N" for c in h) for h in haps]
    return base, [x for h in haps for x in (h, _rc(h))]


def _read_table(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append([x.strip() for x in line.split("|")])
    return rows


# --- expansion --------------------------------------------------------------

def test_expand_order_and_complement():
    data = np.frombuffer(b"ACGTNacg", dtype=np.uint8)
    codes, lens = oracle.expand(data, np.array([5, 3]))
    assert list(lens) == [5, 5, 3, 3]
    got = _bwt_str(codes)
    assert got == "ACGTN" + "NACGT" + "ACG" + "CGT"


def test_expand_rejects_bad_bytes_and_empty():
    with pytest.raises(ValueError):
        oracle.expand(np.frombuffer(b"ACXT", dtype=np.uint8), np.array([4]))
    with pytest.raises(ValueError):
        oracle.expand(np.frombuffer(b"ACGT", dtype=np.uint8), np.array([0, 4]))


# --- BWT --------------------------------------------------------------------

def test_bwt_hand_worked():
    for strands, want, _ in _read_table("bwt_hand.txt"):
        codes, lens = _codes(strands.split(","))
        B = oracle.bwt(codes, lens, nthreads=1)
        assert _bwt_str(B) == want, strands


def test_bwt_double_strand_hand_worked_from_expand():
    codes, lens = oracle.expand(np.frombuffer(b"AC", dtype=np.uint8), np.array([2]))
    assert _bwt_str(oracle.bwt(codes, lens)) == "CT$A$G"
    codes, lens = oracle.expand(np.frombuffer(b"AN", dtype=np.uint8), np.array([2]))
    assert _bwt_str(oracle.bwt(codes, lens)) == "NT$NA$"


def test_bwt_single_string_is_textbook_rotation_sort():
    rnd = random.Random(7)
    for _ in range(300):
        s = "".join(rnd.choice("ACGTN" if rnd.random() < 0.3 else "ACGT")
                    for _ in range(rnd.randint(1, 40)))
        codes, lens = _codes([s])
        assert _bwt_str(oracle.bwt(codes, lens, nthreads=1)) == _rotation_bwt(s), s


def test_bwt_exhaustive_tiny_lists():
    """Every list of 1-2 strings of length 1-3 over ACGT (and a sample of
    3-string lists with N) against the pure-Python suffix sort."""
    words = ["".join(w) for L in (1, 2, 3) for w in itertools.product("ACGT", repeat=L)]
    lists = [[w] for w in words] + [[a, b] for a in words for b in words]
    rnd = random.Random(11)
    for _ in range(1500):
        lists.append(["".join(rnd.choice("ACGTN") for _ in range(rnd.randint(1, 3)))
                      for _ in range(3)])
    for strands in lists:
        codes, lens = _codes(strands)
        B = _bwt_str(oracle.bwt(codes, lens, nthreads=1))
        assert B == _brute_bwt(strands), strands


def test_bwt_random_lists_brute_and_lf_decode():
    rnd = random.Random(3)
    for _ in range(200):
        raw = ["".join(rnd.choice("ACGT") for _ in range(rnd.randint(1, 12)))
               for _ in range(rnd.randint(1, 5))]
        strands = [x for s in raw for x in (s, _rc(s))]
        codes, lens = _codes(strands)
        B = _bwt_str(oracle.bwt(codes, lens, nthreads=2))
        assert B == _brute_bwt(strands)
        assert _lf_decode(B, len(strands)) == strands


def test_bwt_parallel_sort_matches_serial():
    rnd = random.Random(5)
    strands = ["".join(rnd.choice("ACGT") for _ in range(rnd.randint(50, 400))) for _ in range(40)]
    strands += strands[:10]  # exact duplicates: ties broken only by sentinels
    codes, lens = _codes(strands)
    assert np.array_equal(oracle.bwt(codes, lens, nthreads=1), oracle.bwt(codes, lens, nthreads=7))


def test_bwt_symbol_counts_and_sentinel_rows():
    rnd = random.Random(9)
    strands = ["".join(rnd.choice("ACGTN") for _ in range(rnd.randint(1, 30))) for _ in range(25)]
    codes, lens = _codes(strands)
    B = oracle.bwt(codes, lens)
    assert int((B == 0).sum()) == len(strands)
    for c in range(1, 6):
        assert int((B == c).sum()) == int((codes == c).sum())
    # row j < m holds the suffix $_j, so B[j] is the last symbol of string j
    for j, s in enumerate(strands):
        assert SYM[B[j]] == s[-1]


# --- inverse-BWT verifier ---------------------------------------------------

def test_verify_accepts_true_bwt_and_rejects_every_transposition():
    rnd = random.Random(13)
    for _ in range(60):
        strands = ["".join(rnd.choice("ACGT") for _ in range(rnd.randint(1, 6)))
                   for _ in range(rnd.randint(1, 4))]
        codes, lens = _codes(strands)
        B = oracle.bwt(codes, lens)
        assert oracle.verify(B, codes, lens) == 0
        n = B.shape[0]
        for i in range(n):
            for j in range(i + 1, n):
                if B[i] != B[j]:
                    X = B.copy()
                    X[i], X[j] = X[j], X[i]
                    assert oracle.verify(X, codes, lens) != 0, (strands, i, j)


def test_verifier_in_parts_agrees_with_verify():
    # walking the strings one at a time reports the same first failing
    # string as the one-call check, on the true BWT and on every transposition
    rnd = random.Random(17)
    for _ in range(25):
        strands = ["".join(rnd.choice("ACGT") for _ in range(rnd.randint(1, 5)))
                   for _ in range(rnd.randint(1, 4))]
        codes, lens = _codes(strands)
        B = oracle.bwt(codes, lens)
        n = B.shape[0]
        cases = [B]
        for i in range(n):
            for j in range(i + 1, n):
                if B[i] != B[j]:
                    X = B.copy()
                    X[i], X[j] = X[j], X[i]
                    cases.append(X)
        for X in cases:
            want = oracle.verify(X, codes, lens)
            v = oracle.Verifier(X, codes, lens)
            if v.status != 0:
                assert v.status == want
                continue
            bad = [r for r in (v.walk(j, j + 1) for j in range(lens.shape[0])) if r]
            got = min(bad) if bad else 0
            assert got == want and v.walk(0, lens.shape[0], nthreads=3) == want
            v.close()
    v = oracle.Verifier(B[:-1], codes, lens)
    assert v.status == -1


def test_verify_rejects_wrong_length_and_counts():
    codes, lens = _codes(["ACGT", "GG"])
    B = oracle.bwt(codes, lens)
    assert oracle.verify(B[:-1], codes, lens) == -1
    X = B.copy()
    X[X != 0] = 1
    assert oracle.verify(X, codes, lens) == -2


# --- counts -----------------------------------------------------------------

def test_count_hand_worked():
    for strands, pat, lo, hi in _read_table("count_hand.txt"):
        codes, lens = _codes(strands.split(","))
        P = "" if pat == "-" else pat
        q = np.array([CODE[c] for c in P], dtype=np.uint8)
        glo, ghi = oracle.count(codes, lens, q, np.array([len(P)]))
        assert (int(glo[0]), int(ghi[0])) == (int(lo), int(hi)), (strands, pat)


def test_count_brute_force_and_strand_symmetry():
    rnd = random.Random(17)
    raw = ["".join(rnd.choice("ACGT") for _ in range(rnd.randint(5, 25))) for _ in range(6)]
    strands = [x for s in raw for x in (s, _rc(s))]
    codes, lens = _codes(strands)
    pats = [s[a:a + L] for s in raw for a in range(0, len(s) - 3, 3) for L in (1, 2, 4)]
    pats += ["".join(rnd.choice("ACGT") for _ in range(rnd.randint(1, 5))) for _ in range(40)]
    qc = np.array([CODE[c] for p in pats for c in p], dtype=np.uint8)
    ql = np.array([len(p) for p in pats], dtype=np.int64)
    lo, hi = oracle.count(codes, lens, qc, ql, nthreads=3)
    text = oracle.Text(codes, lens)
    for i, p in enumerate(pats):
        assert (lo[i], hi[i]) == _brute_interval(strands, p), p
        assert text.interval(np.array([CODE[c] for c in p], np.uint8)) == (lo[i], hi[i])
    # occ(P) = occ(rc P) on a double-strand list (Sec. 2.5)
    rcq = np.array([CODE[c] for p in pats for c in _rc(p)], dtype=np.uint8)
    lo2, hi2 = oracle.count(codes, lens, rcq, ql)
    assert np.array_equal(hi - lo, hi2 - lo2)


# --- SMEMs ------------------------------------------------------------------

def _smem_fixture():
    d = {}
    with open(os.path.join(GOLD, "smem_paper_example.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, *v = line.split()
                d[k] = v
    return d


@pytest.mark.parametrize("both", [False, True])
def test_smem_paper_example(both):
    fx = _smem_fixture()
    T, P = fx["text"][0], fx["pattern"][0]
    a, b, toff = map(int, fx["smem"])
    assert T[toff:toff + (b - a)] == P[a:b]
    strands = [T, _rc(T)] if both else [T]
    codes, lens = _codes(strands)
    text = oracle.Text(codes, lens)
    q = np.array([CODE[c] for c in P], np.uint8)
    for min_len in (1, 2, 3, 4):
        got = text.smem(q, min_len, 1)
        assert [tuple(r[:2]) for r in got] == [(a, b)]
        assert got[0][2] == 1
    na, nb, _ = map(int, fx["not_smem"])
    assert all(tuple(r[:2]) != (na, nb) for r in text.smem(q, 1, 1))
    assert len(text.smem(q, 5, 1)) == 0


def test_smem_brute_force_mem_containment():
    rnd = random.Random(23)
    for trial in range(120):
        raw = ["".join(rnd.choice("ACGT") for _ in range(rnd.randint(3, 14)))
               for _ in range(rnd.randint(1, 3))]
        strands = [x for s in raw for x in (s, _rc(s))]
        codes, lens = _codes(strands)
        text = oracle.Text(codes, lens)
        src = rnd.choice(raw)
        P = "".join(c if rnd.random() > 0.2 else rnd.choice("ACGT") for c in src)
        P += "".join(rnd.choice("ACGT") for _ in range(rnd.randint(0, 4)))
        q = np.array([CODE[c] for c in P], np.uint8)
        for min_len in (1, 2, 3):
            got = [tuple(int(x) for x in r[:3]) for r in text.smem(q, min_len, 1)]
            assert got == _brute_smem(strands, P, min_len), (strands, P, min_len)


def test_smem_intervals_and_bi_interval_symmetry():
    rnd = random.Random(29)
    raw = ["".join(rnd.choice("ACGT") for _ in range(60)) for _ in range(4)]
    strands = [x for s in raw for x in (s, _rc(s))]
    codes, lens = _codes(strands)
    text = oracle.Text(codes, lens)
    P = raw[1][5:40] + "T" + raw[2][10:50]
    q = np.array([CODE[c] for c in P], np.uint8)
    rows = text.smem(q, 5, 1)
    assert len(rows) >= 2
    for a, b, occ, k, krc in rows:
        sub = P[a:b]
        lo, hi = _brute_interval(strands, sub)
        lo2, hi2 = _brute_interval(strands, _rc(sub))
        # (k, k', s) is the bi-interval of P[a,b); swapping gives rc's (Sec. 2.5)
        assert (k, occ, krc) == (lo, hi - lo, lo2) and hi2 - lo2 == occ


def test_smem_min_occ():
    """With min_occ > 1 each reported match occurs that often and cannot be
    extended on either side without falling below it."""
    rnd = random.Random(31)
    raw = ["".join(rnd.choice("ACGT") for _ in range(40)) for _ in range(3)]
    raw.append(raw[0][:25] + "".join(rnd.choice("ACGT") for _ in range(15)))
    strands = [x for s in raw for x in (s, _rc(s))]
    codes, lens = _codes(strands)
    text = oracle.Text(codes, lens)
    P = raw[0]
    q = np.array([CODE[c] for c in P], np.uint8)
    for smin in (1, 2, 3):
        rows = text.smem(q, 1, smin)
        for a, b, occ, _, _ in rows:
            assert occ >= smin
            if b < len(P):
                lo, hi = _brute_interval(strands, P[a:b + 1])
                assert hi - lo < smin
            if a > 0:
                lo, hi = _brute_interval(strands, P[a - 1:b])
                assert hi - lo < smin


def test_smem_brute_force_min_occ():
    """orc_smem at min_occ 2 and 3 against the containment definition, with
    occ, lo and lo_rc from brute-force intervals: a dropped or misplaced SMEM,
    a wrong count or a wrong interval fails here."""
    rnd = random.Random(41)
    cases = 0
    for trial in range(60):
        base, strands = _pangenome_strands(rnd, rnd.randint(2, 4), rnd.randint(6, 16), 0.15)
        codes, lens = _codes(strands)
        text = oracle.Text(codes, lens)
        P = "".join(c if rnd.random() > 0.15 else rnd.choice("ACGT") for c in base)
        P = "".join(rnd.choice("ACGT") for _ in range(rnd.randint(0, 2))) + P
        q = np.array([CODE[c] for c in P], np.uint8)
        for smin in (2, 3):
            for min_len in (1, 2, 3):
                want = _brute_smem_occ(strands, P, min_len, smin)
                got = text.smem(q, min_len, smin)
                assert [tuple(int(x) for x in r[:3]) for r in got] == want, (strands, P, min_len, smin)
                for a, b, occ, k, krc in got:
                    assert (k, k + occ) == _brute_interval(strands, P[a:b])
                    assert (krc, krc + occ) == _brute_interval(strands, _rc(P[a:b]))
                cases += len(want)
    assert cases > 100


# --- batched intervals and the seeded SMEM scan --------------------------------

def _scan_patterns(rnd, strands, n, k=oracle.SCAN_K):
    """Patterns at least k long whose first k symbols are A..T: excerpts of
    the strands (some running past a strand's end, some mutated) and random
    strings."""
    out = []
    while len(out) < n:
        if rnd.random() < 0.75:
            s = rnd.choice(strands)
            if len(s) < 2:
                continue
            t = rnd.randrange(len(s))
            L = rnd.randint(k, k + 25)
            p = s[t:t + L]
            if len(p) < L and rnd.random() < 0.5:
                p += "".join(rnd.choice("ACGT") for _ in range(L - len(p)))
            if rnd.random() < 0.3:
                p = "".join(c if rnd.random() > 0.1 else rnd.choice("ACGT") for c in p)
        else:
            p = "".join(rnd.choice("ACGTN" if i >= k else "ACGT") for i in range(rnd.randint(k, k + 10)))
        if len(p) >= k and all(c in "ACGT" for c in p[:k]):
            out.append(p)
    return out


def test_scan_intervals_brute_force():
    """scan_intervals against pure-Python intervals on small lists, with N in
    the text, patterns that run past strand ends, duplicates and prefixes of
    one another."""
    rnd = random.Random(43)
    for trial in range(25):
        _, strands = _pangenome_strands(rnd, rnd.randint(1, 4), rnd.randint(10, 45), 0.05, with_n=trial % 2 == 0)
        strands += ["".join(rnd.choice("ACGT") for _ in range(rnd.randint(1, 14)))]
        pats = _scan_patterns(rnd, strands, 40)
        pats += [pats[0], pats[1] + "A", pats[1] + "T", pats[2][:oracle.SCAN_K]]
        codes, lens = _codes(strands)
        pc, pl = _codes(pats)
        lo, hi = oracle.scan_intervals(codes, lens, pc, pl)
        for i, p in enumerate(pats):
            assert (int(lo[i]), int(hi[i])) == _brute_interval(strands, p), (strands, p)


def test_scan_intervals_equals_count():
    """On a larger pangenome-like list, the one-pass intervals equal the
    per-pattern scan of orc_count."""
    rnd = random.Random(47)
    _, strands = _pangenome_strands(rnd, 16, 3000, 0.01, with_n=True)
    pats = _scan_patterns(rnd, strands, 3000)
    codes, lens = _codes(strands)
    pc, pl = _codes(pats)
    lo, hi = oracle.scan_intervals(codes, lens, pc, pl, nthreads=3)
    lo2, hi2 = oracle.count(codes, lens, pc, pl)
    assert np.array_equal(lo, lo2) and np.array_equal(hi, hi2)
    assert (hi - lo).max() >= 8


def test_scan_intervals_precondition():
    codes, lens = _codes(["ACGTACGTACGTACGT"])
    for bad in ("ACGTACGTACG", "ACGTNCGTACGTA"):
        pc, pl = _codes([bad])
        with pytest.raises(ValueError):
            oracle.scan_intervals(codes, lens, pc, pl)


def test_smem_scan_brute_force():
    """The seeded scan against the containment definition directly (pure
    Python) at min_len 12 and 13, min_occ 1-3."""
    rnd = random.Random(53)
    total = 0
    for trial in range(12):
        base, strands = _pangenome_strands(rnd, rnd.randint(2, 4), rnd.randint(20, 34), 0.04)
        P = "".join(c if rnd.random() > 0.04 else rnd.choice("ACGT") for c in base)
        codes, lens = _codes(strands)
        q = np.array([CODE[c] for c in P], np.uint8)
        for smin in (1, 2, 3):
            for min_len in (12, 13):
                recs, off = oracle.smem_scan(codes, lens, q, np.array([len(P)], np.int64), min_len, smin)
                want = _brute_smem_occ(strands, P, min_len, smin)
                assert [tuple(int(x) for x in r[:3]) for r in recs] == want, (strands, P, min_len, smin)
                for a, b, occ, k, krc in recs:
                    assert (k, k + occ) == _brute_interval(strands, P[a:b])
                    assert (krc, krc + occ) == _brute_interval(strands, _rc(P[a:b]))
                total += len(want)
    assert total > 20


def test_smem_scan_equals_text_smem():
    """On pangenome-like lists (the shape the scan is used on), the scan's
    SMEMs equal Text.smem's, for several min_len and min_occ."""
    import synth
    base = synth.random_genome(6000, synth.rng(61, 0))
    haps = [synth.haplotype(base, 5e-3, 1e-3, synth.rng(61, 1 + h)) for h in range(10)]
    S = synth.pack(haps)
    codes, lens = oracle.expand(S.data, S.lens)
    text = oracle.Text(codes, lens)
    unseen = [synth.haplotype(base, 5e-3, 1e-3, synth.rng(61, 100 + h)) for h in range(3)]
    g = np.random.default_rng(61)
    qs = []
    for k in range(30):
        h = unseen[k % 3]
        L = int(g.integers(40, 1500))
        st = int(g.integers(0, len(h) - L))
        q = synth.mutate(h[st:st + L].copy(), 0.01, 0.001, synth.rng(62, k))
        if k % 2:  # half of them from the other strand
            q = np.frombuffer(bytes(q[::-1]).translate(bytes.maketrans(b"ACGT", b"TGCA")), np.uint8)
        qs.append(q)
    Q = synth.pack(qs)
    qc, ql = oracle.encode(Q.data, Q.lens)
    qo = np.concatenate([[0], np.cumsum(ql)])
    total = 0
    for min_len, smin in ((12, 1), (15, 2), (20, 3), (31, 1), (31, 2)):
        recs, off = oracle.smem_scan(codes, lens, qc, ql, min_len, smin, nthreads=4)
        for i in range(len(qs)):
            want = text.smem(qc[qo[i]:qo[i + 1]], min_len, smin)
            assert np.array_equal(recs[off[i]:off[i + 1]], want), (i, min_len, smin)
            total += len(want)
    assert total > 500


def test_smem_scan_precondition():
    codes, lens = _codes(["ACGTACGTACGTACGTACGT", "ACGTACGTACGTACGTACGT"])
    q = np.array([CODE[c] for c in "ACGTACGTACGTACGT"], np.uint8)
    with pytest.raises(ValueError):
        oracle.smem_scan(codes, lens, q, np.array([16], np.int64), 11, 1)


# --- insertion ranks ----------------------------------------------------------

def test_insertion_ranks_brute_force():
    rnd = random.Random(37)
    for _ in range(40):
        old = [x for s in ["".join(rnd.choice("ACGT") for _ in range(rnd.randint(1, 8)))
                           for _ in range(rnd.randint(1, 3))] for x in (s, _rc(s))]
        new = [x for s in ["".join(rnd.choice("ACGT") for _ in range(rnd.randint(1, 8)))
                           for _ in range(rnd.randint(1, 3))] for x in (s, _rc(s))]
        codes, lens = _codes(old + new)
        _, S = oracle.bwt(codes, lens, want_sa=True)
        l = oracle.insertion_ranks(S, lens, len(old))
        old_suf = [x[0] for x in _suffixes(old)]
        allsuf = _suffixes(old + new)
        k = 0
        for j in range(len(old), len(old) + len(new)):
            for t in range(len(new[j - len(old)]) + 1):
                x = [s for s in allsuf if s[1] == j and s[2] == t][0][0]
                # old sentinels are $0..$(m1-1) in both lists, so tuples compare directly
                assert l[k] == sum(1 for y in old_suf if y < x)
                k += 1
        # a new sentinel suffix is above exactly the m1 old sentinels (Algorithm 1 starts l at m1)
        off = 0
        for s in new:
            off += len(s)
            assert l[off] == len(old)
            off += 1


# --- locate (suffix-array positions) -------------------------------------------

def test_locate_hand_worked():
    for strands, want, _ in _read_table("locate_hand.txt"):
        codes, lens = _codes(strands.split(","))
        _, S = oracle.bwt(codes, lens, nthreads=1, want_sa=True)
        j, off = oracle.locate(S, lens, np.arange(S.shape[0]))
        got = " ".join(f"{a}:{b}" for a, b in zip(j, off))
        assert got == want, strands


def test_locate_brute_force_and_inverse():
    """Every row's position against the pure-Python suffix sort, and rows_of
    as its inverse."""
    rnd = random.Random(41)
    for _ in range(150):
        strands = ["".join(rnd.choice("ACGTN") for _ in range(rnd.randint(1, 9)))
                   for _ in range(rnd.randint(1, 5))]
        codes, lens = _codes(strands)
        _, S = oracle.bwt(codes, lens, want_sa=True)
        j, off = oracle.locate(S, lens, np.arange(S.shape[0]))
        want = [(x[1], x[2]) for x in sorted(_suffixes(strands))]
        assert list(zip(j.tolist(), off.tolist())) == want
        assert np.array_equal(oracle.rows_of(S, lens, j, off), np.arange(S.shape[0]))


def test_locate_follows_lf_on_the_bwt():
    """LF on the BWT alone (pi(r) = C(B[r]) + rank(B[r], r), Table 1) moves a
    row to the suffix one position earlier in the same string; rows whose BWT
    symbol is $ hold offset 0. This ties locate to B, not to the sort."""
    rnd = random.Random(43)
    for _ in range(60):
        raw = ["".join(rnd.choice("ACGT") for _ in range(rnd.randint(1, 30)))
               for _ in range(rnd.randint(1, 6))]
        strands = [x for s in raw for x in (s, _rc(s))]
        codes, lens = _codes(strands)
        B, S = oracle.bwt(codes, lens, want_sa=True)
        n = B.shape[0]
        C = [int((B < c).sum()) for c in range(6)]
        j, off = oracle.locate(S, lens, np.arange(n))
        for r in range(n):
            c = int(B[r])
            if c == 0:
                assert off[r] == 0
                continue
            assert off[r] > 0 and strands[j[r]][off[r] - 1] == SYM[c]
            pr = C[c] + int((B[:r] == c).sum())
            assert (j[pr], off[pr]) == (j[r], off[r] - 1)
