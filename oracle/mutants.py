"""Strength of the oracle's pins: plausible one-line mistakes, each applied
to a temporary copy of the oracle's C sources, must make at least one of the
CPU pins (tests/test_oracle*.py) fail.

Test infrastructure, run by hand (a few minutes, not part of the test
suite):

    python oracle/mutants.py [NAME ...]

Each mutant is built with gcc into a temporary directory and the pins run in
a child process with the oracle's library path pointed at it; the real
sources and liboracle.so are never touched. Exit status 1 if any mutant
passes every pin.
"""
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = ("oracle.c", "rle.c", "hapl.c")
PINS = ("tests/test_oracle.py", "tests/test_oracle_rle.py", "tests/test_oracle_hapl.py")

# (name, file, text, replacement, the mistake)
MUTANTS = [
    ("sentinel-order", "oracle.c", "T[p++] = (int32_t)j;", "T[p++] = (int32_t)(m - 1 - j);",
     "sentinels ordered by decreasing string index"),
    ("complement", "oracle.c", "static const uint8_t tab[6] = {0, 4, 3, 2, 1, 5};",
     "static const uint8_t tab[6] = {0, 3, 4, 1, 2, 5};", "A paired with G and C with T"),
    ("rc-not-reversed", "oracle.c", "codes[out + L + t] = orc_comp(codes[out + L - 1 - t]);",
     "codes[out + L + t] = orc_comp(codes[out + t]);", "the reverse strand complemented but not reversed"),
    ("bwt-first-row", "oracle.c", "int64_t p = S[i] == 0 ? n - 1 : S[i] - 1;",
     "int64_t p = S[i] == 0 ? 0 : S[i] - 1;", "the symbol before the text's first suffix"),
    ("sentinel-above-bases", "oracle.c", "        if (v < m) return -1;\n        int c = (int)(v - (m - 1));",
     "        if (v < m) return 1;\n        int c = (int)(v - (m - 1));", "a sentinel compared above a pattern base"),
    ("interval-end", "oracle.c", "if (orc_cmp_pattern(T, m, S[mid], P, len) <= 0) a = mid + 1; else b = mid;",
     "if (orc_cmp_pattern(T, m, S[mid], P, len) < 0) a = mid + 1; else b = mid;",
     "the interval's end searched as its start"),
    ("verifier-rank", "oracle.c", "    for (; i < k; ++i) r += (B[i] == c);", "    for (; i <= k; ++i) r += (B[i] == c);",
     "rank counting the symbol at k itself"),
    ("smem-contained", "oracle.c", "if ((i == 0 || e > eprev) && e - i >= min_len && e > i) {",
     "if ((i == 0 || e >= eprev) && e - i >= min_len && e > i) {", "contained matches reported as SMEMs"),
    ("smem-min-occ", "oracle.c", "            if (hi2 - lo2 < min_occ) break;", "            if (hi2 - lo2 <= min_occ) break;",
     "an extension needing one occurrence more than min_occ"),
    ("smem-rc-uncomplemented", "oracle.c", "for (int64_t t = 0; t < L; ++t) rc[t] = orc_comp(P[e - 1 - t]);",
     "for (int64_t t = 0; t < L; ++t) rc[t] = P[e - 1 - t];", "the reverse-strand interval of the reversed match"),
    ("scan-sentinel", "oracle.c",
     "        if (t + d == L) return 1;              /* the suffix's sentinel is below every base */",
     "        if (t + d == L) return 0;              /* the suffix's sentinel is below every base */",
     "the scan's sentinel above the probes"),
    ("scan-probe-order", "oracle.c", "    if (la < lb) return (a & 1) ? 1 : -1;", "    if (la < lb) return (a & 1) ? -1 : 1;",
     "a shorter probe's terminal on the wrong side"),
    ("seedscan-kth-end", "oracle.c", "                    if (c >= min_occ) lo_ = mid; else hi_ = mid - 1;",
     "                    if (c > min_occ) lo_ = mid; else hi_ = mid - 1;", "e(i) as the (min_occ+1)-th run end"),
    ("seedscan-contained", "oracle.c", "            if (e >= 0 && (i == 0 || e > eprev)) {", "            if (e >= 0) {",
     "the seeded scan reporting contained matches"),
    ("seedscan-run-cover", "oracle.c", "                if (act[a] - ell >= i) act[w++] = act[a];",
     "                if (act[a] - ell > i) act[w++] = act[a];", "a seed run dropped one position early"),
    ("delta-length", "rle.c", "    return (K - 1) + K + (N - 1);", "    return (K - 1) + K + N;",
     "the Elias delta code's length with the leading bit"),
    ("rle-rank-offset", "rle.c", "        if (off == 0) continue;", "        if (off <= 1) continue;",
     "rank skipping the first symbol of a segment"),
    ("insertion-extension", "hapl.c", "const int e = hp_max(eh, ee) - gap_ext;",
     "const int e = hp_max(eh - gap_ext, ee);", "an insertion run that stops paying its extension"),
    ("deletion-extension", "hapl.c", "const int f = hp_max(fh, ff) - gap_ext;",
     "const int f = hp_max(fh - gap_ext, ff);", "a deletion run that stops paying its extension"),
    ("representative-order", "hapl.c", "if (v == x->v && x->str && kr >= x->kr) return 0;",
     "if (v == x->v && x->str && kr <= x->kr) return 0;", "equal scores keeping the larger reverse-complement start"),
    ("gap-representative", "hapl.c", "    if (a != b || !G->str) return a >= b ? H : G;",
     "    if (a != b || !G->str) return H;", "a gap passing on H's string when the gap's own score wins"),
    ("band-tie-order", "hapl.c", "if (a->k != b->k) return a->k < b->k;", "if (a->k != b->k) return a->k > b->k;",
     "tied cells of the band ordered by larger k first"),
]

CHILD = """
import sys
sys.path.insert(0, {root!r})
sys.path.insert(0, {tests!r})
import oracle
oracle._LIB_PATH = {lib!r}
oracle.build = lambda force=True: oracle._LIB_PATH
import pytest
sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', '-m', 'not gpu'] + {pins!r}))
"""


def run_one(name, fname, old, new, tmp):
    d = os.path.join(tmp, name)
    os.makedirs(d)
    for s in SRCS:
        shutil.copy(os.path.join(HERE, s), d)
    path = os.path.join(d, fname)
    text = open(path).read()
    if text.count(old) != 1:
        return "stale"  # the source changed: the mutant no longer applies
    open(path, "w").write(text.replace(old, new))
    lib = os.path.join(d, "liboracle.so")
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-std=c99", "-o", lib] +
                          [os.path.join(d, s) for s in SRCS])
    code = CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib,
                        pins=[os.path.join(ROOT, p) for p in PINS])
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT)
    if r.returncode == 0:
        return "survived"
    failed = [ln.split("::")[-1].split(" ")[0] for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    return "caught by " + (failed[0] if failed else "an error (exit %d)" % r.returncode)


def main(argv):
    pick = set(argv)
    bad = 0
    with tempfile.TemporaryDirectory() as tmp:
        for name, fname, old, new, what in MUTANTS:
            if pick and name not in pick:
                continue
            res = run_one(name, fname, old, new, tmp)
            bad += res != "stale" and not res.startswith("caught")
            print(f"{name:24s} {what:55s} {res}", flush=True)
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
