"""Definitional CPU oracle (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library does not use it and shares no code with
it. The arithmetic lives in ``oracle.c`` (plain C, built with gcc); this module
only marshals numpy arrays.

Functions (each follows a definition of arXiv 2409.00613):
  expand      double-strand string list P0, rc(P0), P1, rc(P1), ... (Sec. 2.5)
  bwt         BWT by sorting every suffix of the sentinel-terminated list (Sec. 2.1)
  verify      inverse-BWT check of a candidate BWT (LF relation, Sec. 2.1);
              Verifier does the same check in parts for very large lists
  count       SA interval [lo, hi) by scanning every suffix (Sec. 2.3)
  Text.interval / Text.smem
              SA interval by binary search; SMEMs by their definition (Sec. 2.6)
  insertion_ranks
              l(x) of each new suffix: number of existing-index suffixes below
              it (the quantity Algorithm 1 accumulates)
  scan_intervals
              the same [lo, hi) for a batch of patterns in one pass over every
              suffix (for texts too large for a suffix sort)
  smem_scan   the SMEMs of Text.smem for a batch of queries by a seeded scan
              of the text (hashed min_len-mers, diagonal runs), no suffix array
  locate      the suffix-array entry of a row written as (string index,
              offset within the string) (Sec. 2.4)
  rows_of     the inverse: the row of the suffix at (string index, offset)
  Text.hapl   local haplotype enumeration (Sec. 2.8): semi-global alignment
              of a query to the prefix DAWG by the revised BWA-SW recurrences
              (Sec. 2.7, Algorithm 5) and the bi-interval redundancy filter
              (``hapl.c`` holds the readings)
  rle_encode / rle_decode / rle_rank / delta_code
              the run-length static format (Sec. 2.2, Fig. 2b): blocks of
              Elias-delta coded runs with marginal counts and an index row,
              and rank by decoding them (``rle.c`` holds the definition)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "rle.c"), os.path.join(_HERE, "hapl.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile oracle.c, rle.c and hapl.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-std=c99",
                               "-Wall", "-Wextra", "-o", tmp] + _SRCS)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_expand.argtypes = [_u8p, _i64p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _u8p, _i64p]
    lib.orc_expand.restype = ctypes.c_int
    lib.orc_bwt.argtypes = [_u8p, _i64p, ctypes.c_int64, ctypes.c_int, _u8p, _i64p]
    lib.orc_bwt.restype = ctypes.c_int
    lib.orc_verify.argtypes = [_u8p, ctypes.c_int64, _u8p, _i64p, ctypes.c_int64, ctypes.c_int]
    lib.orc_verify.restype = ctypes.c_int64
    lib.orc_verifier_new.argtypes = [_u8p, ctypes.c_int64, _u8p, _i64p, ctypes.c_int64, _i64p]
    lib.orc_verifier_new.restype = ctypes.c_void_p
    lib.orc_verifier_new_mt.argtypes = [_u8p, ctypes.c_int64, _u8p, _i64p, ctypes.c_int64, ctypes.c_int, _i64p]
    lib.orc_verifier_new_mt.restype = ctypes.c_void_p
    lib.orc_verifier_walk.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
    lib.orc_verifier_walk.restype = ctypes.c_int64
    lib.orc_verifier_free.argtypes = [ctypes.c_void_p]
    lib.orc_verifier_free.restype = None
    lib.orc_count.argtypes = [_u8p, _i64p, ctypes.c_int64, _u8p, _i64p, ctypes.c_int64,
                              ctypes.c_int, _i64p, _i64p]
    lib.orc_count.restype = ctypes.c_int
    lib.orc_text_new.argtypes = [_u8p, _i64p, ctypes.c_int64]
    lib.orc_text_new.restype = ctypes.c_void_p
    lib.orc_text_free.argtypes = [ctypes.c_void_p]
    lib.orc_text_free.restype = None
    lib.orc_sa_interval.argtypes = [ctypes.c_void_p, _i64p, _u8p, ctypes.c_int64, _i64p, _i64p]
    lib.orc_sa_interval.restype = ctypes.c_int
    lib.orc_smem.argtypes = [ctypes.c_void_p, _i64p, _u8p, ctypes.c_int64, ctypes.c_int64,
                             ctypes.c_int64, _i64p, ctypes.c_int64]
    lib.orc_smem.restype = ctypes.c_int64
    lib.orc_scan_intervals.argtypes = [_u8p, _i64p, ctypes.c_int64, _u8p, _i64p, ctypes.c_int64,
                                       ctypes.c_int, _i64p, _i64p]
    lib.orc_scan_intervals.restype = ctypes.c_int
    lib.orc_smem_scan.argtypes = [_u8p, _i64p, ctypes.c_int64, _u8p, _i64p, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_int, _i64p, ctypes.c_int64, _i64p]
    lib.orc_smem_scan.restype = ctypes.c_int64
    _u64p = ctypes.POINTER(ctypes.c_uint64)
    _u16p = ctypes.POINTER(ctypes.c_uint16)
    lib.orc_delta_len.argtypes = [ctypes.c_uint64]
    lib.orc_delta_len.restype = ctypes.c_int
    lib.orc_delta_string.argtypes = [ctypes.c_uint64, ctypes.c_char_p]
    lib.orc_delta_string.restype = ctypes.c_int
    lib.orc_rle_encode.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int, _u64p, _i64p, _u16p, _i64p]
    lib.orc_rle_encode.restype = ctypes.c_int
    lib.orc_rle_decode.argtypes = [_u64p, _i64p, ctypes.c_int64, _u8p]
    lib.orc_rle_decode.restype = ctypes.c_int
    lib.orc_rle_rank.argtypes = [_u64p, _i64p, _u16p, ctypes.c_int64, ctypes.c_int, _i64p, ctypes.c_int64,
                                 _i64p]
    lib.orc_rle_rank.restype = ctypes.c_int
    lib.orc_hapl.argtypes = [ctypes.c_void_p, _i64p, ctypes.c_int64, _u8p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                             ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64p, ctypes.c_int64, _i64p, ctypes.c_int]
    lib.orc_hapl.restype = ctypes.c_int64
    _lib = lib
    return lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def host_threads() -> int:
    """Threads the oracle uses by default: the CPUs this process may run on,
    no more than OMP_NUM_THREADS when that is set (a shared GPU host grants
    each GPU a share of its cores that way)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def _threads(nthreads):
    return int(nthreads) if nthreads else host_threads()


def expand(data: np.ndarray, lens: np.ndarray, both: bool = True, allow_empty: bool = False):
    """Encode ASCII strings ($=0 A=1 C=2 G=3 T=4 N=5) and, when ``both``, follow
    each string by its reverse complement. Returns (codes, lens)."""
    lib = _load()
    data = np.ascontiguousarray(data, dtype=np.uint8)
    lens = np.ascontiguousarray(lens, dtype=np.int64)
    k = 2 if both else 1
    codes = np.empty(max(1, k * int(lens.sum())), dtype=np.uint8)
    out_lens = np.empty(max(1, k * lens.shape[0]), dtype=np.int64)
    dat = data if data.size else np.zeros(1, np.uint8)
    rc = lib.orc_expand(_p(dat, _u8p), _p(lens, _i64p), lens.shape[0], int(both), int(allow_empty),
                        _p(codes, _u8p), _p(out_lens, _i64p))
    if rc == -1:
        raise ValueError("byte outside ACGTNacgtn")
    if rc == -2:
        raise ValueError("empty string")
    return codes[:k * int(lens.sum())], out_lens[:k * lens.shape[0]]


def encode(data: np.ndarray, lens: np.ndarray):
    """Encode patterns without reverse complements; empty patterns allowed."""
    return expand(data, lens, both=False, allow_empty=True)


def bwt(codes: np.ndarray, lens: np.ndarray, nthreads: int | None = None, want_sa: bool = False):
    """BWT (codes 0..5) of the ordered list; optionally also its suffix array."""
    lib = _load()
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    lens = np.ascontiguousarray(lens, dtype=np.int64)
    n = int(lens.sum()) + lens.shape[0]
    B = np.empty(max(n, 1), dtype=np.uint8)
    S = np.empty(max(n, 1), dtype=np.int64) if want_sa else None
    cod = codes if codes.size else np.zeros(1, np.uint8)
    rc = lib.orc_bwt(_p(cod, _u8p), _p(lens, _i64p), lens.shape[0], _threads(nthreads),
                     _p(B, _u8p), _p(S, _i64p) if want_sa else None)
    if rc != 0:
        raise MemoryError("oracle bwt: allocation failed")
    if want_sa:
        return B[:n], S[:n]
    return B[:n]


def verify(B: np.ndarray, codes: np.ndarray, lens: np.ndarray, nthreads: int | None = None) -> int:
    """0 if B is the BWT of the list; otherwise a nonzero diagnostic
    (-1 wrong length, -2 wrong symbol counts, j+1 string j not recovered)."""
    lib = _load()
    B = np.ascontiguousarray(B, dtype=np.uint8)
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    lens = np.ascontiguousarray(lens, dtype=np.int64)
    cod = codes if codes.size else np.zeros(1, np.uint8)
    b = B if B.size else np.zeros(1, np.uint8)
    return int(lib.orc_verify(_p(b, _u8p), B.shape[0], _p(cod, _u8p), _p(lens, _i64p),
                              lens.shape[0], _threads(nthreads)))


class Verifier:
    """The inverse-BWT check in parts: the constructor checks the length and
    the symbol counts (``status`` 0, or -1 / -2 as for verify); walk(j0, j1)
    checks strings [j0, j1) and returns 0 or the first failing j + 1. The
    list passes when status is 0 and every string of [0, m) walks cleanly.
    The arrays are kept referenced for the verifier's lifetime."""

    def __init__(self, B: np.ndarray, codes: np.ndarray, lens: np.ndarray, nthreads: int | None = None):
        lib = _load()
        self.B = np.ascontiguousarray(B, dtype=np.uint8)
        self.codes = np.ascontiguousarray(codes, dtype=np.uint8)
        self.lens = np.ascontiguousarray(lens, dtype=np.int64)
        self.m = self.lens.shape[0]
        b = self.B if self.B.size else np.zeros(1, np.uint8)
        cod = self.codes if self.codes.size else np.zeros(1, np.uint8)
        self._keep = (b, cod)
        st = ctypes.c_int64(0)
        self._h = lib.orc_verifier_new_mt(_p(b, _u8p), self.B.shape[0], _p(cod, _u8p), _p(self.lens, _i64p),
                                          self.m, _threads(nthreads), ctypes.byref(st))
        self.status = int(st.value)

    def walk(self, j0: int, j1: int, nthreads: int | None = None) -> int:
        if not self._h:
            raise RuntimeError("verifier was not created (status %d)" % self.status)
        return int(_load().orc_verifier_walk(self._h, j0, j1, _threads(nthreads)))

    def close(self):
        if getattr(self, "_h", None):
            _load().orc_verifier_free(self._h)
            self._h = None

    def __del__(self):
        self.close()


def count(codes: np.ndarray, lens: np.ndarray, qcodes: np.ndarray, qlens: np.ndarray,
          nthreads: int | None = None):
    """Brute-force SA intervals (lo, hi) of each query."""
    lib = _load()
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    lens = np.ascontiguousarray(lens, dtype=np.int64)
    qcodes = np.ascontiguousarray(qcodes, dtype=np.uint8)
    qlens = np.ascontiguousarray(qlens, dtype=np.int64)
    nq = qlens.shape[0]
    lo = np.zeros(max(nq, 1), dtype=np.int64)
    hi = np.zeros(max(nq, 1), dtype=np.int64)
    q = qcodes if qcodes.size else np.zeros(1, np.uint8)
    cod = codes if codes.size else np.zeros(1, np.uint8)
    rc = lib.orc_count(_p(cod, _u8p), _p(lens, _i64p), lens.shape[0], _p(q, _u8p),
                       _p(qlens, _i64p), nq, _threads(nthreads), _p(lo, _i64p), _p(hi, _i64p))
    if rc != 0:
        raise MemoryError("oracle count: allocation failed")
    return lo[:nq], hi[:nq]


# Patterns given to scan_intervals / SMEMs found by smem_scan: at least this
# long, and their first SCAN_K symbols are A..T (the scan's bucket key).
SCAN_K = 12


def scan_intervals(codes: np.ndarray, lens: np.ndarray, pcodes: np.ndarray, plens: np.ndarray,
                   nthreads: int | None = None):
    """SA intervals (lo, hi) of each pattern, as count() gives them, by one
    pass over every suffix. Each pattern must be at least SCAN_K long and
    start with SCAN_K symbols of A..T (ValueError otherwise)."""
    lib = _load()
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    lens = np.ascontiguousarray(lens, dtype=np.int64)
    pcodes = np.ascontiguousarray(pcodes, dtype=np.uint8)
    plens = np.ascontiguousarray(plens, dtype=np.int64)
    npat = plens.shape[0]
    lo = np.zeros(max(npat, 1), dtype=np.int64)
    hi = np.zeros(max(npat, 1), dtype=np.int64)
    pp = pcodes if pcodes.size else np.zeros(1, np.uint8)
    cod = codes if codes.size else np.zeros(1, np.uint8)
    rc = lib.orc_scan_intervals(_p(cod, _u8p), _p(lens, _i64p), lens.shape[0], _p(pp, _u8p), _p(plens, _i64p),
                                npat, _threads(nthreads), _p(lo, _i64p), _p(hi, _i64p))
    if rc == -4:
        raise ValueError(f"scan_intervals: every pattern must start with {SCAN_K} symbols of A..T")
    if rc != 0:
        raise MemoryError("oracle scan_intervals: allocation failed")
    return lo[:npat], hi[:npat]


def smem_scan(codes: np.ndarray, lens: np.ndarray, qcodes: np.ndarray, qlens: np.ndarray, min_len: int,
              min_occ: int = 1, nthreads: int | None = None):
    """SMEMs of each query (as Text.smem gives them) by a seeded scan of the
    text. Returns (records, offsets): records is an (k, 5) int64 array of
    start, end, occ, lo, lo_rc; query i owns records[offsets[i]:offsets[i+1]].
    min_len must be at least SCAN_K, and each SMEM and its reverse complement
    must start with SCAN_K symbols of A..T (ValueError otherwise)."""
    lib = _load()
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    lens = np.ascontiguousarray(lens, dtype=np.int64)
    qcodes = np.ascontiguousarray(qcodes, dtype=np.uint8)
    qlens = np.ascontiguousarray(qlens, dtype=np.int64)
    nq = qlens.shape[0]
    qq = qcodes if qcodes.size else np.zeros(1, np.uint8)
    cod = codes if codes.size else np.zeros(1, np.uint8)
    cap = max(1024, int(qlens.sum()) // 32)
    while True:
        out = np.zeros((cap, 5), dtype=np.int64)
        off = np.zeros(nq + 1, dtype=np.int64)
        k = lib.orc_smem_scan(_p(cod, _u8p), _p(lens, _i64p), lens.shape[0], _p(qq, _u8p), _p(qlens, _i64p), nq,
                              int(min_len), int(min_occ), _threads(nthreads), _p(out, _i64p), cap, _p(off, _i64p))
        if k == -4:
            raise ValueError(f"smem_scan: min_len must be >= {SCAN_K} and every SMEM must start with "
                             f"{SCAN_K} symbols of A..T on both strands")
        if k == -5:
            raise RuntimeError("smem_scan: run count and suffix count of an SMEM disagree")
        if k < 0:
            raise MemoryError("oracle smem_scan: allocation failed")
        if k <= cap:
            return out[:k], off
        cap = int(k)


class Text:
    """The concatenated text of a list plus its suffix array (by the oracle's
    own sort), for interval and SMEM queries."""

    def __init__(self, codes: np.ndarray, lens: np.ndarray, nthreads: int | None = None):
        lib = _load()
        self.codes = np.ascontiguousarray(codes, dtype=np.uint8)
        self.lens = np.ascontiguousarray(lens, dtype=np.int64)
        self.B, self.S = bwt(self.codes, self.lens, nthreads, want_sa=True)
        self.n = int(self.S.shape[0])
        cod = self.codes if self.codes.size else np.zeros(1, np.uint8)
        self._keep = cod
        self._h = lib.orc_text_new(_p(cod, _u8p), _p(self.lens, _i64p), self.lens.shape[0])
        if not self._h:
            raise MemoryError("oracle text: allocation failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_text_free(h)
            self._h = None

    def interval(self, P: np.ndarray):
        P = np.ascontiguousarray(P, dtype=np.uint8)
        lo = np.zeros(1, np.int64)
        hi = np.zeros(1, np.int64)
        pp = P if P.size else np.zeros(1, np.uint8)
        _lib.orc_sa_interval(self._h, _p(self.S, _i64p), _p(pp, _u8p), P.shape[0],
                             _p(lo, _i64p), _p(hi, _i64p))
        return int(lo[0]), int(hi[0])

    def smem(self, P: np.ndarray, min_len: int, min_occ: int = 1) -> np.ndarray:
        """SMEMs as an (k, 5) int64 array: start, end, occ, lo, lo_rc."""
        P = np.ascontiguousarray(P, dtype=np.uint8)
        pp = P if P.size else np.zeros(1, np.uint8)
        cap = max(16, P.shape[0] // 8)
        while True:
            out = np.zeros((cap, 5), dtype=np.int64)
            k = _lib.orc_smem(self._h, _p(self.S, _i64p), _p(pp, _u8p), P.shape[0],
                              int(min_len), int(min_occ), _p(out, _i64p), cap)
            if k < 0:
                raise MemoryError("oracle smem: allocation failed")
            if k <= cap:
                return out[:k]
            cap = int(k)


def _text_hapl(self, P: np.ndarray, match: int = 1, mismatch: int = 4, gap_open: int = 6, gap_ext: int = 1,
               band: int = 25, raw: bool = False) -> np.ndarray:
    """Local haplotype enumeration of one query (codes 1..5): rows of
    (k, k_rc, s, score), ordered by decreasing score; raw=True gives every
    cell of the query's start before the redundancy filter."""
    P = np.ascontiguousarray(P, dtype=np.uint8)
    pp = P if P.size else np.zeros(1, np.uint8)
    cap = 256
    while True:
        out = np.zeros((cap, 5), np.int64)
        nraw = np.zeros(1, np.int64)
        k = _lib.orc_hapl(self._h, _p(self.S, _i64p), self.n, _p(pp, _u8p), P.shape[0], int(match),
                          int(mismatch), int(gap_open), int(gap_ext), int(band), _p(out, _i64p), cap,
                          _p(nraw, _i64p), 1 if raw else 0)
        if k < 0:
            raise MemoryError("oracle hapl: allocation failed")
        if k <= cap:
            return out[:k, :4]
        cap = int(k)


Text.hapl = _text_hapl


def insertion_ranks(S: np.ndarray, lens: np.ndarray, m1: int) -> np.ndarray:
    """From the suffix array S of the list (existing strings 0..m1-1 followed
    by new strings), return l(x) for every position x of the new strings'
    part of the text (sentinels included): the number of suffixes of the
    existing strings that are smaller than x."""
    lens = np.asarray(lens, dtype=np.int64)
    n1 = int(lens[:m1].sum()) + m1
    n = int(S.shape[0])
    is_new = S >= n1
    rows_old_before = np.cumsum(~is_new) - (~is_new)   # old suffixes strictly before each row
    l = np.empty(n - n1, dtype=np.int64)
    l[S[is_new] - n1] = rows_old_before[is_new]
    return l


def _string_starts(lens: np.ndarray) -> np.ndarray:
    """Start of each string in the concatenated text (each string is
    followed by its sentinel)."""
    lens = np.asarray(lens, dtype=np.int64)
    return np.concatenate([[0], np.cumsum(lens + 1)])[:-1]


def locate(S: np.ndarray, lens: np.ndarray, rows) -> tuple[np.ndarray, np.ndarray]:
    """Position of the suffix at each row (Sec. 2.4): S(row) is a position of
    the concatenated text; it is reported as the index of the string that
    holds it and the offset within that string (offset = the string's length
    for its sentinel suffix)."""
    rows = np.asarray(rows, dtype=np.int64)
    starts = _string_starts(lens)
    pos = np.asarray(S, dtype=np.int64)[rows]
    j = np.searchsorted(starts, pos, side="right") - 1
    return j.astype(np.int64), (pos - starts[j]).astype(np.int64)


def rows_of(S: np.ndarray, lens: np.ndarray, strings, offsets) -> np.ndarray:
    """Row of the suffix starting at (string, offset): the inverse suffix
    array at that text position."""
    S = np.asarray(S, dtype=np.int64)
    inv = np.empty_like(S)
    inv[S] = np.arange(S.shape[0], dtype=np.int64)
    starts = _string_starts(lens)
    return inv[starts[np.asarray(strings, dtype=np.int64)] + np.asarray(offsets, dtype=np.int64)]


# ---------------------------------------------------------------------------
# Run-length static format (rle.c)
# ---------------------------------------------------------------------------

RLE_SEG_SHIFT = 20
RLE_WORDS = 16


def delta_code(L: int) -> str:
    """The Elias delta code of L >= 1 as a '0'/'1' string (MSB first)."""
    buf = ctypes.create_string_buffer(80)
    _load().orc_delta_string(ctypes.c_uint64(L), buf)
    return buf.value.decode()


class Rle:
    """The format's three arrays: blocks (nblocks x 16 uint64), seg
    ((nseg + 1) x 8 int64), row (uint16), with n and the row shift q."""

    def __init__(self, blocks, seg, row, n, q):
        self.blocks, self.seg, self.row, self.n, self.q = blocks, seg, row, int(n), int(q)

    @property
    def nbytes(self) -> int:
        return self.blocks.nbytes + self.seg.nbytes + self.row.nbytes


def rle_encode(B: np.ndarray, q: int) -> Rle:
    """Encode a BWT (codes 0..5) in the run-length format with row shift q."""
    lib = _load()
    B = np.ascontiguousarray(B, dtype=np.uint8)
    n = B.shape[0]
    _u64p = ctypes.POINTER(ctypes.c_uint64)
    _u16p = ctypes.POINTER(ctypes.c_uint16)
    nb = np.zeros(1, np.int64)
    if lib.orc_rle_encode(_p(B, _u8p), n, q, None, None, None, _p(nb, _i64p)) != 0:
        raise ValueError("rle_encode: bad arguments")
    nseg = (n + (1 << RLE_SEG_SHIFT) - 1) >> RLE_SEG_SHIFT
    blocks = np.zeros((int(nb[0]), RLE_WORDS), np.uint64)
    seg = np.zeros((nseg + 1, 8), np.int64)
    row = np.zeros(((n - 1) >> q) + 1, np.uint16)
    lib.orc_rle_encode(_p(B, _u8p), n, q, _p(blocks, _u64p), _p(seg, _i64p), _p(row, _u16p), _p(nb, _i64p))
    return Rle(blocks, seg, row, n, q)


def rle_decode(r: Rle) -> np.ndarray:
    """The BWT back out of its blocks."""
    out = np.zeros(r.n, np.uint8)
    blocks = np.ascontiguousarray(r.blocks, dtype=np.uint64)
    seg = np.ascontiguousarray(r.seg, dtype=np.int64)
    if _load().orc_rle_decode(_p(blocks, ctypes.POINTER(ctypes.c_uint64)), _p(seg, _i64p), r.n,
                              _p(out, _u8p)) != 0:
        raise ValueError("rle_decode: malformed blocks")
    return out


def rle_rank(r: Rle, positions) -> np.ndarray:
    """Occurrences of $, A, C, G, T, N in B[0, i) for each position i, by the
    format's rank rule (rows of 6)."""
    pos = np.ascontiguousarray(positions, dtype=np.int64)
    out = np.zeros((pos.shape[0], 6), np.int64)
    blocks = np.ascontiguousarray(r.blocks, dtype=np.uint64)
    seg = np.ascontiguousarray(r.seg, dtype=np.int64)
    row = np.ascontiguousarray(r.row, dtype=np.uint16)
    if _load().orc_rle_rank(_p(blocks, ctypes.POINTER(ctypes.c_uint64)), _p(seg, _i64p),
                            _p(row, ctypes.POINTER(ctypes.c_uint16)), r.n, r.q, _p(pos, _i64p),
                            pos.shape[0], _p(out, _i64p)) != 0:
        raise ValueError("rle_rank: bad position or malformed blocks")
    return out
