"""Pins of the oracle's run-length static format (rle.c; the bit-packed
format of Sec. 2.2, Fig. 2b): Elias delta codes against the textbook values,
the decoded BWT against the input, rank at every position against prefix
counts, and the bytes against a second reader of the format written here
from its definition (header fields, greedy packing, maximal pieces, index
row)."""
import numpy as np
import pytest

import oracle

SEG = 1 << 20
BITS = 896


def test_delta_codes_textbook():
    # Elias (1975) delta code: the bit length N of L in the Elias gamma code,
    # then L without its leading 1
    table = {
        1: "1", 2: "0100", 3: "0101", 4: "01100", 5: "01101", 6: "01110", 7: "01111",
        8: "00100000", 9: "00100001", 15: "00100111", 16: "001010000", 17: "001010001",
        32: "0011000000", 100: "00111100100",
    }
    for L, code in table.items():
        assert oracle.delta_code(L) == code, L
    # 2^20: N = 21 = 10101 (K = 5): four zeros, 10101, twenty zeros
    assert oracle.delta_code(1 << 20) == "0000" + "10101" + "0" * 20


def _prefix_counts(B, positions):
    out = np.zeros((len(positions), 6), np.int64)
    for c in range(6):
        cs = np.concatenate([[0], np.cumsum(B == c)])
        out[:, c] = cs[positions]
    return out


# --- a second reader of the format, from its definition -----------------

def _bits_of(words):
    return "".join(format(int(w), "064b") for w in words)


def _read_piece(s, t):
    sym = int(s[t:t + 3], 2)
    t += 3
    z = 0
    while s[t + z] == "0":
        z += 1
    N = int(s[t + z:t + 2 * z + 1], 2)
    t += 2 * z + 1
    L = int("1" + s[t:t + N - 1], 2) if N > 1 else 1
    return sym, L, t + N - 1


def _parse(r, B):
    """Walk every block; check the layout rules; return the decoded BWT."""
    n = r.n
    nseg = (n + SEG - 1) // SEG
    out = np.full(n, 255, np.uint8)
    assert r.seg.shape == (nseg + 1, 8)
    tot = np.zeros(6, np.int64)
    for s in range(nseg):
        s0, s1 = s * SEG, min(n, (s + 1) * SEG)
        assert list(r.seg[s, :6]) == list(tot), s
        b0, b1 = int(r.seg[s, 6]), int(r.seg[s + 1, 6])
        pos = s0
        cnt = np.zeros(6, np.int64)
        last_sym = -1
        starts = []
        for b in range(b0, b1):
            w = r.blocks[b]
            h0, h1 = int(w[0]), int(w[1])
            off = h0 & 0xFFFFF
            hc = [None, (h0 >> 20) & 0xFFFFF, (h0 >> 40) & 0xFFFFF, h1 & 0xFFFFF, (h1 >> 20) & 0xFFFFF,
                  (h1 >> 40) & 0xFFFFF]
            npc = (h0 >> 60) | ((h1 >> 60) << 4)
            assert s0 + off == pos, (s, b)
            assert hc[1:] == list(cnt[1:]) and off - sum(hc[1:]) == cnt[0], (s, b)
            starts.append(off)
            st = _bits_of(w[2:])
            t = 0
            for _ in range(npc):
                sym, L, t = _read_piece(st, t)
                assert sym != last_sym, "pieces of a segment are maximal runs"
                out[pos:pos + L] = sym
                cnt[sym] += L
                pos += L
                last_sym = sym
            assert t <= BITS and set(st[t:]) <= {"0"}
            # greedy: the next piece of the segment did not fit
            if b + 1 < b1:
                nxt = r.blocks[b + 1]
                sym, L, t2 = _read_piece(_bits_of(nxt[2:]), 0)
                assert t + t2 > BITS, (s, b)
        assert pos == s1
        tot += cnt
        # index row: entry j names the block holding j << q
        for j in range((s0 + (1 << r.q) - 1) >> r.q, ((s1 - 1) >> r.q) + 1):
            p = (j << r.q) - s0
            k = int(r.row[j])
            assert starts[k] <= p and (k + 1 == len(starts) or starts[k + 1] > p), (s, j)
    assert list(r.seg[nseg, :6]) == list(tot) and int(r.seg[nseg, 6]) == r.blocks.shape[0]
    return out


def _inputs():
    g = np.random.default_rng(20240613)
    yield "random short runs", g.integers(0, 6, 7000).astype(np.uint8), 4
    # pangenome-like: long runs with rare breaks
    runs = []
    for _ in range(400):
        runs.append(np.full(int(g.integers(1, 300)), int(g.integers(1, 5)), np.uint8))
    B = np.concatenate(runs)
    B[g.integers(0, B.shape[0], 20)] = 0
    yield "long runs", B, 6
    # one symbol per piece, alternating: the most pieces a block can hold
    yield "alternating", np.tile(np.array([1, 2], np.uint8), 3000), 4
    yield "single symbol", np.array([3], np.uint8), 4


@pytest.mark.parametrize("case", list(range(4)))
def test_rle_parse_round_trip_and_rank(case):
    name, B, q = list(_inputs())[case]
    r = oracle.rle_encode(B, q)
    assert np.array_equal(_parse(r, B), B), name
    assert np.array_equal(oracle.rle_decode(r), B), name
    pos = np.arange(B.shape[0] + 1)
    assert np.array_equal(oracle.rle_rank(r, pos), _prefix_counts(B, pos)), name


def test_rle_alternating_fills_blocks_with_4_bit_pieces():
    B = np.tile(np.array([1, 2], np.uint8), 3000)
    r = oracle.rle_encode(B, 4)
    npc = (r.blocks[:, 0] >> np.uint64(60)) | ((r.blocks[:, 1] >> np.uint64(60)) << np.uint64(4))
    assert list(npc[:-1]) == [BITS // 4] * (r.blocks.shape[0] - 1)


def test_rle_runs_across_segments():
    # a run longer than a segment is cut at segment starts; n one past two
    # segments; positions at and around every segment start
    B = np.concatenate([np.full(SEG + 5, 1, np.uint8), np.full(SEG - 3, 4, np.uint8), [0, 2, 2, 5]]).astype(np.uint8)
    n = B.shape[0]
    r = oracle.rle_encode(B, 12)
    assert r.seg.shape[0] == (n + SEG - 1) // SEG + 1
    assert np.array_equal(oracle.rle_decode(r), B)
    pos = np.array(sorted({0, 1, n, n - 1} | {k * SEG + d for k in range(3) for d in (-2, -1, 0, 1, 2)
                                            if 0 <= k * SEG + d <= n}))
    assert np.array_equal(oracle.rle_rank(r, pos), _prefix_counts(B, pos))
    g = np.random.default_rng(3)
    pos = g.integers(0, n + 1, 3000)
    assert np.array_equal(oracle.rle_rank(r, pos), _prefix_counts(B, pos))


@pytest.mark.parametrize("n", [SEG, SEG + 1])
def test_rle_segment_edges(n):
    g = np.random.default_rng(n)
    B = np.repeat(g.integers(0, 6, n // 4 + 2).astype(np.uint8), 4)[:n]
    for q in (4, 20):
        r = oracle.rle_encode(B, q)
        assert np.array_equal(oracle.rle_decode(r), B)
        pos = np.concatenate([g.integers(0, n + 1, 2000), [0, n, n - 1, SEG - 1, min(SEG, n)]])
        assert np.array_equal(oracle.rle_rank(r, pos), _prefix_counts(B, pos)), q


def test_rle_of_a_bwt_ranks_match_the_oracle_count():
    # the format serves backward search: pi(a, k) = C[a] + rank gives the
    # oracle's SA intervals
    g = np.random.default_rng(11)
    import synth
    w = synth.config_pangenome(genome_len=3000, n_b1=4, n_new=1)
    codes, lens = oracle.expand(w.b1.data, w.b1.lens)
    B = oracle.bwt(codes, lens)
    r = oracle.rle_encode(B, 5)
    C = np.concatenate([[0], np.cumsum(np.bincount(B, minlength=6))])[:6]
    pats = [codes[s:s + L] for s, L in zip(g.integers(0, codes.shape[0] - 40, 50), g.integers(1, 30, 50))]
    pats = [p for p in pats if (p != 0).all()]
    for p in pats:
        lo, hi = 0, B.shape[0]
        for a in p[::-1]:
            lo = C[a] + oracle.rle_rank(r, [lo])[0, a]
            hi = C[a] + oracle.rle_rank(r, [hi])[0, a]
        olo, ohi = oracle.count(codes, lens, p, np.array([len(p)], np.int64))
        assert (lo, hi) == (int(olo[0]), int(ohi[0]))
