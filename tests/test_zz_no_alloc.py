"""rb3_count_noalloc (the count entry point that allocates nothing) against
rb3_count, called through the C ABI: two calls in a row, the second with a
smaller input, with device and with host buffers, plus its error paths."""
import ctypes

import numpy as np
import pytest

import synth
from paper_2409_00613_amd import rb3

pytestmark = pytest.mark.gpu

_i64p = ctypes.POINTER(ctypes.c_int64)


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def index():
    w = synth.config_tiny(n_str=16, length=700, n_queries=600)
    idx = rb3.rb3_build(w.b1.data, w.b1.lens)
    rb3.rb3_merge(idx, w.new.data, w.new.lens)
    yield idx, w.queries
    idx.close()


def _noalloc_device(idx, qs):
    """Direct C-ABI call with device queries and preallocated device outputs."""
    import torch
    L = rb3.lib()
    dq = torch.from_numpy(qs.data).cuda() if qs.total else torch.zeros(1, dtype=torch.uint8, device="cuda")
    lens = np.ascontiguousarray(qs.lens, dtype=np.int64)
    n = lens.shape[0]
    lo = torch.full((max(n, 1),), -7, dtype=torch.int64, device="cuda")
    hi = torch.full((max(n, 1),), -7, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    rc = L.rb3_count_noalloc(idx.handle, ctypes.c_void_p(dq.data_ptr()), lens.ctypes.data_as(_i64p), n,
                             rb3.RB3_MEM_DEVICE, ctypes.cast(lo.data_ptr(), _i64p), ctypes.cast(hi.data_ptr(), _i64p))
    assert rc == rb3.RB3_OK, L.rb3_strerror(rc)
    assert torch.cuda.memory_allocated() == before
    return lo[:n].cpu().numpy(), hi[:n].cpu().numpy()


def test_noalloc_matches_count_device(index):
    idx, qs = index
    for a, b in ((0, qs.n), (0, qs.n // 3)):  # second call smaller than the first
        part = qs.slice(a, b)
        say(f"case: noalloc count, device buffers, {part.n} queries ({part.total} bases)")
        want = rb3.rb3_count(idx, part.data, part.lens)
        got = _noalloc_device(idx, part)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_noalloc_matches_count_host(index):
    idx, qs = index
    for a, b in ((0, qs.n), (qs.n // 2, qs.n // 2 + 37)):
        part = qs.slice(a, b)
        say(f"case: noalloc count, host buffers, {part.n} queries")
        want = rb3.rb3_count(idx, part.data, part.lens)
        got = rb3.rb3_count_noalloc(idx, part.data, part.lens)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_noalloc_empty_queries(index):
    idx, _ = index
    say("case: noalloc count, empty queries give [0, n)")
    n, _, _ = idx.info()
    lo, hi = rb3.rb3_count_noalloc(idx, b"ACGT", [0, 4, 0])
    want = rb3.rb3_count(idx, b"ACGT", [0, 4, 0])
    assert np.array_equal(lo, want[0]) and np.array_equal(hi, want[1])
    assert lo[0] == 0 and hi[0] == n


def test_noalloc_errors(index):
    idx, _ = index
    say("case: noalloc count, bad byte and oversized input")
    with pytest.raises(rb3.RB3Error) as e:
        rb3.rb3_count_noalloc(idx, b"ACGXT", [5])
    assert e.value.code == rb3.RB3_EINVAL
    big = np.full((32 << 20) + 1, ord("A"), np.uint8)  # more bytes than the scratch holds (host check)
    with pytest.raises(rb3.RB3Error) as e:
        rb3.rb3_count_noalloc(idx, big, [big.size])
    assert e.value.code == rb3.RB3_ELIMIT
    # the array still works after the refusals
    lo, hi = rb3.rb3_count_noalloc(idx, b"ACGTACGT", [8])
    want = rb3.rb3_count(idx, b"ACGTACGT", [8])
    assert lo[0] == want[0][0] and hi[0] == want[1][0]
