"""Host logic of the serving module, on the CPU: which requests go into a
pack, how a stream is cut into batches under a request count and a byte
budget, the bytes a packed product may need, and the slot memory that
batches carve their buffers from.  No GPU and no library call."""
import numpy as np
import pytest
import torch

from paper_1004_4548_amd import inputs as I
from paper_1004_4548_amd import serve


@pytest.fixture(scope="module")
def staged():
    return serve.stage([I.request(r) for r in range(60)], device="cpu")


def test_stage_keeps_the_requests(staged):
    for r, s in zip(range(60), staged):
        q = I.request(r)
        assert s.rid == q["id"] and s.pairs == len(q["a"][1]) * len(q["b"][1])
        np.testing.assert_array_equal(s.a.exps.numpy(), q["a"][0])
        np.testing.assert_array_equal(s.b.coef.numpy(), q["b"][1])
        assert s.meta["nv"] == s.a.nv


@pytest.mark.parametrize("limit", [0, 10_000, 1 << 22, 1 << 40])
def test_split_partitions_by_pairs(staged, limit):
    small, large = serve.split(staged, limit)
    assert sorted(small + large) == list(range(len(staged)))
    assert all(staged[i].pairs <= limit for i in small)
    assert all(staged[i].pairs > limit for i in large)


def test_pack_bytes_bounds_the_result():
    """At least the result of one term per pair (exponents and coefficient),
    aligned, and growing with the pairs."""
    s = serve.stage([I.request(3)], device="cpu")[0]
    b = serve.pack_bytes(s)
    assert b % 256 == 0
    assert b >= s.pairs * (4 * s.a.nv + 8)
    bigger = serve.Staged(s.rid, s.a, s.b, 2 * s.pairs)
    assert serve.pack_bytes(bigger) > b


@pytest.mark.parametrize("max_batch,max_bytes", [(1, 1 << 40), (16, 1 << 40), (16, 1 << 28),
                                                 (64, 1 << 20), (5, 0)])
def test_groups_respect_count_and_budget(staged, max_batch, max_bytes):
    """Consecutive groups, every request once and in order, at most max_batch
    requests each, and within the byte budget unless a request alone exceeds
    it (then it forms a group of its own)."""
    plans = [None] * len(staged)   # packed requests need no plan
    pack_pairs = 1 << 40           # every request is packed here
    out = serve.groups(staged, plans, max_batch, max_bytes, pack_pairs)
    flat = [s for g, _ in out for s in g]
    assert [s.rid for s in flat] == [s.rid for s in staged]
    for g, p in out:
        assert 1 <= len(g) <= max_batch and len(p) == len(g)
        need = [serve.request_bytes(s, None, pack_pairs) for s in g]
        assert sum(need) <= max_bytes or len(g) == 1
    # a group is closed only when the next request would not fit it
    for (g, _), (h, _) in zip(out, out[1:]):
        used = sum(serve.request_bytes(s, None, pack_pairs) for s in g)
        nxt = serve.request_bytes(h[0], None, pack_pairs)
        assert len(g) == max_batch or used + nxt > max_bytes


def test_slot_memory_carves_and_grows():
    m = serve.SlotMemory("cpu", 1 << 20)
    m.ensure(1000)
    a = m.take(10, torch.int64)
    b = m.take(3, torch.int32)
    assert a.numel() == 10 and b.numel() == 3 and b.dtype == torch.int32
    base = m.buf.data_ptr()   # offsets in the slot are 256-byte aligned (the device allocator aligns the base)
    assert (a.data_ptr() - base) % 256 == 0 and (b.data_ptr() - base) % 256 == 0
    assert b.data_ptr() >= a.data_ptr() + 256   # views of one batch do not overlap
    a.fill_(7)
    b.fill_(-1)
    assert int(a.sum()) == 70
    with pytest.raises(RuntimeError):
        m.take(1 << 20, torch.uint8)             # more than the slot holds
    m.ensure(3 << 20)                            # a larger batch replaces the buffer
    assert m.buf.numel() >= 3 << 20 and m.off == 0
    c = m.take(1 << 20, torch.int16)
    assert c.numel() == 1 << 20


def test_percentiles():
    lat = np.linspace(0.001, 0.1, 100)
    p = serve.percentiles(lat)
    assert p["p50_ms"] == pytest.approx(50.5, rel=1e-9)
    assert p["p50_ms"] <= p["p99_ms"] <= 100.0 and p["mean_ms"] == pytest.approx(50.5)
