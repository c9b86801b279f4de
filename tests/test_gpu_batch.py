"""GPU: batched execution (kp_batch, eager and replayed HIP graph) and the
serving paths give the same products as single calls and as the oracle."""
import numpy as np
import pytest

import oracle as O
import paper_1004_4548_amd as kp
from paper_1004_4548_amd import inputs as I
from paper_1004_4548_amd import serve
from tests.helpers import assert_exact, assert_tolerance

pytestmark = pytest.mark.gpu
TOL = 1e-13


def say(*a):
    print("[case]", *a, flush=True)


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _oracle_check(a, b, exps, coef, what):
    oe, oc, oab = O.laurent_mul(a[0], a[1], b[0], b[1], threads=4)
    if np.asarray(a[1]).dtype == np.float64:
        assert_tolerance([exps], coef, [oe], oc, oab, TOL, what)
    else:
        assert_exact([exps], coef, [oe], oc, what)


def _cases():
    """Small products of every kind: dense and hash, int64 and fp64."""
    out = []
    a, b = I.config(1, scale=0.4)
    out.append(("box int64", a, b))
    a, b = I.config(2, scale=0.1)
    out.append(("simplex int64", a, b))
    out.append(("simplex fp64", (a[0], a[1].astype(np.float64) / 8), (b[0], b[1].astype(np.float64))))
    a, b = I.config(3, scale=0.05)
    out.append(("sparse int64", a, b))
    return out


def _queue(bt, cases, ctx):
    import torch
    outs = []
    for what, a, b in cases:
        pa, pb = kp.Poly(dev(a[0]), dev(a[1])), kp.Poly(dev(b[0]), dev(b[1]))
        lay = kp.laurent_layout(pa, pb, ctx)
        ka, _ = kp.encode(lay, 0, pa.exps, ctx=ctx)
        kb, _ = kp.encode(lay, 1, pb.exps, ctx=ctx)
        mode, cap, ws = kp.mul_bound(lay, False, kp._dt(pa.coef), "auto", len(a[1]), len(b[1]),
                                     ctx)
        out = (torch.empty(max(cap, 1), dtype=torch.int64, device="cuda"),
               torch.empty(max(cap, 1), dtype=pa.coef.dtype, device="cuda"),
               torch.empty(1, dtype=torch.int64, device="cuda"))
        wbuf = torch.empty(max(ws, 256), dtype=torch.uint8, device="cuda")
        tid = bt.add_laurent(lay, ka, pa.coef, kb, pb.coef, out, wbuf)
        outs.append((what, a, b, lay, out, tid, mode))
    return outs


def _collect(bt, outs, ctx):
    res = []
    for what, a, b, lay, (oc, ov, on), tid, mode in outs:
        n = bt.status(tid)
        assert n == int(on.item())
        e = kp.decode(lay, oc[:n], ctx=ctx).cpu().numpy()
        res.append((e, ov[:n].cpu().numpy()))
    return res


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_oracle(graph):
    ctx = kp.context()
    cases = _cases()
    say("batch of", len(cases), "graph" if graph else "eager")
    bt = kp.Batch(len(cases), ctx)
    outs = _queue(bt, cases, ctx)
    for rep in range(3 if graph else 1):
        for _, _, _, _, (oc, ov, on), _, _ in outs:   # eager work between replays
            on.fill_(-99)
            ov.zero_()
        bt.launch(graph=graph)
        got = _collect(bt, outs, ctx)
        for (what, a, b, *_), (e, c) in zip(outs, got):
            _oracle_check(a, b, e, c, f"{what} (launch {rep})")


def test_batch_rejects_bad_tasks():
    import torch
    ctx = kp.context()
    bt = kp.Batch(1, ctx)
    a, b = I.config(1, scale=0.2)
    pa, pb = kp.Poly(dev(a[0]), dev(a[1])), kp.Poly(dev(b[0]), dev(b[1]))
    lay = kp.laurent_layout(pa, pb, ctx)
    ka, _ = kp.encode(lay, 0, pa.exps, ctx=ctx)
    kb, _ = kp.encode(lay, 1, pb.exps, ctx=ctx)
    _, cap, ws = kp.mul_bound(lay, False, kp.KP_I64, "auto", len(a[1]), len(b[1]), ctx)
    out = (torch.empty(cap, dtype=torch.int64, device="cuda"),
           torch.empty(cap, dtype=torch.int64, device="cuda"),
           torch.empty(1, dtype=torch.int64, device="cuda"))
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(kp.KPError) as e:
        bt.add_laurent(lay, ka, pa.coef, kb, pb.coef, out, small)
    assert e.value.status == kp.KP_E_WORKSPACE
    wbuf = torch.empty(max(ws, 256), dtype=torch.uint8, device="cuda")
    bt.add_laurent(lay, ka, pa.coef, kb, pb.coef, out, wbuf)
    with pytest.raises(kp.KPError):   # full
        bt.add_laurent(lay, ka, pa.coef, kb, pb.coef, out, wbuf)


def test_served_alone_equals_in_a_mix():
    # requests of the mixed stream, shrunk: alone (per call) and batched
    reqs = [_shrink(I.request(r)) for r in range(12)]
    say("stream requests", [(q["type"], q["nv"], len(q["a"][1]), len(q["b"][1])) for q in reqs])
    st = serve.stage(reqs)
    alone, _ = serve.run_per_call(st)
    # one batch: products of at most 50,000 pairs in a pack, the others one by one
    mixed = serve.run_batch(st, pack_pairs=50_000)
    # continuous batching: batches of 3 on 3 streams, overlapping on the device
    # (every product in the slots' packs, replayed graphs)
    _, served, _ = serve.serve_stream(st, np.zeros(len(st)), max_batch=3, slots=3)
    for q, x, y in zip(reqs, alone, served):
        ex, cx = x.exps.cpu().numpy(), x.coef.cpu().numpy()
        ey, cy = y.exps.cpu().numpy(), y.coef.cpu().numpy()
        ox, oy = np.lexsort(ex.T[::-1]), np.lexsort(ey.T[::-1])
        assert np.array_equal(ex[ox], ey[oy]), q["id"]
        if q["dtype"] == "i64":
            assert np.array_equal(cx[ox], cy[oy]), q["id"]
        else:   # fp64 sums in another order: each within the tolerance
            _oracle_check(q["a"], q["b"], ey, cy, f"served request {q['id']}")
    for q, x, y in zip(reqs, alone, mixed):
        ex, cx = x.exps.cpu().numpy(), x.coef.cpu().numpy()
        ey, cy = y.exps.cpu().numpy(), y.coef.cpu().numpy()
        ox, oy = np.lexsort(ex.T[::-1]), np.lexsort(ey.T[::-1])
        assert np.array_equal(ex[ox], ey[oy]), q["id"]
        if q["dtype"] == "i64":
            assert np.array_equal(cx[ox], cy[oy]), q["id"]
        _oracle_check(q["a"], q["b"], ey, cy, f"request {q['id']}")


def _gpu_keys(e, lo, w):
    import torch
    k = torch.zeros(e.shape[0], dtype=torch.int64, device=e.device)
    m = 1
    for v in range(e.shape[1]):
        k += (e[:, v].long() - int(lo[v])) * m
        m *= int(w[v])
    return k


def test_served_stream_equals_per_call():
    """The first 300 requests of the bench's stream, less those of more than
    2e7 pairs (264 requests, 6e8 pairs): served by continuous batching (packs
    and per-product kernels, 3 slots) against one call each, compared on the
    device.  int64: the same terms bit for bit.  fp64: the same keys, and each
    coefficient within 2e-13 of the term's sum of |contributions| (each side is
    within 1e-13 of the exact sum), that sum taken from the product of the
    factors' absolute values."""
    import torch
    reqs = [q for q in (I.request(r) for r in range(300))
            if len(q["a"][1]) * len(q["b"][1]) <= 2e7]
    say("served stream against single calls,", len(reqs), "requests")
    st = serve.stage(reqs)
    alone, _ = serve.run_per_call(st)
    _, served, _ = serve.serve_stream(st, np.zeros(len(st)), max_batch=16, slots=3)
    for q, s, x, y in zip(reqs, st, alone, served):
        what = f"request {q['id']} type {q['type']} {q['dtype']}"
        assert x.exps.shape == y.exps.shape, what
        if x.exps.shape[0] == 0:
            continue
        both = torch.cat([x.exps, y.exps])
        lo = both.min(0).values.cpu().numpy()
        w = (both.max(0).values.cpu().numpy() - lo + 1).astype(np.float64)
        assert np.prod(w) < 2.0**62, what
        kx, ox = torch.sort(_gpu_keys(x.exps, lo, w))
        ky, oy = torch.sort(_gpu_keys(y.exps, lo, w))
        assert torch.equal(kx, ky), what
        cx, cy = x.coef[ox], y.coef[oy]
        if q["dtype"] == "i64":
            assert torch.equal(cx, cy), what
            continue
        pa = kp.Poly(s.a.exps, s.a.coef.abs())
        pb = kp.Poly(s.b.exps, s.b.coef.abs())
        z, _ = kp.mul_laurent(pa, pb)
        # the absolute product covers every key of the product (and more)
        zlo = torch.minimum(z.exps.min(0).values, both.min(0).values).cpu().numpy()
        zw = (torch.maximum(z.exps.max(0).values, both.max(0).values).cpu().numpy() - zlo + 1)
        zk, oz = torch.sort(_gpu_keys(z.exps, zlo, zw.astype(np.float64)))
        kk = _gpu_keys(x.exps[ox], zlo, zw.astype(np.float64))
        pos = torch.searchsorted(zk, kk)
        assert torch.equal(zk[pos], kk), what
        bound = 2e-13 * z.coef[oz][pos]
        assert bool(((cx - cy).abs() <= bound).all()), what


def test_open_loop_serves_every_request():
    reqs = [_shrink(I.request(r)) for r in range(20, 36)]
    st = serve.stage(reqs)
    lat, wall = serve.open_loop(st, rate=2000.0, max_batch=4)
    assert len(lat) == len(reqs) and np.all(lat > 0) and wall > 0
    p = serve.percentiles(lat)
    assert p["p50_ms"] <= p["p99_ms"]


def _shrink(q, n=400):
    """A request with at most n terms per factor (the oracle stays quick)."""
    q = dict(q)
    q["a"] = (q["a"][0][:n], q["a"][1][:n])
    q["b"] = (q["b"][0][:n], q["b"][1][:n])
    return q


def test_autotuner_keeps_results():
    """The autotuner only moves knobs that do not change a product."""
    from paper_1004_4548_amd import tune
    ctx = kp.context()
    a, b = I.config(2, scale=0.2)
    pa, pb = kp.Poly(dev(a[0]), dev(a[1])), kp.Poly(dev(b[0]), dev(b[1]))
    before, _ = kp.mul_laurent(pa, pb, ctx=ctx)
    best, table = tune.tune_dense(ctx, scale=0.2, reps=2)
    assert len(table) == len(tune.DENSE_GRID) and best in tune.DENSE_GRID
    thr, rows = tune.tune_threshold(ctx, n=400, reps=1)
    assert thr >= 0 and rows
    bins, btable = tune.tune_bins(ctx, scale=0.05, reps=1)
    assert len(btable) == len(tune.BIN_GRID) and bins in tune.BIN_GRID
    hashed, htable = tune.tune_hash(ctx, scale=0.03, reps=1)
    assert hashed in tune.HASH_GRID and "hash_partitioned" not in hashed
    assert ctx.tune.hash_partitioned == 1   # the knob held while timing is restored
    ctx.set_tune(**best)
    after, _ = kp.mul_laurent(pa, pb, ctx=ctx)
    assert np.array_equal(before.exps.cpu().numpy(), after.exps.cpu().numpy())
    assert np.array_equal(before.coef.cpu().numpy(), after.coef.cpu().numpy())
