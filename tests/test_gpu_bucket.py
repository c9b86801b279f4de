"""GPU: Section 3.2's bucketed hash table (code mod N into buckets of m
slots, an overflow table, terms ordered by code mod N) against the oracle.

Each case prints what it runs before touching the GPU.
"""
import numpy as np
import pytest

import oracle as O
import paper_1004_4548_amd as kp
from paper_1004_4548_amd import inputs as I
from tests.helpers import assert_exact, assert_tolerance

pytestmark = pytest.mark.gpu
TOL = 1e-13


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(autouse=True)
def _fresh_ctx():
    ctx = kp.context()
    saved = ctx.tune
    yield
    ctx.clear_truncation()
    ctx.hash_stats(False)
    ctx.set_tune(**{f: getattr(saved, f) for f, _ in kp.Tune._fields_})


def gpu(a, b, ctx, mode="hash"):
    pa = kp.Poly(dev(np.asarray(a[0], np.int32)), dev(a[1]))
    pb = kp.Poly(dev(np.asarray(b[0], np.int32)), dev(b[1]))
    r, _ = kp.mul_laurent(pa, pb, mode=mode, ctx=ctx)
    return r.exps.cpu().numpy(), r.coef.cpu().numpy()


def check(a, b, ctx, what):
    say(what, len(a[1]), "x", len(b[1]))
    ge, gc = gpu(a, b, ctx)
    oe, oc, oab = O.laurent_mul(a[0], a[1], b[0], b[1], threads=4)
    if np.asarray(a[1]).dtype == np.float64:
        assert_tolerance([ge], gc, [oe], oc, oab, TOL, what)
    else:
        assert_exact([ge], gc, [oe], oc, what)


@pytest.mark.parametrize("m,order", [(1, 1), (2, 0), (8, 1), (8, 0), (16, 1)])
def test_bucketed_matches_oracle(m, order):
    ctx = kp.context()
    ctx.set_tune(hash_bucket=m, hash_order=order)
    a, b = I.config(3, scale=0.05)
    check(a, b, ctx, f"sparse int64, m={m} order={order}")
    a64 = (a[0], a[1].astype(np.float64) / 8)
    b64 = (b[0], b[1].astype(np.float64))
    check(a64, b64, ctx, f"sparse fp64, m={m} order={order}")
    a, b = I.config(1, scale=0.5)   # many products per code
    check(a, b, ctx, f"box int64, m={m} order={order}")


def test_bucketed_overflow_table_is_used_and_exact():
    """One slot per bucket and as many buckets as result terms: buckets
    collide, the colliding codes go to the overflow table, the result is
    unchanged, and the statistics count them."""
    ctx = kp.context()
    rng = np.random.default_rng(77)
    a = (rng.integers(0, 40, (60, 2)).astype(np.int32), rng.integers(-9, 10, 60))
    b = (rng.integers(0, 40, (50, 2)).astype(np.int32), rng.integers(-9, 10, 50))
    oe, oc, _ = O.laurent_mul(a[0], a[1], b[0], b[1])
    ctx.set_tune(hash_bucket=1, hash_order=1, hash_capacity=len(oe))
    ctx.hash_stats_read()
    ctx.hash_stats(True)
    say("overflow, m=1, capacity", len(oe))
    ge, gc = gpu(a, b, ctx)
    ins, extra, ovf = ctx.hash_stats_read()
    ctx.hash_stats(False)
    assert_exact([ge], gc, [oe], oc, "overflowing buckets")
    assert ins > 0 and ovf > 0 and extra >= ovf


def test_bucketed_full_overflow_table_is_a_capacity_error():
    """Codes that all fall in one bucket (multiples of N) overflow far beyond
    the Poisson estimate the overflow table is sized for: reported as a
    capacity error, not hung; the next product is unaffected."""
    ctx = kp.context()
    n = 3000
    # bound 3000 terms -> capacity 6001 slots -> N = ceil(6001 / 16) = 376
    # buckets of 16; every code k * 376 goes to bucket 0, 1024 overflow slots
    nbk = -(-(2 * n + 1) // 16)
    a = (np.arange(n, dtype=np.int32).reshape(-1, 1) * nbk, np.ones(n, np.int64))
    b = (np.zeros((1, 1), np.int32), np.ones(1, np.int64))
    ctx.set_tune(hash_bucket=16, hash_partitioned=0)
    say("bucketed capacity error,", n, "codes in one bucket of", nbk)
    with pytest.raises(kp.KPError) as e:
        gpu(a, b, ctx)
    assert e.value.status == kp.KP_E_CAPACITY
    ctx.sync_check()
    a2, b2 = I.config(3, scale=0.03)
    check(a2, b2, ctx, "after the capacity error")


@pytest.mark.parametrize("order", [0, 1])
def test_bucketed_truncated(order):
    ctx = kp.context()
    ctx.set_tune(hash_bucket=8, hash_order=order)
    a, b = I.config(3, scale=0.05)
    w, D = [1] * 6, 300
    say("bucketed truncated, order", order)
    with ctx.truncation(w, D):
        ge, gc = gpu(a, b, ctx)
    oe, oc, _ = O.laurent_mul_truncated(a[0], a[1], b[0], b[1], w, D, threads=4)
    full = len(O.laurent_mul(a[0], a[1], b[0], b[1], threads=4)[0])
    assert 0 < len(oe) < full
    assert_exact([ge], gc, [oe], oc, "bucketed truncated")


def test_bucketed_not_used_for_poisson_or_exact():
    """Poisson series and 128-bit sums ignore hash_bucket and take the other layouts."""
    ctx = kp.context()
    ctx.set_tune(hash_bucket=4)
    pa, pb = I.config(4, scale=0.02)
    s = [kp.PoissonSeries(dev(p[0]), dev(p[1]), dev(p[2]), dev(p[3])) for p in (pa, pb)]
    say("poisson with hash_bucket set")
    r, _ = kp.mul_poisson(s[0], s[1], mode="hash", ctx=ctx)
    ox, oy, ot, oc, oab = O.poisson_mul(pa, pb, 3, 6)
    got = {(tuple(x), tuple(y), int(t)): c for x, y, t, c in
           zip(r.x.cpu().tolist(), r.y.cpu().tolist(), r.is_sin.cpu().tolist(), r.coef.cpu().tolist())}
    want = {(tuple(x), tuple(y), int(t)): (c, ab) for x, y, t, c, ab in
            zip(ox.tolist(), oy.tolist(), ot, oc, oab)}
    for k, c in got.items():
        assert abs(c - want[k][0]) <= TOL * want[k][1]
    a, b = I.config(1, scale=0.3)
    say("exact with hash_bucket set")
    r, _ = kp.mul_laurent(kp.Poly(dev(a[0]), dev(a[1])), kp.Poly(dev(b[0]), dev(b[1])),
                          mode="hash", ctx=ctx, exact=True)
    oe, oc, _ = O.laurent_mul(a[0], a[1], b[0], b[1], exact=True)
    assert_exact([r.exps.cpu().numpy()], r.coef.cpu().numpy(), [oe], oc, "exact, hash_bucket set")
