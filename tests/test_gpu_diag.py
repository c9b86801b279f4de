"""GPU: the diagnostics of the C ABI -- hash probe-length counters and the
LDS atomic-throughput probe -- report sane values and leave products as they
were."""
import math

import numpy as np
import pytest

import oracle as O
import paper_1004_4548_amd as kp
from paper_1004_4548_amd import inputs as I
from tests.helpers import assert_exact

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_hash_stats_count_every_insertion():
    ctx = kp.context()
    a, b = I.config(3, scale=0.05)
    say("hash stats", len(a[1]), "x", len(b[1]))
    pa, pb = kp.Poly(dev(a[0]), dev(a[1])), kp.Poly(dev(b[0]), dev(b[1]))
    ctx.hash_stats_read()          # start from zero
    kp.mul_laurent(pa, pb, mode="hash", ctx=ctx)
    assert ctx.hash_stats_read() == (0, 0, 0)   # off by default
    ctx.hash_stats(True)
    try:
        r, _ = kp.mul_laurent(pa, pb, mode="hash", ctx=ctx)
        ins, extra, ovf = ctx.hash_stats_read()
    finally:
        ctx.hash_stats(False)
    # coefficients in [1, 1000]: every term product is nonzero and inserted
    assert ins == len(a[1]) * len(b[1])
    assert 0 <= extra and extra / ins < 8.0
    oe, oc, _ = O.laurent_mul(a[0], a[1], b[0], b[1], threads=4)
    assert_exact([r.exps.cpu().numpy()], r.coef.cpu().numpy(), [oe], oc, "hash with stats")


def test_hash_stats_poisson_counts_both_pieces():
    ctx = kp.context()
    a, b = I.config(4, scale=0.04)
    say("poisson hash stats", len(a[3]), "x", len(b[3]))
    sa = kp.PoissonSeries(dev(a[0]), dev(a[1]), dev(a[2]), dev(a[3]))
    sb = kp.PoissonSeries(dev(b[0]), dev(b[1]), dev(b[2]), dev(b[3]))
    ctx.hash_stats_read()
    ctx.hash_stats(True)
    try:
        kp.mul_poisson(sa, sb, mode="hash", ctx=ctx)
        ins, extra, ovf = ctx.hash_stats_read()
    finally:
        ctx.hash_stats(False)
    # each pair gives the difference and the sum term; only sines of the zero
    # multiplier vector are dropped
    assert 0 < ins <= 2 * len(a[3]) * len(b[3])
    assert extra >= 0


@pytest.mark.parametrize("pattern", [0, 1, 2, 3, 4])
def test_lds_atomic_probe(pattern):
    ctx = kp.context()
    say("lds atomic probe pattern", pattern)
    r = ctx.probe_lds_atomic(pattern)
    assert math.isfinite(r) and r > 1e11
    # no more than one 8-byte atomic lane per LDS bank-pair per clock per CU
    assert r < 256 * 32 * 3.0e9
