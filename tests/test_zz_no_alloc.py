"""GPU: the allocation-free entry point (kp_mul_laurent_noalloc) against
kp_mul_laurent with a caller workspace, through the C ABI.

Two calls in a row on one stream, the second on smaller factors (the scratch
array keeps the first call's contents), must give the results of the
entry point with a workspace: bit-exact int64 (dense mode returns ascending
codes, so the arrays are compared as they are; hash mode as term sets).  A
product whose workspace exceeds the scratch array is refused before anything
is queued."""
import ctypes as C

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


def _coded(ctx, a, b):
    pa, pb = kp.Poly(dev(a[0]), dev(a[1])), kp.Poly(dev(b[0]), dev(b[1]))
    lay = kp.laurent_layout(pa, pb, ctx)
    ka, _ = kp.encode(lay, 0, pa.exps, ctx=ctx)
    kb, _ = kp.encode(lay, 1, pb.exps, ctx=ctx)
    return lay, ka, pa.coef, kb, pb.coef


def _noalloc(ctx, lay, ka, ca, kb, cb, mode):
    import torch
    _, cap, ws = kp.mul_bound(lay, False, kp._dt(ca), mode, ka.shape[0], kb.shape[0], ctx)
    assert ws <= kp.KP_SCRATCH_BYTES
    out = (torch.empty(cap, dtype=torch.int64, device="cuda"),
           torch.empty(cap, dtype=ca.dtype, device="cuda"),
           torch.empty(1, dtype=torch.int64, device="cuda"))
    n = kp.mul_laurent_noalloc(lay, ka, ca, kb, cb, out, mode=mode, ctx=ctx)
    return out[0][:n].cpu().numpy(), out[1][:n].cpu().numpy()


@pytest.mark.parametrize("mode", ["dense", "hash"])
def test_noalloc_equals_workspace_entry_point(mode):
    ctx = kp.context()
    cfg = 2 if mode == "dense" else 3
    first = I.config(cfg, scale=0.3 if mode == "dense" else 0.02)
    second = I.config(cfg, scale=0.12 if mode == "dense" else 0.01)
    for what, (a, b) in (("first", first), ("second, smaller", second)):
        say("noalloc", mode, what, len(a[1]), "x", len(b[1]))
        lay, ka, ca, kb, cb = _coded(ctx, a, b)
        gk, gc = _noalloc(ctx, lay, ka, ca, kb, cb, mode)
        wk, wc, _ = kp.mul_laurent_codes(lay, ka, ca, kb, cb, mode, ctx)
        wk, wc = wk.cpu().numpy(), wc.cpu().numpy()
        if mode == "dense":
            np.testing.assert_array_equal(gk, wk)
            np.testing.assert_array_equal(gc, wc)
        else:
            assert_exact([gk], gc, [wk], wc, f"noalloc {mode} {what}")
        ex = kp.decode(lay, dev(gk)).cpu().numpy()
        oe, oc, _ = O.laurent_mul(a[0], a[1], b[0], b[1], threads=4)
        assert_exact([ex], gc, [oe], oc, f"noalloc {mode} {what} vs oracle")


def test_noalloc_refuses_a_product_larger_than_its_scratch():
    import torch
    ctx = kp.context()
    a, b = I.config(3, scale=0.1)
    say("noalloc too large", len(a[1]), "x", len(b[1]))
    lay, ka, ca, kb, cb = _coded(ctx, a, b)
    _, cap, ws = kp.mul_bound(lay, False, kp.KP_I64, "hash", ka.shape[0], kb.shape[0], ctx)
    assert ws > kp.KP_SCRATCH_BYTES
    on = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    out = (torch.empty(1, dtype=torch.int64, device="cuda"),
           torch.empty(1, dtype=torch.int64, device="cuda"), on)
    with pytest.raises(kp.KPError) as e:
        kp.mul_laurent_noalloc(lay, ka, ca, kb, cb, out, mode="hash", ctx=ctx)
    assert e.value.status == kp.KP_E_WORKSPACE
    torch.cuda.synchronize()
    assert int(on.item()) == 7   # nothing was queued
