"""GPU: exact products of int64 coefficients in 128-bit accumulators
(KP_I128) against the oracle's exact mode and against closed forms.

Results must agree bit for bit in both 64-bit words.  Each case prints what
it runs before touching the GPU.
"""
import math

import numpy as np
import pytest

import oracle as O
import paper_1004_4548_amd as kp
from paper_1004_4548_amd import inputs as I
from tests.helpers import adversarial_codes, assert_exact

pytestmark = pytest.mark.gpu


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
    ctx.set_tune(**{f: getattr(saved, f) for f, _ in kp.Tune._fields_})


def gpu_exact(a, b, mode, ctx=None):
    ctx = ctx or kp.context()
    pa = kp.Poly(dev(np.asarray(a[0], np.int32)), dev(np.asarray(a[1], np.int64)))
    pb = kp.Poly(dev(np.asarray(b[0], np.int32)), dev(np.asarray(b[1], np.int64)))
    r, lay = kp.mul_laurent(pa, pb, mode=mode, ctx=ctx, exact=True)
    assert tuple(r.coef.shape) == (r.exps.shape[0], 2)
    return r.exps.cpu().numpy(), r.coef.cpu().numpy(), lay


def check_exact(a, b, mode, what, ctx=None):
    say(what, mode, len(a[1]), "x", len(b[1]))
    ge, gc, lay = gpu_exact(a, b, mode, ctx)
    oe, oc, _ = O.laurent_mul(a[0], a[1], b[0], b[1], threads=4, exact=True)
    assert_exact([ge], gc, [oe], oc, what)
    return ge, gc, lay


def _big(rng, n, bits=62):
    return rng.integers(-2**bits, 2**bits, n, dtype=np.int64)


@pytest.mark.parametrize("mode", ["dense", "hash"])
def test_exact_matches_oracle(mode):
    rng = np.random.default_rng(128)
    (ea, _), (eb, _) = I.config(1, scale=0.5)
    check_exact((ea, _big(rng, len(ea))), (eb, _big(rng, len(eb))), mode, "box, 62-bit coefficients")
    (ea, _), (eb, _) = I.config(2, scale=0.08)
    check_exact((ea, _big(rng, len(ea), 63)), (eb, _big(rng, len(eb), 63)), mode,
                "simplex, 63-bit coefficients (sums wrap modulo 2^128)")
    (ea, ca), (eb, cb) = I.config(2, scale=0.08)
    check_exact((ea, ca), (eb, cb), mode, "simplex, benchmark coefficients")


def test_exact_sparse_hash():
    rng = np.random.default_rng(3)
    (ea, _), (eb, _) = I.config(3, scale=0.03)
    check_exact((ea, _big(rng, len(ea))), (eb, _big(rng, len(eb))), "hash", "6-variable sparse")


@pytest.mark.parametrize("part", [0, 2])
def test_exact_hash_layouts(part):
    """Both hash layouts with 128-bit sums: one HBM table of 32-byte slots
    (partitioned=0), and products grouped by hash bits (partitioned=2), whose
    entries carry the pair's term indices; the bins form each product and add
    it into 24-byte LDS slots, the carry taken from the low word's returning
    add.  Every bin table size (8192 slots are capped at 4096 for these)."""
    ctx = kp.context()
    ctx.set_tune(hash_partitioned=part)
    rng = np.random.default_rng(40 + part)
    (ea, _), (eb, _) = I.config(1, scale=0.5)
    check_exact((ea, _big(rng, len(ea))), (eb, _big(rng, len(eb))), "hash",
                f"box, 62-bit coefficients (partitioned={part})", ctx)
    (ea, _), (eb, _) = I.config(3, scale=0.03)
    ca, cb = _big(rng, len(ea), 63), _big(rng, len(eb), 63)
    ca[::7] = 0   # zero terms make no products
    check_exact((ea, ca), (eb, cb), "hash", f"sparse, 63-bit, zero terms (partitioned={part})", ctx)
    n = 4097   # one code, every add after the first carries out of the low word
    a = (np.zeros((n, 1), np.int32), np.full(n, 2**32 + 1, np.int64))
    b = (np.zeros((1, 1), np.int32), np.array([2**32 - 1], np.int64))
    say("one code,", n, "adds, partitioned", part)
    ge, gc, _ = gpu_exact(a, b, "hash", ctx)
    assert O.wide_to_int(gc) == [n * (2**64 - 1)]
    if part == 2:
        (ea, _), (eb, _) = I.config(2, scale=0.08)
        a, b = (ea, _big(rng, len(ea))), (eb, _big(rng, len(eb)))
        for slots in (2048, 4096, 8192):
            ctx.set_tune(hash_bin_slots=slots)
            check_exact(a, b, "hash", f"simplex, bins of {slots} slots", ctx)


@pytest.mark.parametrize("slots", [2048, 4096])
def test_exact_full_bin_recovers(slots):
    """128-bit sums in the grouped layout: slots + 1000 distinct codes in one
    bin overflow its table, and the bin is redone by code interval (62-bit
    coefficients times a 62-bit constant: every product carries into the high
    word)."""
    ctx = kp.context()
    ctx.set_tune(hash_partitioned=2, hash_bin_slots=slots)
    rng = np.random.default_rng(77 + slots)
    a, b = adversarial_codes(slots, _big(rng, slots + 1000))
    b = (b[0], np.array([3 * 2**60 + 12345], np.int64))
    check_exact(a, b, "hash", f"{slots + 1000} codes in one bin of {slots}", ctx)


def test_exact_split_windows_and_small_windows():
    """Windows split across tasks add their 128-bit partial sums into the HBM
    accumulator with a carry between the words."""
    ctx = kp.context()
    rng = np.random.default_rng(5)
    (ea, _), (eb, _) = I.config(2, scale=0.2)
    a, b = (ea, _big(rng, len(ea))), (eb, _big(rng, len(eb)))
    for window, block, tpc in ((4096, 256, 64), (8192, 512, 16), (18432, 1024, 1)):
        ctx.set_tune(window=window, block=block, tasks_per_cu=tpc)
        check_exact(a, b, "dense", f"window {window} block {block} tasks/CU {tpc}", ctx)


def test_exact_carries_and_cancellation():
    """All-ones low words carry on every add; products that cancel exactly
    leave no term."""
    ea = np.array([[0, 0], [1, 0], [0, 1], [1, 0]], np.int32)
    eb = np.array([[0, 0], [2, 1], [1, 1]], np.int32)
    for what, ca, cb in (
            ("largest magnitudes", [2**63 - 1, -2**63, 2**63 - 1, -2**63 + 1],
             [2**63 - 1, -2**63, 2**63 - 1]),
            ("cancelling pair", [5, 7, -3, -7], [11, 2**62, -2**62]),
            ("products of -1 (low word all ones)", [-1, -1, -1, -1], [1, 1, 1])):
        a = (ea, np.array(ca, np.int64))
        b = (eb, np.array(cb, np.int64))
        for mode in ("dense", "hash"):
            check_exact(a, b, mode, what)
    # many adds of (2^32 + 1)(2^32 - 1) = 2^64 - 1 into one code: every add
    # after the first carries out of the low word
    n = 4097
    a = (np.zeros((n, 1), np.int32), np.full(n, 2**32 + 1, np.int64))
    b = (np.zeros((1, 1), np.int32), np.array([2**32 - 1], np.int64))
    for mode in ("dense", "hash"):
        say("one code,", n, "adds", mode)
        ge, gc, _ = gpu_exact(a, b, mode)
        assert O.wide_to_int(gc) == [n * (2**64 - 1)]


def test_exact_fateman_closed_form():
    """Section 5: f = (1+x+y+z+t)^30, g = f + 1.  f g = (1+...)^60 + (1+...)^30,
    whose largest coefficient, 60!/(12!)^5 + ..., lies between 2^127 and
    2^128: every one of the 635,376 terms must be the exact multinomial sum
    when the 128 bits are read as unsigned (all coefficients are positive)."""
    fe, fc = I.fateman(30)
    ge_, gc_ = I.fateman(30, plus_one=True)
    say("Fateman k=30, exact, dense")
    ex, co, _ = gpu_exact((fe, fc), (ge_, gc_), "dense")
    assert len(ex) == math.comb(64, 4)
    f = [math.factorial(i) for i in range(61)]
    got = [v % 2**128 for v in O.wide_to_int(co)]   # the unsigned reading
    assert got == kp.to_pyint(co, unsigned=True)
    big = 0
    for e, v in zip(ex.tolist(), got):
        s = sum(e)
        want = f[60] // (f[60 - s] * f[e[0]] * f[e[1]] * f[e[2]] * f[e[3]])
        if s <= 30:
            want += f[30] // (f[30 - s] * f[e[0]] * f[e[1]] * f[e[2]] * f[e[3]])
        assert v == want, (e, v, want)
        big = max(big, v)
    assert 2**127 < big < 2**128


def test_exact_fateman_hash_closed_form():
    k = 12
    fe, fc = I.fateman(k)
    ge_, gc_ = I.fateman(k, plus_one=True)
    c = 3**25   # scaled so that the products pass 2^64 (the factors stay below 2^63)
    say("scaled Fateman k=12, exact, hash")
    ex, co, _ = gpu_exact((fe, fc * c), (ge_, gc_ * c), "hash")
    assert len(ex) == math.comb(2 * k + 4, 4)
    for e, v in zip(ex.tolist(), O.wide_to_int(co)):
        e = tuple(e)
        want = c * c * (I.multinomial(2 * k, e) + (I.multinomial(k, e) if sum(e) <= k else 0))
        assert v == want


@pytest.mark.parametrize("mode", ["dense", "hash"])
def test_exact_truncated(mode):
    ctx = kp.context()
    rng = np.random.default_rng(11)
    (ea, _), (eb, _) = I.config(2, scale=0.06)
    a, b = (ea, _big(rng, len(ea))), (eb, _big(rng, len(eb)))
    w, D = [1, 1, 1, 1], 20
    say("exact truncated", mode)
    with ctx.truncation(w, D):
        ge, gc, _ = gpu_exact(a, b, mode, ctx)
    oe, oc, _ = O.laurent_mul(a[0], a[1], b[0], b[1], threads=4, exact=True)
    keep = oe.astype(np.int64) @ np.asarray(w, np.int64) <= D
    assert keep.sum() > 0 and (~keep).sum() > 0
    assert_exact([ge], gc, [oe[keep]], oc[keep], "exact truncated")


def test_exact_codes_path_batch_and_errors():
    import torch
    ctx = kp.context()
    rng = np.random.default_rng(17)
    (ea, _), (eb, _) = I.config(1, scale=0.4)
    ca, cb = _big(rng, len(ea)), _big(rng, len(eb))
    oe, oc, _ = O.laurent_mul(ea, ca, eb, cb, exact=True)
    lay = kp.layout_product(3, 0, ea.min(0), ea.max(0), eb.min(0), eb.max(0))
    ka, _ = kp.encode(lay, 0, dev(ea))
    kb, _ = kp.encode(lay, 1, dev(eb))
    for mode in ("dense", "hash"):
        say("exact codes path", mode)
        codes, coef, _ = kp.mul_laurent_codes(lay, ka, dev(ca), kb, dev(cb), mode, exact=True)
        assert_exact([kp.decode(lay, codes).cpu().numpy()], coef.cpu().numpy(), [oe], oc,
                     f"codes path {mode}")
    # batched, eager and replayed graph
    for graph in (False, True):
        say("exact batch", "graph" if graph else "eager")
        bt = kp.Batch(2, ctx)
        outs = []
        for mode in ("dense", "hash"):
            _, cap, ws = kp.mul_bound(lay, False, kp.KP_I128, mode, len(ca), len(cb), ctx)
            out = (torch.empty(cap, dtype=torch.int64, device="cuda"),
                   torch.empty((cap, 2), dtype=torch.int64, device="cuda"),
                   torch.empty(1, dtype=torch.int64, device="cuda"))
            wbuf = torch.empty(max(ws, 256), dtype=torch.uint8, device="cuda")
            tid = bt.add_laurent(lay, ka, dev(ca), kb, dev(cb), out, wbuf, mode, exact=True)
            outs.append((tid, out, wbuf))
        for rep in range(2 if graph else 1):
            for _, (_, ov, on), _ in outs:
                on.fill_(-99)
                ov.zero_()
            bt.launch(graph=graph)
            for tid, (oc_, ov, on), _ in outs:
                n = bt.status(tid)
                ex = kp.decode(lay, oc_[:n]).cpu().numpy()
                assert_exact([ex], ov[:n].cpu().numpy(), [oe], oc, f"batch launch {rep}")
    # exact products need int64 factors; Poisson series have no exact mode
    with pytest.raises(ValueError):
        kp.mul_laurent(kp.Poly(dev(ea), dev(ca.astype(np.float64))),
                       kp.Poly(dev(eb), dev(cb.astype(np.float64))), exact=True)
    with pytest.raises(kp.KPError) as e:
        kp.mul_bound(kp.layout_product(1, 1, [0], [1], [0], [1], [1], [1]), True, kp.KP_I128,
                     "auto", 4, 4, ctx)
    assert e.value.status == kp.KP_E_DTYPE
    # empty factor
    say("exact empty factor")
    ge, gc, _ = gpu_exact((ea[:0], ca[:0]), (eb, cb), "auto")
    assert len(ge) == 0 and gc.shape == (0, 2)



P31 = (1 << 31) - 1   # prime; residues below 2^31 keep every product within 64 bits


def _eval_mod(exps, coef_mod, point):
    """sum_i c_i prod_v point_v^e_iv modulo P31 (exponents >= 0), vectorised."""
    acc = np.asarray(coef_mod, np.uint64) % P31
    for v in range(exps.shape[1]):
        e = exps[:, v].astype(np.int64)
        assert e.min() >= 0
        table = np.ones(int(e.max()) + 1, np.uint64)
        for k in range(1, len(table)):
            table[k] = table[k - 1] * np.uint64(point[v]) % P31
        acc = acc * table[e] % P31
    return int(acc.sum(dtype=object) % P31)


def _words_mod(words):
    """(hi * 2^64 + lo) mod P31 of int64 [n, 2] words, the sum read unsigned."""
    lo = words[:, 0].view(np.uint64)
    hi = words[:, 1].view(np.uint64)
    t = np.uint64((1 << 64) % P31)
    return ((hi % P31) * t + lo % P31) % P31


def test_exact_mp_sparse_full_size_evaluation():
    """Section 5's sparse benchmark at full size (3.8e7 pairs, 5.8 million
    terms, products up to 1.3e22): the exact product evaluated modulo a
    prime at random points equals f(point) g(point), and its low words are
    the int64 product."""
    f, g = I.mp_sparse(12, "f"), I.mp_sparse(12, "g")
    say("MP-sparse k=12, exact, auto mode")
    ex, co, _ = gpu_exact(f, g, "auto")
    say("MP-sparse k=12, int64, auto mode")
    pa = kp.Poly(dev(f[0]), dev(f[1]))
    pb = kp.Poly(dev(g[0]), dev(g[1]))
    r, _ = kp.mul_laurent(pa, pb)
    e64, c64 = r.exps.cpu().numpy(), r.coef.cpu().numpy()
    assert len(ex) == 5821335
    # low words against the int64 product (both orders: sort by code-like key)
    assert_exact([ex], co[:, 0], [e64], c64, "low words of the exact product")
    # the values: nonnegative factors, so every sum is nonnegative and the
    # unsigned reading applies; all fit far below 2^127 here
    assert (co[:, 1] >= 0).all()
    rng = np.random.default_rng(1231)
    cm = _words_mod(co)
    for _ in range(2):
        pt = [int(x) for x in rng.integers(2, P31, 5)]
        lhs = _eval_mod(ex, cm, pt)
        rhs = _eval_mod(f[0], np.asarray(f[1], np.uint64) % P31, pt) * \
            _eval_mod(g[0], np.asarray(g[1], np.uint64) % P31, pt) % P31
        assert lhs == rhs
