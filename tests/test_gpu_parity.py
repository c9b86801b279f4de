"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

int64 results must be bit-exact; fp64 results must satisfy
|gpu - oracle| <= 1e-13 * sum|contributions| per term.  Each case prints what
it runs before touching the GPU.
"""
import math

import numpy as np
import pytest

import oracle as O
import paper_1004_4548_amd as kp
from paper_1004_4548_amd import inputs as I
from tests.helpers import (P61, adversarial_codes, assert_exact, assert_tolerance,
                           eval_mod2_64_device, eval_modp_device, parallel_chunks)

pytestmark = pytest.mark.gpu
TOL = 1e-13


def _torch():
    import torch
    return torch


def dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def say(*a):
    print("[case]", *a, flush=True)


def gpu_laurent(a, b, mode="auto", ctx=None):
    ctx = ctx or kp.context()
    pa = kp.Poly(dev(np.asarray(a[0], np.int32)), dev(a[1]))
    pb = kp.Poly(dev(np.asarray(b[0], np.int32)), dev(b[1]))
    r, lay = kp.mul_laurent(pa, pb, mode=mode, ctx=ctx)
    return r.exps.cpu().numpy(), r.coef.cpu().numpy(), lay


def gpu_poisson(a, b, mode="auto", ctx=None):
    ctx = ctx or kp.context()
    sa = kp.PoissonSeries(dev(np.asarray(a[0], np.int32)), dev(np.asarray(a[1], np.int32)),
                          dev(np.asarray(a[2], np.uint8)), dev(np.asarray(a[3], np.float64)))
    sb = kp.PoissonSeries(dev(np.asarray(b[0], np.int32)), dev(np.asarray(b[1], np.int32)),
                          dev(np.asarray(b[2], np.uint8)), dev(np.asarray(b[3], np.float64)))
    r, lay = kp.mul_poisson(sa, sb, mode=mode, ctx=ctx)
    return (r.x.cpu().numpy(), r.y.cpu().numpy(), r.is_sin.cpu().numpy(),
            r.coef.cpu().numpy(), lay)


def check_laurent(a, b, mode, what, ctx=None):
    say(what, mode, len(a[1]), "x", len(b[1]), a[1].dtype)
    ge, gc, lay = gpu_laurent(a, b, mode, ctx)
    oe, oc, oab = O.laurent_mul(a[0], a[1], b[0], b[1], threads=4)
    if np.asarray(a[1]).dtype == np.float64:
        assert_tolerance([ge], gc, [oe], oc, oab, TOL, what)
    else:
        assert_exact([ge], gc, [oe], oc, what)
    return ge, gc, lay


@pytest.fixture(autouse=True)
def _fresh_ctx():
    ctx = kp.context()
    saved = ctx.tune
    yield
    ctx.clear_truncation()
    ctx.set_tune(**{f: getattr(saved, f) for f, _ in kp.Tune._fields_})


# ------------------------------------------------------------------ codec
def test_minmax_encode_decode_on_device():
    torch = _torch()
    (ea, ca), (eb, cb) = I.config(1)
    mm = kp.minmax(dev(ea)).cpu().numpy()
    np.testing.assert_array_equal(mm, np.concatenate([ea.min(0), ea.max(0)]))
    lay = kp.layout_product(3, 0, ea.min(0), ea.max(0), eb.min(0), eb.max(0))
    ka, _ = kp.encode(lay, 0, dev(ea))
    kb, _ = kp.encode(lay, 1, dev(eb))
    np.testing.assert_array_equal(ka.cpu().numpy(), kp.encode_host(lay, 0, ea)[0])
    np.testing.assert_array_equal(kb.cpu().numpy(), kp.encode_host(lay, 1, eb)[0])
    s = (ka[:100] + kb[:100]).contiguous()
    np.testing.assert_array_equal(kp.decode(lay, s).cpu().numpy(), ea[:100] + eb[:100])
    # Table 1 codes on the device
    l1 = kp.layout_product(3, 0, [0, 0, 0], [3, 3, 3], [0, 0, 0], [0, 0, 0])
    e = np.array([[0, 0, 0], [1, 0, 0], [3, 0, 0], [0, 1, 0], [0, 2, 0], [3, 3, 3]], np.int32)
    np.testing.assert_array_equal(kp.encode(l1, 0, dev(e))[0].cpu().numpy(), [0, 1, 3, 4, 8, 63])
    # empty input
    mm0 = kp.minmax(torch.zeros((0, 2), dtype=torch.int32, device="cuda")).cpu().numpy()
    assert mm0.tolist() == [0, 0, -1, -1]


def test_device_range_and_canonical_errors():
    lay = kp.layout_product(2, 0, [0, 0], [3, 3], [0, 0], [3, 3])
    with pytest.raises(kp.KPError) as e:
        kp.encode(lay, 0, dev(np.array([[1, 1], [4, 0]], np.int32)))
    assert e.value.status == kp.KP_E_RANGE
    lp = kp.layout_product(1, 2, [0], [1], [0], [1], [2, 2], [2, 2])
    with pytest.raises(kp.KPError) as e:
        kp.encode(lp, 0, dev(np.array([[0]], np.int32)), dev(np.array([[-1, 1]], np.int32)),
                  dev(np.array([0], np.uint8)))
    assert e.value.status == kp.KP_E_NONCANONICAL
    # the context recovers after an error
    kx, _ = kp.encode(lay, 0, dev(np.array([[1, 1]], np.int32)))
    assert kx.cpu().tolist() == [1 + 7 * 1]      # product widths are 7


def test_poisson_decode_round_trip_on_device():
    lay = kp.layout_product(2, 3, [-2, 0], [2, 3], [-1, 0], [1, 1], [2, 1, 3], [1, 2, 0])
    rng = np.random.default_rng(3)
    keys = rng.integers(0, lay.nkeys, size=5000, dtype=np.int64)
    x, y, t = kp.decode(lay, dev(keys), poisson=True)
    hx, hy, ht = kp.decode_host(lay, keys, poisson=True)
    np.testing.assert_array_equal(x.cpu().numpy(), hx)
    np.testing.assert_array_equal(y.cpu().numpy(), hy)
    np.testing.assert_array_equal(t.cpu().numpy(), ht)


# ------------------------------------------------------------------ Laurent
@pytest.mark.parametrize("mode", ["dense", "hash", "auto"])
def test_laurent_500x500_box(mode):
    a, b = I.config(1)
    check_laurent(a, b, mode, "3 vars [-5,5], 500 x 500")


@pytest.mark.parametrize("mode", ["dense", "hash"])
def test_laurent_simplex_2000(mode):
    a, b = I.config(2, scale=0.2)
    check_laurent(a, b, mode, "4-var simplex deg 20, 2000 x 2000")


def test_laurent_sparse_3000():
    a, b = I.config(3, scale=0.1)
    check_laurent(a, b, "auto", "6 vars [0,80], 3000 x 3000 (hash)")
    with pytest.raises(kp.KPError) as e:       # 161^6 codes: too many for dense mode
        gpu_laurent(a, b, "dense")
    assert e.value.status == kp.KP_E_MODE


@pytest.mark.parametrize("mode", ["dense", "hash"])
def test_laurent_fp64(mode):
    (ea, _), (eb, _) = I.config(1)
    rng = np.random.default_rng(12)
    a = (ea, rng.standard_normal(len(ea)))
    b = (eb, rng.standard_normal(len(eb)))
    check_laurent(a, b, mode, "fp64 N(0,1) 500 x 500")
    # dyadic coefficients: every sum is exact, so the result is bit-exact
    a = (ea, rng.integers(-999, 1000, len(ea)) / 64.0)
    b = (eb, rng.integers(-999, 1000, len(eb)) / 8.0)
    say("fp64 dyadic", mode)
    ge, gc, _ = gpu_laurent(a, b, mode)
    oe, oc, _ = O.laurent_mul(a[0], a[1], b[0], b[1])
    nz = oc != 0
    assert_exact([ge], gc, [oe[nz]], oc[nz], "dyadic fp64")


@pytest.mark.parametrize("mode", ["dense", "hash"])
def test_laurent_coefficient_widths(mode):
    # 24-bit, 32-bit and full 64-bit (wrapping) coefficient paths
    (ea, _), (eb, _) = I.config(1, scale=0.4)
    rng = np.random.default_rng(5)
    for lo, hi in ((-(2**23), 2**23 - 1), (-(2**31), 2**31 - 1), (-(2**62), 2**62)):
        a = (ea, rng.integers(lo, hi, len(ea), dtype=np.int64))
        b = (eb, rng.integers(lo, hi, len(eb), dtype=np.int64))
        check_laurent(a, b, mode, f"coefficients in [{lo},{hi}]")


def test_dense_narrow_kind_largest_products():
    """The narrowest coefficient kind (both factors in [0, 2^16), one 24-bit
    multiply per pair) at its largest products, just below 2^32, whose sums
    pass 2^32 many times over: in whole windows and in windows split across
    tasks."""
    ctx = kp.context()
    (ea, _), (eb, _) = I.config(1, scale=0.6)
    rng = np.random.default_rng(65535)
    cases = [("all 65535", np.full(len(ea), 65535, np.int64), np.full(len(eb), 65535, np.int64)),
             ("random [0, 65535]", rng.integers(0, 65536, len(ea)), rng.integers(0, 65536, len(eb)))]
    for window, block, tpc in ((18432, 1024, 1), (2048, 256, 64)):
        ctx.set_tune(window=window, block=block, tasks_per_cu=tpc)
        for what, ca, cb in cases:
            check_laurent((ea, ca), (eb, cb), "dense", f"{what}, window {window} tasks/CU {tpc}")


@pytest.mark.parametrize("na,nb", [(1, 1), (1, 700), (63, 65), (4095, 4097), (8193, 130)])
def test_laurent_ragged_sizes(na, nb):
    rng = np.random.default_rng(na * 7 + nb)
    a = (rng.integers(-6, 7, (na, 3)).astype(np.int32), rng.integers(-50, 50, na))
    b = (rng.integers(-4, 9, (nb, 3)).astype(np.int32), rng.integers(-50, 50, nb))
    for mode in ("dense", "hash"):
        check_laurent(a, b, mode, f"ragged {na} x {nb} (duplicates allowed)")


def test_laurent_many_windows_and_split_windows():
    # small windows and many tasks per CU: many windows per product, busy
    # windows split into several tasks whose partial windows are combined
    ctx = kp.context()
    a, b = I.config(2, scale=0.3)
    for window, block, tpc in ((2048, 256, 64), (4096, 512, 16), (16384, 1024, 8),
                               (18432, 1024, 1)):
        ctx.set_tune(window=window, block=block, tasks_per_cu=tpc)
        check_laurent(a, b, "dense", f"window {window} block {block} tasks/CU {tpc}")
        a64 = (a[0], a[1].astype(np.float64) / 4)
        b64 = (b[0], b[1].astype(np.float64))
        check_laurent(a64, b64, "dense", f"fp64 window {window}")


def test_dense_layout_of_many_windows():
    """A product of more than 4096 windows lays out its tasks in the count
    kernel's last workgroup (smaller ones in the items kernel): both paths
    against the oracle."""
    ctx = kp.context()
    rng = np.random.default_rng(4096)
    ea = np.unique(rng.integers(0, 6_000_000, 2500)).reshape(-1, 1).astype(np.int32)
    eb = np.unique(rng.integers(0, 6_000_000, 1500)).reshape(-1, 1).astype(np.int32)
    a = (ea, rng.integers(-9, 10, len(ea)))
    b = (eb, rng.integers(-9, 10, len(eb)))
    for window in (2048, 18432):   # about 5900 and 650 windows
        ctx.set_tune(window=window, block=1024, tasks_per_cu=2)
        check_laurent(a, b, "dense", f"univariate over 12e6 codes, window {window}")


def test_laurent_univariate_long_range():
    # one variable, codes spanning many windows with sparse hits
    rng = np.random.default_rng(9)
    ea = np.unique(rng.integers(-200000, 200000, 3000)).reshape(-1, 1).astype(np.int32)
    eb = np.unique(rng.integers(0, 300000, 2000)).reshape(-1, 1).astype(np.int32)
    a = (ea, rng.integers(-9, 10, len(ea)))
    b = (eb, rng.integers(-9, 10, len(eb)))
    for mode in ("dense", "hash"):
        check_laurent(a, b, mode, "univariate, 700k codes")


def test_laurent_empty_and_cancelling():
    torch = _torch()
    ctx = kp.context()
    a = kp.Poly(torch.zeros((0, 2), dtype=torch.int32, device="cuda"),
                torch.zeros(0, dtype=torch.int64, device="cuda"))
    b = kp.Poly(dev(np.array([[1, 2]], np.int32)), dev(np.array([3], np.int64)))
    for mode in ("dense", "hash", "auto"):
        r, _ = kp.mul_laurent(a, b, mode=mode)
        assert r.coef.shape[0] == 0
        r, _ = kp.mul_laurent(b, a, mode=mode)
        assert r.coef.shape[0] == 0
    # (1 + x)(1 - x): the x term cancels and is dropped
    p = (np.array([[0], [1]], np.int32), np.array([1, 1], np.int64))
    q = (np.array([[0], [1]], np.int32), np.array([1, -1], np.int64))
    for mode in ("dense", "hash"):
        ge, gc, _ = gpu_laurent(p, q, mode)
        order = np.argsort(ge[:, 0])
        assert ge[order, 0].tolist() == [0, 2] and gc[order].tolist() == [1, -1]


def test_capacity_errors():
    ctx = kp.context()
    a, b = I.config(1, scale=0.4)
    lay = kp.layout_product(3, 0, a[0].min(0), a[0].max(0), b[0].min(0), b[0].max(0))
    ka, _ = kp.encode(lay, 0, dev(a[0]))
    kb, _ = kp.encode(lay, 1, dev(b[0]))
    torch = _torch()
    for mode in ("dense", "hash"):
        small = (torch.empty(10, dtype=torch.int64, device="cuda"),
                 torch.empty(10, dtype=torch.int64, device="cuda"),
                 torch.empty(1, dtype=torch.int64, device="cuda"))
        with pytest.raises(kp.KPError) as e:
            kp.mul_laurent_codes(lay, ka, dev(a[1]), kb, dev(b[1]), mode, out=small)
        assert e.value.status == kp.KP_E_CAPACITY
    # a forced hash table smaller than the result fills up: reported, not hung
    ctx.set_tune(hash_capacity=64, hash_partitioned=0)
    with pytest.raises(kp.KPError) as e:
        kp.mul_laurent_codes(lay, ka, dev(a[1]), kb, dev(b[1]), "hash")
    assert e.value.status == kp.KP_E_CAPACITY
    # async: the count carries -(status)
    on = kp.mul_laurent_codes(lay, ka, dev(a[1]), kb, dev(b[1]), "hash",
                              flags=kp.KP_FLAG_ASYNC)[2]
    assert int(on.item()) == -kp.KP_E_CAPACITY
    with pytest.raises(kp.KPError):
        ctx.sync_check()
    ctx.set_tune(hash_capacity=0)
    check_laurent(a, b, "hash", "after recovery")


def _with_partitioning(ctx, mode):
    ctx.set_tune(hash_partitioned=mode)


@pytest.mark.parametrize("part", [0, 2])
def test_hash_layouts_match_oracle(part):
    """Both hash layouts (global table, products partitioned through HBM into
    LDS tables), forced, on sparse, colliding, fp64, ragged and duplicate-heavy
    products."""
    ctx = kp.context()
    _with_partitioning(ctx, part)
    a, b = I.config(3, scale=0.1)
    check_laurent(a, b, "hash", f"sparse 3000 (partitioned={part})")
    a, b = I.config(1)
    check_laurent(a, b, "hash", f"box 500 x 500, many products per code (partitioned={part})")
    a, b = I.config(2, scale=0.05)
    a64 = (a[0], a[1].astype(np.float64) / 8)
    check_laurent(a64, (b[0], b[1].astype(np.float64)), "hash", f"fp64 simplex (partitioned={part})")
    rng = np.random.default_rng(31 + part)
    for na, nb in ((1, 1), (1, 700), (63, 65), (257, 1)):
        ra = (rng.integers(-40, 40, (na, 2)).astype(np.int32), rng.integers(-9, 10, na))
        rb = (rng.integers(-40, 40, (nb, 2)).astype(np.int32), rng.integers(-9, 10, nb))
        check_laurent(ra, rb, "hash", f"ragged {na} x {nb} (partitioned={part})")
    # three product codes only: every bin but three is empty, each busy bin
    # holds one code many times
    da = (rng.integers(0, 2, (600, 1)).astype(np.int32), rng.integers(1, 50, 600))
    db = (rng.integers(0, 2, (500, 1)).astype(np.int32), rng.integers(1, 50, 500))
    check_laurent(da, db, "hash", f"3 codes from 3e5 products (partitioned={part})")


@pytest.mark.parametrize("part", [0, 2])
def test_poisson_hash_layouts(part):
    ctx = kp.context()
    _with_partitioning(ctx, part)
    a, b = I.config(4, scale=0.06)
    check_poisson(a, b, f"poisson hash (partitioned={part})", mode="hash")


@pytest.mark.parametrize("slots", [2048, 4096, 8192])
def test_partitioned_bin_tables(slots):
    """Every size of a bin's LDS table (bins hold half a table of products on
    average) on sparse, duplicate-heavy, fp64, truncated and Poisson
    products."""
    ctx = kp.context()
    ctx.set_tune(hash_partitioned=2, hash_bin_slots=slots)
    a, b = I.config(3, scale=0.1)
    check_laurent(a, b, "hash", f"sparse 3000, bins of {slots}")
    a, b = I.config(1)
    check_laurent(a, b, "hash", f"box 500 x 500, bins of {slots}")
    a, b = I.config(2, scale=0.05)
    a64 = (a[0], a[1].astype(np.float64) / 8)
    check_laurent(a64, (b[0], b[1].astype(np.float64)), "hash", f"fp64 simplex, bins of {slots}")
    what, ta, tb, w, D = _trunc_cases()[-1]
    say("truncated", what, "bins of", slots)
    with ctx.truncation(w, D):
        ge, gc, _ = gpu_laurent(ta, tb, "hash", ctx)
    oe, oc, _ = O.laurent_mul_truncated(ta[0], ta[1], tb[0], tb[1], w, D, threads=4)
    assert_exact([ge], gc, [oe], oc, what)
    pa, pb = I.config(4, scale=0.06)
    check_poisson(pa, pb, f"poisson hash, bins of {slots}", mode="hash")


@pytest.mark.parametrize("slots", [2048, 4096, 8192])
def test_two_level_grouping_recovers_from_full_bins(slots):
    """With the two-level hash grouping forced, the adversarial codes put
    slots + 1000 distinct codes into one bin: its table overflows, the bin is
    redone one code interval at a time, and the product is the oracle's
    (int64 and fp64); the next product is unaffected."""
    ctx = kp.context()
    ctx.set_tune(hash_partitioned=2, hash_bin_slots=slots, hash_grouping=1)
    a, b = adversarial_codes(slots)
    check_laurent(a, b, "hash", f"two-level grouping, {slots + 1000} codes in one bin of {slots}", ctx)
    check_laurent((a[0], a[1].astype(np.float64) * 0.5), (b[0], b[1].astype(np.float64)), "hash",
                  f"two-level grouping, fp64, one bin of {slots}", ctx)
    a2, b2 = I.config(3, scale=0.03)
    check_laurent(a2, b2, "hash", f"after the overflowing bin, bins of {slots}", ctx)


@pytest.mark.parametrize("slots", [2048, 4096, 8192])
def test_range_grouping_recovers_from_full_bins(slots):
    """Grouped by code range (the default), the same adversarial codes give
    the oracle's product in auto mode.  With at most one bin per range
    (hash_max_bin_bits = 0) every bin of the sparse products holds several
    tables' worth of distinct codes, overflows, and is redone one hash
    interval at a time: still the oracle's product, int64 and fp64."""
    ctx = kp.context()
    ctx.set_tune(hash_bin_slots=slots)
    a, b = adversarial_codes(slots)
    check_laurent(a, b, "auto", f"adversarial codes grouped by range, bins of {slots}", ctx)
    ctx.set_tune(hash_max_bin_bits=0)
    a, b = I.config(3, scale=0.1)
    check_laurent(a, b, "hash", f"one bin per range, bins of {slots}", ctx)
    check_laurent((a[0], a[1].astype(np.float64) / 4), (b[0], b[1].astype(np.float64)), "hash",
                  f"one bin per range, fp64, bins of {slots}", ctx)


@pytest.mark.parametrize("grouping", [0, 1, 2])
@pytest.mark.parametrize("cfg,scale,fp", [(3, 0.1, False), (3, 0.05, True), (2, 0.2, False),
                                          (1, 1.0, True)])
def test_grouped_hash_matches_oracle(grouping, cfg, scale, fp):
    """Every grouping of the hash products against the oracle (0 automatic,
    1 two levels, 2 ranges): the highly sparse product (few collisions: each
    range's terms fill its own slots, the few beyond the count are moved), the
    simplex forced into hash mode (many products per code: more entries than
    result slots, so a shared counter places the terms), and the small box."""
    ctx = kp.context()
    ctx.set_tune(hash_partitioned=2, hash_grouping=grouping)
    a, b = I.config(cfg, scale=scale)
    if fp:
        a, b = (a[0], a[1].astype(np.float64) * 0.75), (b[0], b[1].astype(np.float64))
    check_laurent(a, b, "hash", f"grouped {grouping}, config {cfg} x{scale}", ctx)


def test_range_grouping_wide_int64_entries():
    """int64 products too wide to sit above the hash bits of an 8-byte entry
    take 16-byte entries (and the grouping kernel's shorter chunks): the
    ranges against the oracle, then a factor holding every term of B twice
    with opposite signs, whose product is zero term by term."""
    ctx = kp.context()
    ctx.set_tune(hash_partitioned=2, hash_grouping=2)
    a, b = I.config(3, scale=0.1)
    a = (a[0], np.asarray(a[1], np.int64) << 24)
    check_laurent(a, b, "hash", "ranges, int64 products past the packed width", ctx)
    bb = np.asarray(b[1], np.int64)
    both = (np.concatenate([b[0], b[0]]), np.concatenate([bb, -bb]))
    ge, gc, _ = check_laurent(a, both, "hash", "ranges, every sum cancels", ctx)
    assert len(gc) == 0


def test_repeat_runs_bit_identical():
    a, b = I.config(2, scale=0.2)
    r1 = gpu_laurent(a, b, "hash")
    r2 = gpu_laurent(a, b, "hash")
    assert_exact([r1[0]], r1[1], [r2[0]], r2[1], "hash repeat")
    d1 = gpu_laurent(a, b, "dense")
    assert_exact([d1[0]], d1[1], [r1[0]], r1[1], "dense vs hash")
    # dense output is ascending in code
    lay = d1[2]
    codes = sum((d1[0][:, v].astype(np.int64) - lay.xmin[v]) * lay.xc[v] for v in range(4))
    assert (np.diff(codes) > 0).all()


# ------------------------------------------------------------------ Poisson
def _pkeys(x, y, t):
    return [x, y, np.asarray(t).reshape(-1, 1)]


def check_poisson(a, b, what, nx=3, ny=6, mode="auto"):
    say(what, len(a[3]), "x", len(b[3]))
    gx, gy, gt, gc, lay = gpu_poisson(a, b, mode)
    ox, oy, ot, oc, oab = O.poisson_mul(a, b, nx, ny, threads=4)
    assert_tolerance(_pkeys(gx, gy, gt), gc, _pkeys(ox, oy, ot), oc, oab, TOL, what)
    return gx, gy, gt, gc


@pytest.mark.parametrize("w,H", [([1] * 6, 6), ([1] * 6, 12), ([1, 2, 1, 0, 3, 1], 10),
                                 ([1] * 6, 0), ([1] * 6, -1), ([1] * 6, 10**6)])
def test_poisson_harmonic_truncation_matches_oracle(w, H):
    """Truncation by weighted harmonic order: the whole-product path and the
    codes path (grouped hash, automatic mode) against the oracle's full
    product filtered; the limit 0 keeps the terms without harmonics, -1 none,
    a huge one all."""
    ctx = kp.context()
    a, b = I.config(4, scale=0.06)
    say("poisson truncated by harmonic order", w, H, len(a[3]), "x", len(b[3]))
    ox, oy, ot, oc, oab = O.poisson_mul_truncated(a, b, 3, 6, w, H, threads=4)
    with ctx.harmonic_truncation(w, H):
        gx, gy, gt, gc, lay = gpu_poisson(a, b, "auto", ctx)
        assert_tolerance(_pkeys(gx, gy, gt), gc, _pkeys(ox, oy, ot), oc, oab, TOL,
                         f"harmonic {w} <= {H}")
        # the codes path: the same terms as keys
        dts = (np.int32, np.int32, np.uint8, np.float64)
        sa = [dev(np.asarray(a[k], dts[k])) for k in range(4)]
        sb = [dev(np.asarray(b[k], dts[k])) for k in range(4)]
        ka = kp.encode(lay, 0, sa[0], sa[1], sa[2], ctx=ctx)
        kb = kp.encode(lay, 1, sb[0], sb[1], sb[2], ctx=ctx)
        keys, coef, n = kp.mul_poisson_codes(lay, (ka[0], ka[1], sa[2], sa[3]),
                                             (kb[0], kb[1], sb[2], sb[3]), "auto", ctx)
        assert int(n) == len(gc)
        if H >= 0:
            x, y, t = kp.decode(lay, keys, poisson=True, ctx=ctx)
            assert_tolerance(_pkeys(x.cpu().numpy(), y.cpu().numpy(), t.cpu().numpy()),
                             coef.cpu().numpy(), _pkeys(ox, oy, ot), oc, oab, TOL,
                             f"harmonic codes path {w} <= {H}")


def test_poisson_harmonic_truncation_large_multipliers():
    """Multipliers past a signed byte (up to 200): the orders come from each
    factor term's order, pairs whose orders differ by more than the limit make
    no piece, and the bins drop the terms over it; against the oracle."""
    ctx = kp.context()
    rng = np.random.default_rng(12)
    n = 300
    def series(seed):
        r = np.random.default_rng(seed)
        y = r.integers(-200, 201, (n, 2)).astype(np.int32)
        first = np.where(y[:, 0] != 0, y[:, 0], y[:, 1])
        y[first < 0] *= -1                       # canonical: first nonzero positive
        t = r.integers(0, 2, n).astype(np.uint8)
        t[(y == 0).all(1)] = 0                   # no sin of the zero vector
        x = r.integers(-2, 3, (n, 1)).astype(np.int32)
        key = np.concatenate([x, y, t[:, None].astype(np.int32)], 1)
        _, keep = np.unique(key, axis=0, return_index=True)
        keep = np.sort(keep)
        return x[keep], y[keep], t[keep], r.standard_normal(len(keep))
    a, b = series(1), series(2)
    for w, H in (([1, 1], 150), ([1, 2], 300), ([0, 1], 40)):
        say("poisson, multipliers up to 200, harmonic", w, H)
        ox, oy, ot, oc, oab = O.poisson_mul_truncated(a, b, 1, 2, w, H, threads=4)
        with ctx.harmonic_truncation(w, H):
            gx, gy, gt, gc, _ = gpu_poisson(a, b, "auto", ctx)
        assert_tolerance(_pkeys(gx, gy, gt), gc, _pkeys(ox, oy, ot), oc, oab, TOL,
                         f"large multipliers {w} <= {H}")


def test_poisson_harmonic_truncation_modes_and_clear():
    """Dense mode is refused under a harmonic truncation; clearing it gives the
    whole product back; a Laurent product is unaffected by it."""
    ctx = kp.context()
    a, b = I.config(4, scale=0.02)
    with ctx.harmonic_truncation([1] * 6, 4):
        say("harmonic truncation, forced dense mode")
        with pytest.raises(kp.KPError) as err:
            gpu_poisson(a, b, "dense", ctx)
        assert err.value.status == kp.KP_E_MODE
        la, lb = I.config(1, scale=0.2)
        check_laurent(la, lb, "auto", "a Laurent product under a harmonic truncation", ctx)
    check_poisson(a, b, "after clearing the harmonic truncation")


def test_poisson_identities_on_device():
    one = lambda x, j, t, c: (np.array([[x]], np.int32), np.array([j], np.int32),
                              np.array([t], np.uint8), np.array([c], np.float64))
    cy, sy = one(0, [1, 0], 0, 1.0), one(0, [1, 0], 1, 1.0)
    gx, gy, gt, gc, _ = gpu_poisson(cy, cy)
    got = {(tuple(y), int(t)): c for y, t, c in zip(gy.tolist(), gt, gc)}
    assert got == {((0, 0), 0): 0.5, ((2, 0), 0): 0.5}
    gx, gy, gt, gc, _ = gpu_poisson(sy, sy)
    got = {(tuple(y), int(t)): c for y, t, c in zip(gy.tolist(), gt, gc)}
    assert got == {((0, 0), 0): 0.5, ((2, 0), 0): -0.5}
    gx, gy, gt, gc, _ = gpu_poisson(sy, cy)                    # sin 0 dropped
    got = {(tuple(y), int(t)): c for y, t, c in zip(gy.tolist(), gt, gc)}
    assert got == {((2, 0), 1): 0.5}
    c1, s2 = one(0, [1, 0], 0, 1.0), one(0, [0, 1], 1, 1.0)
    gx, gy, gt, gc, _ = gpu_poisson(s2, c1)
    got = {(tuple(y), int(t)): c for y, t, c in zip(gy.tolist(), gt, gc)}
    assert got == {((1, 1), 1): 0.5, ((1, -1), 1): -0.5}


@pytest.mark.parametrize("mode", ["dense", "hash"])
def test_poisson_identities_both_modes(mode):
    one = lambda x, j, t, c: (np.array([[x]], np.int32), np.array([j], np.int32),
                              np.array([t], np.uint8), np.array([c], np.float64))
    cy, sy = one(0, [1, 0], 0, 1.0), one(0, [1, 0], 1, 1.0)
    c1, s2 = one(1, [1, 0], 0, 2.0), one(-1, [0, 1], 1, 1.0)
    for a, b, want in ((cy, cy, {((0, 0), 0): 0.5, ((2, 0), 0): 0.5}),
                       (sy, sy, {((0, 0), 0): 0.5, ((2, 0), 0): -0.5}),
                       (sy, cy, {((2, 0), 1): 0.5}),
                       (cy, sy, {((2, 0), 1): 0.5}),
                       (s2, c1, {((1, 1), 1): 1.0, ((1, -1), 1): -1.0})):
        gx, gy, gt, gc, _ = gpu_poisson(a, b, mode)
        got = {(tuple(y), int(t)): c for y, t, c in zip(gy.tolist(), gt, gc)}
        assert got == want, (mode, got)


@pytest.mark.parametrize("jmax", [2, 5])
def test_poisson_dense_matches_oracle_and_hash(jmax):
    """Dense-mode Poisson products (segmented codes, fold to canonical keys)
    against the oracle and against hash mode."""
    a = I.poisson_random(nx=2, ny=2, n=700, xlo=-3, xhi=3, jmax=jmax, cfg=92, factor=0)
    b = I.poisson_random(nx=2, ny=2, n=650, xlo=-2, xhi=4, jmax=jmax, cfg=92, factor=1)
    dx, dy, dt, dc = check_poisson(a, b, f"Poisson dense jmax {jmax}", 2, 2, mode="dense")
    hx, hy, ht, hc = check_poisson(a, b, f"Poisson hash jmax {jmax}", 2, 2, mode="hash")
    assert len(dc) == len(hc)
    ex = np.concatenate([dx, dy, dt.reshape(-1, 1).astype(np.int32)], 1)
    eh = np.concatenate([hx, hy, ht.reshape(-1, 1).astype(np.int32)], 1)
    od, oh = np.lexsort(ex.T[::-1]), np.lexsort(eh.T[::-1])
    assert np.array_equal(ex[od], eh[oh])


def test_poisson_400():
    a, b = I.config(4, scale=0.08)
    check_poisson(a, b, "Poisson 3+6 vars, 400 x 400")


def test_poisson_exact_fp2_and_tiny():
    nx, ny = 2, 3
    a = I.poisson_random(nx=nx, ny=ny, n=300, xlo=-2, xhi=2, jmax=3, coef="f64int", cfg=91,
                         factor=0)
    b = I.poisson_random(nx=nx, ny=ny, n=257, xlo=-1, xhi=3, jmax=2, coef="f64int", cfg=91,
                         factor=1)
    gx, gy, gt, gc = check_poisson(a, b, "Poisson integer coefficients", nx, ny)
    P = O.P61
    rng = np.random.default_rng(1)
    xp = [int(v) for v in rng.integers(2, P - 1, nx)]
    zp = [tuple(int(v) for v in rng.integers(1, P - 1, 2)) for _ in range(ny)]
    lhs = O.poisson_eval_fp2((gx, gy, gt, gc), nx, ny, xp, zp)
    rhs = O.fp2_mul(O.poisson_eval_fp2(a, nx, ny, xp, zp), O.poisson_eval_fp2(b, nx, ny, xp, zp))
    assert lhs == rhs
    check_poisson(a, (b[0][:1], b[1][:1], b[2][:1], b[3][:1]), "Poisson n x 1", nx, ny)


# ------------------------------------------------------------------ full sizes
def test_full_moderately_sparse_10000():
    """The 4-variable simplex product at full size (1e8 pairs), dense mode,
    bit-exact against the oracle's full product."""
    a, b = I.config(2)
    ge, gc, lay = check_laurent(a, b, "auto", "4-var simplex, 10000 x 10000 (full)")
    assert len(gc) > 130000


def _key6(ex, base=161):
    """One int64 per exponent row (entries in [0, base))."""
    k = ex[:, 0].to(_torch().int64) if hasattr(ex, "to") else ex[:, 0].astype(np.int64)
    for v in range(1, ex.shape[1]):
        col = ex[:, v].to(_torch().int64) if hasattr(ex, "to") else ex[:, v].astype(np.int64)
        k = k * base + col
    return k


def test_full_highly_sparse_all_terms():
    """The 6-variable sparse product at full size (9e8 pairs), hash mode, as a
    whole product from exponents.  Every term is checked: keys unique and in
    the product box, coefficients nonzero, and the value of the whole result
    at 3 random points modulo 2^61-1 and 2 random odd points modulo 2^64
    equals A(r) B(r) (Schwartz-Zippel: a misplaced, missing or wrong term
    changes the value except with probability about 1e-16 per point).  Then
    10^4 sampled terms equal the oracle's one-by-one coefficients, and 10^4
    exponent tuples absent from the result (half uniform in the box, half
    next to result terms) have oracle coefficient 0."""
    torch = _torch()
    a, b = I.config(3)
    say("6 vars [0,80], 30000 x 30000 (full, every term)")
    pa = kp.Poly(dev(a[0]), dev(a[1]))
    pb = kp.Poly(dev(b[0]), dev(b[1]))
    r, lay = kp.mul_laurent(pa, pb)
    ex, co = r.exps, r.coef
    n = co.shape[0]
    assert 8.9e8 < n <= 9e8
    assert int(ex.min()) >= 0 and int(ex.max()) <= 160
    assert bool((co != 0).all())
    key = _key6(ex)
    assert int(torch.unique(key).shape[0]) == n
    rng = np.random.default_rng(2010)
    for _ in range(3):
        pt = [int(x) for x in rng.integers(2, P61, 6)]
        want = O.laurent_eval_modp(a[0], a[1], pt) * O.laurent_eval_modp(b[0], b[1], pt) % P61
        assert eval_modp_device(ex, co, pt) == want
    for _ in range(2):
        pt = [int(x) | 1 for x in rng.integers(3, 2**62, 6)]
        want = _eval_mod2_64(a[0], a[1], pt) * _eval_mod2_64(b[0], b[1], pt) % 2**64
        assert eval_mod2_64_device(ex, co, pt) == want
    # 10^4 sampled terms against the oracle, one by one
    sel = torch.from_numpy(rng.choice(n, 10000, replace=False)).cuda()
    qe, qc = ex[sel].cpu().numpy(), co[sel].cpu().numpy()
    got = parallel_chunks(lambda q: O.laurent_coeff_at(a[0], a[1], b[0], b[1], q)[0], [qe])
    np.testing.assert_array_equal(np.concatenate(got), qc)
    # 10^4 absent tuples: uniform in the box, and next to sampled result terms
    uni = rng.integers(0, 161, (20000, 6)).astype(np.int32)
    near = qe.copy()
    near[np.arange(len(near)), rng.integers(0, 6, len(near))] += rng.choice([-1, 1], len(near)).astype(np.int32)
    near = np.clip(near, 0, 160)
    absent = []
    for cand in (uni, near):
        present = torch.isin(_key6(dev(cand)), key).cpu().numpy()
        absent.append(cand[~present][:5000])
    assert len(absent[0]) == 5000 and len(absent[1]) == 5000
    q = np.concatenate(absent)
    got = parallel_chunks(lambda q: O.laurent_coeff_at(a[0], a[1], b[0], b[1], q)[0], [q])
    assert (np.concatenate(got) == 0).all()


def _poisson_keys(x, y, t):
    """One int64 per Poisson term of the 5000 x 5000 product (x in [-8,8]^3,
    multipliers in [-16,16]^6)."""
    k = np.zeros(len(t), dtype=np.int64)
    for v in range(x.shape[1]):
        k = k * 17 + (x[:, v].astype(np.int64) + 8)
    for v in range(y.shape[1]):
        k = k * 33 + (y[:, v].astype(np.int64) + 16)
    return k * 2 + t.astype(np.int64)


def _canonical(y, t):
    """Canonical form of multiplier rows: negate a row whose first nonzero
    entry is negative; the zero row is taken as a cosine."""
    nz = y != 0
    first = np.where(nz.any(1), y[np.arange(len(y)), np.argmax(nz, axis=1)], 0)
    y = np.where((first < 0)[:, None], -y, y)
    t = np.where(nz.any(1), t, 0).astype(np.uint8)
    return y, t


def _check_poisson_keys(gx, gy, gt):
    n = len(gt)
    key = _poisson_keys(gx, gy, gt)
    assert len(np.unique(key)) == n
    nz = np.argmax(gy != 0, axis=1)
    first = gy[np.arange(n), nz]
    assert ((first > 0) | ((gy == 0).all(1) & (gt == 0))).all()
    return key


def test_full_poisson_every_term_exact():
    """The Poisson product at full size (2.5e7 pairs, 5e7 pieces) with the
    configuration's exponents and integer coefficients, so that every half
    product and every sum is exact in fp64: the value of all result terms
    over F_{p^2} (p = 2^61-1; cos and sin of j.y mapped through Z_k for
    exp(i y_k)) equals the product of the factors' values, at 2 random
    points.  Keys unique and canonical."""
    a, b = I.config(4)
    rng = np.random.default_rng(44)
    ai = (*a[:3], (rng.integers(1, 1000, len(a[3])) * rng.choice([-1, 1], len(a[3]))).astype(np.float64))
    bi = (*b[:3], (rng.integers(1, 1000, len(b[3])) * rng.choice([-1, 1], len(b[3]))).astype(np.float64))
    say("Poisson 3+6 vars, 5000 x 5000 (full), integer coefficients, every term")
    gx, gy, gt, gc, lay = gpu_poisson(ai, bi)
    n = len(gc)
    assert 4.9e7 < n <= 5e7
    _check_poisson_keys(gx, gy, gt)
    assert (gc * 2 == np.round(gc * 2)).all()
    for _ in range(2):
        xp = [int(v) for v in rng.integers(2, P61, 3)]
        zp = [(int(u), int(v)) for u, v in rng.integers(2, P61, (6, 2))]
        want = O.fp2_mul(O.poisson_eval_fp2(ai, 3, 6, xp, zp), O.poisson_eval_fp2(bi, 3, 6, xp, zp))
        parts = parallel_chunks(lambda x, y, t, c: O.poisson_eval_fp2((x, y, t, c), 3, 6, xp, zp),
                                [gx, gy, gt, gc])
        got = (sum(p[0] for p in parts) % P61, sum(p[1] for p in parts) % P61)
        assert got == want


def test_full_poisson_sampled_and_absent():
    """The Poisson product at full size (2.5e7 pairs), N(0,1) 2^-sum|j|
    coefficients, hash mode: keys unique and canonical, numeric evaluation at
    random angles, 10^4 sampled terms equal the oracle's one-by-one
    coefficients within 1e-13 sum|contributions|, and 10^4 canonical keys
    absent from the result (half next to result terms, half uniform in the
    product box) have no oracle contribution beyond that tolerance."""
    a, b = I.config(4)
    say("Poisson 3+6 vars, 5000 x 5000 (full), sampled and absent keys")
    gx, gy, gt, gc, lay = gpu_poisson(a, b)
    n = len(gc)
    assert 4.9e7 < n <= 5e7
    key = _check_poisson_keys(gx, gy, gt)
    rng = np.random.default_rng(5)
    for _ in range(2):
        xs = rng.uniform(0.8, 1.2, 3)
        ys = rng.uniform(-np.pi, np.pi, 6)
        def ev(x, y, t, c):
            xv = np.prod(xs[None, :] ** x, axis=1)
            ang = y @ ys
            tr = np.where(t.astype(bool), np.sin(ang), np.cos(ang))
            terms = c * xv * tr
            return terms.sum(), np.abs(terms).sum()
        va, sa = ev(*a)
        vb, sb = ev(*b)
        vp, sp = ev(gx, gy, gt, gc)
        assert abs(vp - va * vb) <= 1e-11 * sa * sb
    sel = rng.choice(n, 10000, replace=False)
    res = parallel_chunks(lambda x, y, t: O.poisson_coeff_at(a, b, 3, 6, x, y, t)[:2],
                          [gx[sel], gy[sel], gt[sel]])
    want = np.concatenate([r[0] for r in res])
    wab = np.concatenate([r[1] for r in res])
    assert np.all(np.abs(gc[sel] - want) <= TOL * wab)
    # absent canonical keys
    ny_ = gy[sel].copy()
    ny_[np.arange(len(sel)), rng.integers(0, 6, len(sel))] += rng.choice([-1, 1], len(sel)).astype(np.int32)
    ny_ = np.clip(ny_, -16, 16)
    ny_, nt_ = _canonical(ny_, gt[sel])
    near = (gx[sel], ny_, nt_)
    ux = rng.integers(-8, 9, (20000, 3)).astype(np.int32)
    uy, ut = _canonical(rng.integers(-16, 17, (20000, 6)).astype(np.int32),
                        rng.integers(0, 2, 20000).astype(np.uint8))
    qs = []
    for cx, cy, ct in (near, (ux, uy, ut)):
        keep = ~np.isin(_poisson_keys(cx, cy, ct), key)
        qs.append((cx[keep][:5000], cy[keep][:5000], ct[keep][:5000]))
    assert all(len(q[2]) == 5000 for q in qs)
    qx, qy, qt = (np.concatenate([q[i] for q in qs]) for i in range(3))
    res = parallel_chunks(lambda x, y, t: O.poisson_coeff_at(a, b, 3, 6, x, y, t)[:2], [qx, qy, qt])
    want = np.concatenate([r[0] for r in res])
    wab = np.concatenate([r[1] for r in res])
    assert np.all(np.abs(want) <= TOL * wab)


# ------------------------------------------------------------------ the paper's benchmarks
def _fateman_closed_form(exps, k):
    """Coefficients of f * (f + 1) = f^2 + f for f = (1 + x + y + z + t)^k, by
    the multinomial theorem, modulo 2^64 as signed int64."""
    fact = [math.factorial(i) for i in range(2 * k + 1)]
    out = np.empty(len(exps), dtype=np.int64)
    for i, p in enumerate(exps.tolist()):
        s = sum(p)
        c = fact[2 * k] // (fact[2 * k - s] * fact[p[0]] * fact[p[1]] * fact[p[2]] * fact[p[3]])
        if s <= k:
            c += fact[k] // (fact[k - s] * fact[p[0]] * fact[p[1]] * fact[p[2]] * fact[p[3]])
        c %= 2**64
        out[i] = c - 2**64 if c >= 2**63 else c
    return out


def test_fateman_benchmark_closed_form():
    """Fateman's benchmark (Section 5): f = (1+x+y+z+t)^30 times f + 1, 46376 x
    46376 terms, dense mode; every one of the C(64,4) result terms equals the
    closed form modulo 2^64 (the coefficients exceed 2^63)."""
    f = I.fateman(30)
    g = I.fateman(30, plus_one=True)
    say("Fateman k=30", len(f[1]), "x", len(g[1]))
    ge, gc, lay = gpu_laurent(f, g, "auto")
    assert len(gc) == math.comb(64, 4)
    assert len(np.unique(ge, axis=0)) == len(gc)
    assert ge.min() >= 0 and ge.sum(1).max() == 60
    np.testing.assert_array_equal(gc, _fateman_closed_form(ge, 30))


def _eval_mod2_64(exps, coef, pt):
    """sum_t c_t prod_k pt_k^e_tk in the ring of integers modulo 2^64 (numpy
    uint64 arithmetic wraps), for non-negative exponents."""
    acc = np.asarray(coef).astype(np.uint64)
    with np.errstate(over="ignore"):
        for v, x in enumerate(pt):
            top = int(exps[:, v].max())
            pw = np.ones(top + 1, dtype=np.uint64)
            for i in range(1, top + 1):
                pw[i] = pw[i - 1] * np.uint64(x)
            acc = acc * pw[exps[:, v]]
        return int(acc.sum(dtype=np.uint64))


def test_mp_sparse_benchmark():
    """Monagan-Pearce's sparse benchmark (Section 5): f = (1+x+y+2z^2+3t^3+5u^5)^12
    times g (variables reversed), 6188 x 6188 terms, hash mode: 5,821,335 terms.
    The coefficients outgrow int64, so the product is the one modulo 2^64: its
    value at random odd points modulo 2^64 equals f(pt) g(pt) from the closed
    form, and sampled terms equal the oracle's (which also wraps)."""
    f = I.mp_sparse(12, "f")
    g = I.mp_sparse(12, "g")
    say("MP-sparse k=12", len(f[1]), "x", len(g[1]))
    ge, gc, lay = gpu_laurent(f, g, "auto")
    assert len(gc) == 5821335
    M = 2**64
    rng = np.random.default_rng(12)
    for _ in range(3):
        pt = [int(v) | 1 for v in rng.integers(3, 2**62, 5)]
        x, y, z, t, u = pt
        fb = (1 + x + y + 2 * z**2 + 3 * t**3 + 5 * u**5) % M
        gb = (1 + u + t + 2 * z**2 + 3 * y**3 + 5 * x**5) % M
        want = pow(fb, 12, M) * pow(gb, 12, M) % M
        assert _eval_mod2_64(ge, gc, pt) == want
    sel = rng.integers(0, len(gc), 200)
    w, _, _ = O.laurent_coeff_at(f[0], f[1], g[0], g[1], ge[sel])
    np.testing.assert_array_equal(gc[sel], w)


# ------------------------------------------------------------------ truncation
def _trunc_cases():
    out = []
    a, b = I.config(2, scale=0.2)
    out.append(("simplex, total degree <= 20", a, b, [1, 1, 1, 1], 20))
    out.append(("simplex fp64, degree in x0, x2 <= 9",
                (a[0], a[1].astype(np.float64) / 8), (b[0], b[1].astype(np.float64)),
                [1, 0, 1, 0], 9))
    a, b = I.config(1, scale=0.6)
    out.append(("box, weights (2, -1, 1) <= 3", a, b, [2, -1, 1], 3))
    a, b = I.config(3, scale=0.04)
    out.append(("sparse, total degree <= 240", a, b, [1] * 6, 240))
    return out


@pytest.mark.parametrize("mode,part,grouping", [("dense", 0, 0), ("hash", 0, 0), ("hash", 2, 0),
                                                ("hash", 2, 1), ("hash", 2, 2)])
def test_truncated_products_match_oracle(mode, part, grouping):
    ctx = kp.context()
    ctx.set_tune(hash_partitioned=part, hash_grouping=grouping)
    for what, a, b, w, D in _trunc_cases():
        if mode == "dense" and "sparse" in what:
            continue
        say("truncated", what, mode, part)
        with ctx.truncation(w, D):
            ge, gc, _ = gpu_laurent(a, b, mode, ctx)
        oe, oc, oab = O.laurent_mul_truncated(a[0], a[1], b[0], b[1], w, D, threads=4)
        assert len(oc) > 0
        if np.asarray(a[1]).dtype == np.float64:
            assert_tolerance([ge], gc, [oe], oc, oab, TOL, what)
        else:
            assert_exact([ge], gc, [oe], oc, what)


@pytest.mark.parametrize("part", [0, 2, 3])
def test_truncation_keeps_few_or_no_pairs(part):
    """A degree limit below every pair's degree gives the empty product; one a
    little above the smallest keeps a handful of pairs (the grouped layout
    then chooses its fewest level-2 bins).  Against the oracle's filter.
    part 3: grouped by code range."""
    ctx = kp.context()
    ctx.set_tune(hash_partitioned=min(part, 2), hash_grouping=2 if part == 3 else 0)
    a, b = I.config(3, scale=0.03)
    da, db = a[0].sum(1).min(), b[0].sum(1).min()
    for D, what in ((int(da + db) - 1, "no pair kept"), (int(da + db) + 25, "a few pairs kept")):
        say("truncated sparse,", what, "partitioned", part)
        with ctx.truncation([1] * 6, D):
            ge, gc, _ = gpu_laurent(a, b, "hash", ctx)
        oe, oc, _ = O.laurent_mul_truncated(a[0], a[1], b[0], b[1], [1] * 6, D, threads=4)
        if what == "no pair kept":
            assert len(oc) == 0 and len(gc) == 0
        else:
            assert 0 < len(oc) < 1000
        assert_exact([ge], gc, [oe], oc, what)


def test_truncation_codes_path_and_errors():
    torch = _torch()
    ctx = kp.context()
    a, b = I.config(1, scale=0.4)
    lay = kp.layout_product(3, 0, a[0].min(0), a[0].max(0), b[0].min(0), b[0].max(0))
    ka, _ = kp.encode(lay, 0, dev(a[0]))
    kb, _ = kp.encode(lay, 1, dev(b[0]))
    say("truncated codes path")
    with ctx.truncation([1, 1, 1], 0):
        codes, coef, _ = kp.mul_laurent_codes(lay, ka, dev(a[1]), kb, dev(b[1]), "dense")
        ex = kp.decode(lay, codes).cpu().numpy()
    oe, oc, _ = O.laurent_mul_truncated(a[0], a[1], b[0], b[1], [1, 1, 1], 0)
    assert_exact([ex], coef.cpu().numpy(), [oe], oc, "codes path, degree <= 0")
    # a factor degree past 2^30 is reported, not silently wrong
    big = (np.array([[40000], [1]], np.int32), np.array([1, 2], np.int64))
    pa, pb = kp.Poly(dev(big[0]), dev(big[1])), kp.Poly(dev(big[0]), dev(big[1]))
    with ctx.truncation([1 << 15], 10):
        with pytest.raises(kp.KPError) as e:
            kp.mul_laurent(pa, pb, ctx=ctx)
    assert e.value.status == kp.KP_E_RANGE
    ctx.sync_check()
    # Poisson products do not take a degree truncation
    p4a, p4b = I.config(4, scale=0.01)
    with ctx.truncation([1, 1, 1], 5):
        with pytest.raises(kp.KPError) as e:
            gpu_poisson(p4a, p4b)
    assert e.value.status == kp.KP_E_ARG
    # cleared: the full product again
    r, _ = kp.mul_laurent(kp.Poly(dev(a[0]), dev(a[1])), kp.Poly(dev(b[0]), dev(b[1])), ctx=ctx)
    assert r.coef.shape[0] == len(O.laurent_mul(a[0], a[1], b[0], b[1])[1])
