"""CPU tests of the C ABI's host side: exports, layout, codec and planning.

The Kronecker codec is pinned by the codes printed in the paper (Tables 1 and
2, eq. c_01 of Section 2, fixtures under tests/golden/), by exhaustive round
trips and by the homomorphism property; the Poisson coding by the sign
property of balanced digits.  No GPU is needed: these calls never launch.
"""
import ctypes as C
import itertools
import os
import re

import numpy as np
import pytest

import paper_1004_4548_amd as kp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [l.split() for l in f if l.strip() and not l.startswith("#")]


def test_library_exports_every_declared_symbol():
    text = open(os.path.join(ROOT, "include", "kp.h")).read()
    declared = set(re.findall(r"\b(kp_[a-z_0-9]+)\s*\(", text))
    assert declared == set(kp.EXPORTED)
    lib = C.CDLL(kp.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def test_status_strings():
    for s in range(10):
        assert kp.status_str(s)


def _layout_laurent(amin, amax, bmin=None, bmax=None):
    nv = len(amin)
    bmin = [0] * nv if bmin is None else bmin
    bmax = [0] * nv if bmax is None else bmax
    return kp.layout_product(nv, 0, amin, amax, bmin, bmax)


def test_table1_codes():
    # factor A spans the table's box, factor B is the constant 1: the product
    # box is the table's box and A's codes are the printed ones
    lay = _layout_laurent([0, 0, 0], [3, 3, 3])
    assert list(lay.xc[:3]) == [1, 4, 16] and lay.nkeys == 64
    for z, y, x, code in _rows("table1_codes.txt"):
        kx, _ = kp.encode_host(lay, 0, [[int(x), int(y), int(z)]])
        assert kx[0] == int(code)
        assert kp.decode_host(lay, [int(code)]).tolist() == [[int(x), int(y), int(z)]]


def test_eq_c01_homomorphism():
    lay = _layout_laurent([0, 0, 0], [3, 3, 3])
    for r in _rows("eq_c01.txt"):
        z1, y1, x1, z2, y2, x2, want = map(int, r)
        c1, _ = kp.encode_host(lay, 0, [[x1, y1, z1]])
        c2, _ = kp.encode_host(lay, 0, [[x2, y2, z2]])
        c12, _ = kp.encode_host(lay, 0, [[x1 + x2, y1 + y2, z1 + z2]])
        assert c1[0] + c2[0] == want == c12[0]


@pytest.mark.parametrize("emin,emax", [((-2, -5, 3), (4, 1, 7)), ((0, 0, 0), (9, 2, 1)),
                                       ((-7, 3, -1), (-3, 8, 0))])
def test_table2_generalised_codes(emin, emax):
    lay = _layout_laurent(list(emin), list(emax))
    w0 = 1 + emax[0] - emin[0]
    assert list(lay.xc[:3]) == [1, w0, w0 * (1 + emax[1] - emin[1])]
    for d1, x0, code in _rows("table2_rows.txt"):
        base, off = x0[:3], int(x0[4:])
        e0 = emin[0] + off if base == "min" else emax[0] - off
        e = [e0, emin[1] + int(d1), emin[2]]
        want = eval(code, {"w0": w0})          # the fixture's printed expression
        kx, _ = kp.encode_host(lay, 0, [e])
        assert kx[0] == want
        # c(e) = c . e - chi with chi = c . e_min
        chi = sum(int(lay.xc[v]) * emin[v] for v in range(3))
        assert kx[0] == sum(int(lay.xc[v]) * e[v] for v in range(3)) - chi


def test_product_codes_add():
    rng = np.random.default_rng(1)
    amin, amax, bmin, bmax = [-3, 0, 2], [2, 4, 5], [-1, -6, 0], [3, 1, 0]
    lay = kp.layout_product(3, 0, amin, amax, bmin, bmax)
    ea = np.stack([rng.integers(amin[v], amax[v] + 1, 200) for v in range(3)], 1)
    eb = np.stack([rng.integers(bmin[v], bmax[v] + 1, 200) for v in range(3)], 1)
    ka, _ = kp.encode_host(lay, 0, ea)
    kb, _ = kp.encode_host(lay, 1, eb)
    np.testing.assert_array_equal(kp.decode_host(lay, ka + kb), ea + eb)
    assert ((ka + kb) >= 0).all() and ((ka + kb) < lay.nkeys).all()


def test_exhaustive_round_trip():
    lay = kp.layout_product(3, 0, [-2, 0, -1], [1, 3, 0], [0, -2, 0], [2, 0, 2])
    codes = np.arange(lay.nkeys)
    ex = kp.decode_host(lay, codes)
    assert len({tuple(r) for r in ex.tolist()}) == lay.nkeys
    lo = np.array([lay.xmin[v] for v in range(3)])
    w = np.array([lay.xw[v] for v in range(3)])
    assert ((ex >= lo) & (ex < lo + w)).all()
    # re-encode against the product box itself (factor A = product box, B = 0)
    lay2 = _layout_laurent(list(lo), list(lo + w - 1))
    kx, _ = kp.encode_host(lay2, 0, ex)
    np.testing.assert_array_equal(kx, codes)


def test_large_widths_decode():
    # widths near 2^31 exercise the invariant-divisor division
    lay = kp.layout_product(2, 0, [-(2**30), 0], [2**30 - 1, 2**20], [0, -5], [2**29, 2**20])
    rng = np.random.default_rng(2)
    codes = rng.integers(0, lay.nkeys, size=20000, dtype=np.int64)
    codes[:3] = [0, lay.nkeys - 1, lay.xw[0] - 1]
    ex = kp.decode_host(lay, codes)
    back = sum((ex[:, v].astype(object) - int(lay.xmin[v])) * int(lay.xc[v]) for v in range(2))
    assert [int(b) for b in back] == codes.tolist()


def test_code_overflow_boundary():
    # 2^31 * 2^31 = 2^62 codes is rejected; 2^31 * (2^31 - 1) is accepted
    with pytest.raises(kp.KPError) as e:
        kp.layout_product(2, 0, [0, 0], [2**31 - 1, 2**31 - 1], [0, 0], [0, 0])
    assert e.value.status == kp.KP_E_CODE_OVERFLOW
    lay = kp.layout_product(2, 0, [0, 0], [2**31 - 1, 2**31 - 2], [0, 0], [0, 0])
    assert lay.nkeys == 2**31 * (2**31 - 1)


def test_range_check():
    lay = _layout_laurent([0, 0], [3, 3])
    with pytest.raises(kp.KPError) as e:
        kp.encode_host(lay, 0, [[4, 0]])
    assert e.value.status == kp.KP_E_RANGE
    with pytest.raises(kp.KPError):
        kp.decode_host(lay, [lay.nkeys])


def test_empty_factor_layout():
    lay = kp.layout_product(2, 0, [0, -1], [-1, 1], [0, 0], [3, 3])
    assert lay.nkeys == 0


# ---------------------------------------------------------------- Poisson codes
def test_balanced_trig_codes_sign_property():
    # every multiplier vector of a small balanced box: sign(ky) is the sign of
    # the first nonzero multiplier, and ky(a) +- ky(b) = ky(a +- b)
    ha, hb = [1, 2, 1], [1, 0, 2]
    lay = kp.layout_product(1, 3, [0], [0], [0], [0], ha, hb)
    box = [range(-(a + b), a + b + 1) for a, b in zip(ha, hb)]
    js = np.array(list(itertools.product(*box)), dtype=np.int32)
    n = len(js)
    ky = np.array([sum(int(lay.yc[v]) * int(j[v]) for v in range(3)) for j in js])
    for j, k in zip(js, ky):
        nz = np.flatnonzero(j)
        assert np.sign(k) == (0 if len(nz) == 0 else np.sign(j[nz[0]]))
    assert len(set(ky.tolist())) == n and ky.max() == lay.Hy
    # canonical decode of |ky| returns the canonical multiplier vector
    Wx = lay.Wx
    for j, k in zip(js, ky):
        if k < 0:
            continue
        x, y, t = kp.decode_host(lay, [2 * (Wx * k) + 0], poisson=True)
        assert y[0].tolist() == j.tolist()


def test_poisson_encode_checks_canonical_form():
    lay = kp.layout_product(1, 2, [0], [2], [0], [2], [3, 3], [3, 3])
    kx, ky = kp.encode_host(lay, 0, [[1]], [[2, -3]], [1])
    assert ky[0] > 0
    for y, t in (([-1, 2], 0), ([0, -1], 1), ([0, 0], 1)):
        with pytest.raises(kp.KPError) as e:
            kp.encode_host(lay, 0, [[1]], [y], [t])
        assert e.value.status == kp.KP_E_NONCANONICAL
    kx, ky = kp.encode_host(lay, 0, [[1]], [[0, 0]], [0])       # cos(0) is canonical
    assert ky[0] == 0


def test_poisson_key_space():
    lay = kp.layout_product(3, 6, [-4] * 3, [4] * 3, [-4] * 3, [4] * 3, [8] * 6, [8] * 6)
    assert lay.Wx == 17**3 and lay.Hy == (33**6 - 1) // 2
    assert lay.nkeys == 2 * lay.Wx * (lay.Hy + 1)


# ---------------------------------------------------------------- planning
def _host_ctx():
    return kp.Context(-1)


def test_mode_selection_for_the_workloads():
    ctx = _host_ctx()
    l1 = kp.layout_product(3, 0, [-5] * 3, [5] * 3, [-5] * 3, [5] * 3)
    assert kp.mul_bound(l1, False, kp.KP_I64, "auto", 500, 500, ctx)[0] == "dense"
    l2 = kp.layout_product(4, 0, [0] * 4, [20] * 4, [0] * 4, [20] * 4)
    m, mo, ws = kp.mul_bound(l2, False, kp.KP_I64, "auto", 10000, 10000, ctx)
    assert m == "dense" and mo == 41**4
    l3 = kp.layout_product(6, 0, [0] * 6, [80] * 6, [0] * 6, [80] * 6)
    m, mo, ws = kp.mul_bound(l3, False, kp.KP_I64, "auto", 30000, 30000, ctx)
    assert m == "hash" and mo == 9 * 10**8
    l4 = kp.layout_product(3, 6, [-4] * 3, [4] * 3, [-4] * 3, [4] * 3, [8] * 6, [8] * 6)
    m, mo, ws = kp.mul_bound(l4, True, kp.KP_F64, "auto", 5000, 5000, ctx)
    assert m == "hash" and mo == 5 * 10**7
    with pytest.raises(kp.KPError) as e:   # eight segments of 6.3e12 codes: no dense mode
        kp.mul_bound(l4, True, kp.KP_F64, "dense", 5000, 5000, ctx)
    assert e.value.status == kp.KP_E_MODE
    # a small Poisson key space: dense (two trig variables, multipliers up to 5)
    l5 = kp.layout_product(2, 2, [-3] * 2, [3] * 2, [-2] * 2, [4] * 2, [5] * 2, [5] * 2)
    m, mo, ws = kp.mul_bound(l5, True, kp.KP_F64, "auto", 700, 650, ctx)
    assert m == "dense" and mo == min(2 * 700 * 650, l5.nkeys)


def test_planning_errors():
    ctx = _host_ctx()
    l3 = kp.layout_product(6, 0, [0] * 6, [80] * 6, [0] * 6, [80] * 6)
    with pytest.raises(kp.KPError) as e:
        kp.mul_bound(l3, False, kp.KP_I64, "dense", 30000, 30000, ctx)
    assert e.value.status == kp.KP_E_MODE
    l4 = kp.layout_product(1, 1, [0], [1], [0], [1], [1], [1])
    with pytest.raises(kp.KPError) as e:
        kp.mul_bound(l4, True, kp.KP_I64, "auto", 5, 5, ctx)
    assert e.value.status == kp.KP_E_DTYPE


def test_tune_validation():
    ctx = _host_ctx()
    t = ctx.tune
    assert t.window == 18432 and t.block == 1024 and t.tasks_per_cu == 1
    ctx.set_tune(window=2048, block=512)
    assert ctx.tune.window == 2048
    assert t.hash_partitioned == 1
    for bad in (dict(window=18432 + 2048), dict(block=100), dict(hash_load=0.95),
                dict(window=1000, block=256), dict(dense_max_keys=(1 << 27) + 1),
                dict(hash_partitioned=3), dict(hash_partitioned=-1), dict(hash_bucket=-1),
                dict(hash_bucket=17), dict(hash_order=2), dict(hash_bin_slots=0),
                dict(hash_bin_slots=3000), dict(hash_bin_slots=16384), dict(hash_grouping=3),
                dict(hash_max_bin_bits=11), dict(hash_max_bin_bits=-1), dict(hash_bin_fill=9),
                dict(hash_bin_fill=91)):
        with pytest.raises(kp.KPError):
            ctx.set_tune(**bad)
    assert t.hash_bucket == 0 and t.hash_order == 1 and t.hash_bin_slots == 4096
    assert t.hash_bin_fill == 42
    for slots in (2048, 4096, 8192):
        ctx.set_tune(hash_bin_slots=slots)
        assert ctx.tune.hash_bin_slots == slots


def test_partitioned_hash_workspace():
    """Grouped by code range (the default for Laurent int64/fp64), hash mode
    keeps every product once (at most 16 bytes) plus small per-range and
    per-bin arrays; grouped by two levels of hash bits, twice (16 bytes each)
    plus a 2-byte bin id; the global table two 16-byte slots per bounded
    result term.  Auto takes a grouped layout only when the products are at
    most 4x the bound."""
    ctx = _host_ctx()
    sparse = kp.layout_product(6, 0, [0] * 6, [80] * 6, [0] * 6, [80] * 6)
    box = kp.layout_product(3, 0, [-5] * 3, [5] * 3, [-5] * 3, [5] * 3)
    na = nb = 3000
    _, mo, ws_auto = kp.mul_bound(sparse, False, kp.KP_I64, "hash", na, nb, ctx)
    assert mo == na * nb and 16 * na * nb <= ws_auto < 17 * na * nb
    ctx.set_tune(hash_grouping=1)
    _, _, ws_two = kp.mul_bound(sparse, False, kp.KP_I64, "hash", na, nb, ctx)
    assert ws_two >= 34 * na * nb
    ctx.set_tune(hash_grouping=0)
    ctx.set_tune(hash_partitioned=0)
    _, _, ws_table = kp.mul_bound(sparse, False, kp.KP_I64, "hash", na, nb, ctx)
    assert 32 * na * nb <= ws_table < 33 * na * nb
    _, mo_box, ws_box_table = kp.mul_bound(box, False, kp.KP_I64, "hash", 500, 500, ctx)
    ctx.set_tune(hash_partitioned=1)
    assert kp.mul_bound(box, False, kp.KP_I64, "hash", 500, 500, ctx)[2] == ws_box_table
    ctx.set_tune(hash_partitioned=2)
    _, _, ws_box_part = kp.mul_bound(box, False, kp.KP_I64, "hash", 500, 500, ctx)
    assert mo_box == 21 ** 3 and ws_box_part >= 16 * 500 * 500 > ws_box_table


def test_bucketed_hash_workspace():
    """The bucketed table: ceil(cap / m) buckets of m 16-byte slots and an
    overflow table of six times N E[(X - m)+] slots, X Poisson with the
    bound's codes per bucket as mean (at least 1024); with the term order
    both factors again (16 bytes a term) plus 4 bytes of rank scratch.  It is
    not used for 128-bit sums."""
    from scipy.stats import poisson
    ctx = _host_ctx()
    sparse = kp.layout_product(6, 0, [0] * 6, [80] * 6, [0] * 6, [80] * 6)
    na, nb = 3000, 2000
    ctx.set_tune(hash_partitioned=0)
    _, mo, ws_table = kp.mul_bound(sparse, False, kp.KP_I64, "hash", na, nb, ctx)
    cap = int(mo / 0.5) + 1
    for m in (1, 3, 8, 16):
        nbk = -(-cap // m)
        lam = mo / nbk
        k = np.arange(0, m + 200)
        excess = float(np.sum(np.maximum(k - m, 0) * poisson.pmf(k, lam)))
        ov = max(1024, int(np.ceil(6 * excess * nbk)))
        ctx.set_tune(hash_bucket=m, hash_order=0)
        _, _, ws0 = kp.mul_bound(sparse, False, kp.KP_I64, "hash", na, nb, ctx)
        ctx.set_tune(hash_order=1)
        _, _, ws1 = kp.mul_bound(sparse, False, kp.KP_I64, "hash", na, nb, ctx)
        # (each workspace buffer starts on a 256-byte boundary; the C side's
        # Poisson sum may round one slot differently)
        assert abs((ws0 - ws_table) - 16 * (nbk * m + ov - cap)) < 256 + 32, m
        assert 20 * (na + nb) <= ws1 - ws0 < 20 * (na + nb) + 5 * 256
        if m == 1:
            assert ov > cap // 5   # a fifth of the codes overflow single-slot buckets at load 0.5
    # 128-bit sums ignore hash_bucket
    ctx.set_tune(hash_bucket=0)
    ws128 = kp.mul_bound(sparse, False, kp.KP_I128, "hash", na, nb, ctx)[2]
    ctx.set_tune(hash_bucket=8)
    assert kp.mul_bound(sparse, False, kp.KP_I128, "hash", na, nb, ctx)[2] == ws128


def test_host_context_rejects_launches():
    ctx = _host_ctx()
    lay = _layout_laurent([0], [3])
    st = kp.lib().kp_encode(ctx.h, C.byref(lay), 0, 0, None, None, None, None, None, 0, None)
    assert st == kp.KP_E_ARG


def test_to_pyint_round_trip():
    # 128-bit result words (low, high) to Python integers, both converters
    import oracle as O
    vals = [0, 1, -1, 2**64, -2**64, 2**127 - 1, -2**127, 3**70, -(5**50)]
    words = np.array([[(v & (2**64 - 1)) - (2**64 if v & (2**63) else 0), v >> 64] for v in vals],
                     np.int64)
    assert kp.to_pyint(words) == vals
    assert O.wide_to_int(words) == vals


def test_hash_plans_of_empty_and_tiny_products():
    """Workspace planning of hash products whose key space is empty, a single
    code or tiny, in both groupings (no launch)."""
    ctx = _host_ctx()
    empty = kp.layout_product(2, 0, [0, 0], [-1, -1], [0, 0], [3, 3])
    one = kp.layout_product(1, 0, [0], [0], [0], [0])
    small = kp.layout_product(2, 0, [0, 0], [3, 1], [0, 0], [2, 2])
    for grouping in (0, 1, 2):
        ctx.set_tune(hash_partitioned=2, hash_grouping=grouping)
        for lay, na, nb in ((empty, 0, 5), (empty, 5, 0), (one, 1, 1), (one, 7, 3), (small, 1, 1),
                            (small, 300, 2)):
            m, mo, ws = kp.mul_bound(lay, False, kp.KP_I64, "hash", na, nb, ctx)
            assert m == "hash" and 0 <= mo <= max(na * nb, 0) and ws >= 0


def test_pack_needs_a_device_context():
    """kp_pack_create refuses a host-only context and bad sizes before
    touching a device; null handles are argument errors."""
    import ctypes as C
    ctx = _host_ctx()
    h = C.c_void_p()
    L = kp.lib()
    assert L.kp_pack_create(ctx.h, 4, C.byref(h)) == kp.KP_E_ARG
    assert L.kp_pack_create(None, 4, C.byref(h)) == kp.KP_E_ARG
    assert L.kp_pack_destroy(None) == kp.KP_E_ARG
    assert L.kp_pack_wait(None, None) == kp.KP_E_ARG
    d = C.c_int32()
    assert L.kp_pack_query(None, C.byref(d)) == kp.KP_E_ARG


def test_tune_cache_round_trip(tmp_path):
    """The autotuner's JSON cache: a stored result comes back under the same
    key; the key changes with the library build and the tuning depth; a
    damaged file reads as empty."""
    from paper_1004_4548_amd import tune
    lib = tmp_path / "lib.so"
    lib.write_bytes(b"build one")
    k1 = tune.cache_key("MI355X", str(lib), True)
    assert k1 != tune.cache_key("MI355X", str(lib), False)
    path = str(tmp_path / "sub" / "tune.json")
    assert tune.load_cache(path) == {}
    res = {"chosen": {"window": 16384, "dense_keys_per_pair": 8.0}}
    tune.save_cache(path, k1, res)
    assert tune.load_cache(path)[k1] == res
    lib.write_bytes(b"build two")
    k2 = tune.cache_key("MI355X", str(lib), True)
    assert k2 != k1 and k2 not in tune.load_cache(path)
    tune.save_cache(path, k2, res)
    assert set(tune.load_cache(path)) == {k1, k2}
    with open(path, "w") as f:
        f.write("{not json")
    assert tune.load_cache(path) == {}


def test_tune_search_sums_products_and_restores_knobs():
    """The autotuner's search: a candidate's time is the sum over the products
    it is timed on, the fastest sum wins (a setting that only ties on one
    product does not beat one that wins on the other), and the knobs held
    while timing are put back."""
    from paper_1004_4548_amd import tune
    import ctypes as C

    class Knobs(C.Structure):
        _fields_ = [("slots", C.c_int32), ("fill", C.c_int32), ("grouping", C.c_int32)]

    class Ctx:
        def __init__(self):
            self.k = Knobs(4096, 42, 0)
            self.seen = []

        @property
        def tune(self):
            return Knobs(self.k.slots, self.k.fill, self.k.grouping)

        def set_tune(self, **kw):
            for f, v in kw.items():
                setattr(self.k, f, v)

    ctx = Ctx()

    class Prod:
        def __init__(self, times):
            self.times = times

        def seconds(self, mode, reps):
            ctx.seen.append((ctx.k.slots, ctx.k.grouping))
            return self.times[ctx.k.slots]

    ranges = Prod({2048: 5.49, 4096: 5.54, 8192: 6.1})   # 2048 ties on this one
    levels = Prod({2048: 1.52, 4096: 1.12, 8192: 1.2})   # and loses on this one
    grid = [dict(slots=s) for s in (2048, 4096, 8192)]
    best, table = tune._search(ctx, [ranges, levels], "hash", grid, 1, fixed=dict(grouping=2))
    assert best == dict(slots=4096)
    assert [round(t, 2) for t, _ in table] == [6.66, 7.01, 7.3]
    assert all(g == 2 for _, g in ctx.seen) and len(ctx.seen) == 6
    assert (ctx.k.slots, ctx.k.fill, ctx.k.grouping) == (4096, 42, 0)
    alone, _ = tune._search(ctx, ranges, "hash", grid, 1)   # one product, not a list
    assert alone == dict(slots=2048)


def test_tune_crossover():
    """The dense/hash switch from timed rows (codes per pair, dense s, hash
    s): the geometric mean of the sparsest shape where dense still wins and
    the densest sparser one where hash wins; 0 when hash always wins; the
    larger of the fallback and the last dense win when dense always wins."""
    from paper_1004_4548_amd import tune
    rows = [(1.0, 1, 2), (4.0, 1, 2), (9.0, 3, 2), (16.0, 5, 2), (2.0, 1, 3)]
    assert tune._crossover(rows, 32.0) == pytest.approx(6.0)   # sqrt(4 * 9)
    assert tune._crossover([(r, 2, 1) for r in (1.0, 5.0)], 32.0) == 0.0
    assert tune._crossover([(r, 1, 2) for r in (1.0, 5.0)], 32.0) == 32.0
    assert tune._crossover([(r, 1, 2) for r in (1.0, 50.0)], 32.0) == 50.0
    # a hash win below the last dense win does not set the upper end
    assert tune._crossover([(1.0, 2, 1), (4.0, 1, 2), (9.0, 2, 1)], 32.0) == pytest.approx(6.0)
