"""Pins for the CPU oracle: each check fixes it against something other than itself.

* Laurent products: n-D convolution of dense coefficient boxes (scipy / numpy,
  a different formulation of the same product), the closed form of Fateman's
  benchmark f*(f+1) = f^2 + f (Section 5), the Monagan-Pearce benchmark through
  its closed-form evaluation (Section 5), wrap-around modulo 2^64, and the
  Schwartz-Zippel evaluation identity eval(A*B) = eval(A)*eval(B) mod 2^61-1.
* Poisson products: the product-to-sum identities (Section 2, eq. werner, with
  the factor 1/2), Chebyshev's recurrence, numeric evaluation at random angles
  and exact evaluation over F_{p^2}.
* The evaluators themselves: binomial closed forms and exact field identities.
* Truncated products (Section 3): brute force that tests every pair against
  the degree limit before it contributes, a binomial closed form, the limits.
"""
import math

import numpy as np
import pytest
from scipy import signal

import oracle as O
from paper_1004_4548_amd import inputs as I

P = O.P61


def _dense(exps, coef, lo, shape, dtype=np.int64):
    d = np.zeros(shape, dtype=dtype)
    for e, c in zip(exps, coef):
        d[tuple(np.asarray(e) - lo)] += c
    return d


def _to_dict(exps, coef):
    return {tuple(int(v) for v in e): c for e, c in zip(exps, coef)}


# ---------------------------------------------------------------- Laurent pins
@pytest.mark.parametrize("nv,lo,hi,n,seed", [(1, -6, 9, 12, 1), (2, -3, 4, 20, 2), (3, -2, 2, 30, 3),
                                             (3, 0, 5, 60, 4), (4, -1, 2, 40, 5)])
def test_laurent_equals_nd_convolution(nv, lo, hi, n, seed):
    rng = np.random.default_rng(seed)
    ae = rng.integers(lo, hi + 1, size=(n, nv)).astype(np.int32)        # duplicates allowed
    be = rng.integers(lo, hi + 1, size=(n + 3, nv)).astype(np.int32)
    ac = rng.integers(-50, 51, size=n)
    bc = rng.integers(-50, 51, size=n + 3)
    w = hi - lo + 1
    da = _dense(ae, ac, lo, (w,) * nv)
    db = _dense(be, bc, lo, (w,) * nv)
    conv = signal.convolve(da, db, method="direct")                   # exact for int64
    ex, co, _ = O.laurent_mul(ae, ac, be, bc)
    got = _dense(ex, co, 2 * lo, conv.shape)
    np.testing.assert_array_equal(got, conv)
    assert len(co) == np.count_nonzero(conv)                          # zeros dropped


def test_laurent_univariate_equals_numpy_convolve():
    rng = np.random.default_rng(7)
    a = rng.integers(-9, 10, size=40)
    b = rng.integers(-9, 10, size=33)
    ae = np.nonzero(a)[0].reshape(-1, 1) - 11
    be = np.nonzero(b)[0].reshape(-1, 1) + 4
    ex, co, _ = O.laurent_mul(ae, a[a != 0], be, b[b != 0])
    ref = np.convolve(a, b)
    got = np.zeros_like(ref)
    got[ex[:, 0] + 11 - 4] = co
    np.testing.assert_array_equal(got, ref)


def test_laurent_fp64_equals_convolution():
    rng = np.random.default_rng(11)
    ae = rng.integers(-2, 3, size=(25, 2)).astype(np.int32)
    be = rng.integers(-2, 3, size=(25, 2)).astype(np.int32)
    ac = rng.integers(-99, 100, size=25).astype(np.float64) / 8.0   # dyadic: exact sums
    bc = rng.integers(-99, 100, size=25).astype(np.float64) / 4.0
    conv = signal.convolve(_dense(ae, ac, -2, (5, 5), np.float64),
                           _dense(be, bc, -2, (5, 5), np.float64), method="direct")
    ex, co, ab = O.laurent_mul(ae, ac, be, bc)
    got = _dense(ex, co, -4, conv.shape, np.float64)
    np.testing.assert_array_equal(got, conv)
    absconv = signal.convolve(_dense(ae, np.abs(ac), -2, (5, 5), np.float64),
                              _dense(be, np.abs(bc), -2, (5, 5), np.float64), method="direct")
    # abs_sum per key equals the convolution of |coefficients| when no input key repeats
    ua, ub = np.unique(ae, axis=0), np.unique(be, axis=0)
    if len(ua) == len(ae) and len(ub) == len(be):
        np.testing.assert_allclose(_dense(ex, ab, -4, conv.shape, np.float64), absconv)


def test_fp64_abs_sum_and_cancellation():
    # (1 + x)(1 - x) = 1 - x^2, the x term cancels to 0 with abs_sum 2
    ex, co, ab = O.laurent_mul([[0], [1]], np.array([1.0, 1.0]), [[0], [1]], np.array([1.0, -1.0]))
    d = _to_dict(ex, zip(co, ab))
    assert d[(0,)] == (1.0, 1.0)
    assert d[(1,)] == (0.0, 2.0)
    assert d[(2,)] == (-1.0, 1.0)


@pytest.mark.parametrize("k", [2, 3, 5, 7])
def test_fateman_closed_form(k):
    # Section 5: f = (1+x+y+z+t)^k, g = f + 1, so f*g = f^2 + f and each
    # coefficient is multinomial(2k; e) + [|e| <= k] multinomial(k; e).
    fe, fc = I.fateman(k)
    ge, gc = I.fateman(k, plus_one=True)
    assert len(fe) == math.comb(k + 4, 4)
    ex, co, _ = O.laurent_mul(fe, fc, ge, gc)
    assert len(ex) == math.comb(2 * k + 4, 4)
    for e, c in zip(ex, co):
        e = tuple(int(v) for v in e)
        want = I.multinomial(2 * k, e) + (I.multinomial(k, e) if sum(e) <= k else 0)
        assert int(c) == want


def test_fateman_30_term_counts():
    # The paper states 46376 terms for f and g at k = 30; the product has C(64, 4).
    fe, _ = I.fateman(30)
    assert len(fe) == 46376 == math.comb(34, 4)
    assert math.comb(64, 4) == 635376


def test_int64_wraps_mod_2_64():
    x = [[1]]
    ex, co, _ = O.laurent_mul(x, np.array([2**62]), [[0]], np.array([4]))
    assert len(ex) == 0                                    # 2^64 wraps to 0 and is dropped
    ex, co, _ = O.laurent_mul(x, np.array([3 * 2**62 - 2**64]), [[0]], np.array([3]))
    assert int(co[0]) == (9 * 2**62 - 3 * 2**64) % 2**64 == 2**62
    big = np.array([2**63 - 1])
    ex, co, _ = O.laurent_mul(x, big, x, big)
    assert int(co[0]) % 2**64 == ((2**63 - 1) ** 2) % 2**64


def test_duplicates_and_commutativity():
    rng = np.random.default_rng(3)
    ae = rng.integers(-3, 4, size=(50, 3)).astype(np.int32)
    be = rng.integers(-3, 4, size=(40, 3)).astype(np.int32)
    ac = rng.integers(-1000, 1000, size=50)
    bc = rng.integers(-1000, 1000, size=40)
    r1 = O.laurent_mul(ae, ac, be, bc)
    r2 = O.laurent_mul(be, bc, ae, ac)
    np.testing.assert_array_equal(r1[0], r2[0])
    np.testing.assert_array_equal(r1[1], r2[1])
    # splitting a term into two halves leaves the product unchanged (bilinearity)
    ae2 = np.concatenate([ae, ae[:1]])
    ac2 = ac.copy()
    ac2[0] = 7
    ac2 = np.concatenate([ac2, [ac[0] - 7]])
    r3 = O.laurent_mul(ae2, ac2, be, bc)
    np.testing.assert_array_equal(r1[0], r3[0])
    np.testing.assert_array_equal(r1[1], r3[1])


def test_threaded_oracle_matches_single_thread():
    a, b = I.config(2, scale=0.03)
    r1 = O.laurent_mul(a[0], a[1], b[0], b[1], threads=1)
    r4 = O.laurent_mul(a[0], a[1], b[0], b[1], threads=4)
    np.testing.assert_array_equal(r1[0], r4[0])
    np.testing.assert_array_equal(r1[1], r4[1])


# ------------------------------------------------------------ evaluator pins
def test_eval_modp_binomial_closed_form():
    n = 20
    e = np.arange(-n, 1).reshape(-1, 1)         # x^-n .. x^0 with binomial coefficients
    c = np.array([math.comb(n, i) for i in range(n, -1, -1)])
    for r in (2, 12345, P - 3):
        rinv = pow(r, P - 2, P)
        assert O.laurent_eval_modp(e, c, [r]) == pow(1 + rinv, n, P)
    # fp64 coefficients are mapped exactly: 3/8 x^2 at r = 4 gives 6
    assert O.laurent_eval_modp([[2]], np.array([0.375]), [4]) == 6
    assert O.laurent_eval_modp([[0]], np.array([-0.5]), [4]) == (P - pow(2, P - 2, P)) % P


def test_fp2_field_identities():
    assert O.fp2_mul((0, 1), (0, 1)) == (P - 1, 0)           # i^2 = -1
    z = (123456789, 987654321)
    zc = O.poisson_eval_fp2(([[0]], [[1]], [0], [1.0]), 1, 1, [5], [z])
    zs = O.poisson_eval_fp2(([[0]], [[1]], [1], [1.0]), 1, 1, [5], [z])
    s = O.fp2_mul(zc, zc)
    t = O.fp2_mul(zs, zs)
    assert ((s[0] + t[0]) % P, (s[1] + t[1]) % P) == (1, 0)   # cos^2 + sin^2 = 1


def test_mp_sparse_closed_form_evaluation():
    # Section 5: f = (1+x+y+2z^2+3t^3+5u^5)^k, g = (1+u+t+2z^2+3y^3+5x^5)^k.
    # eval(f*g) must equal the closed form of the two bases raised to k.
    k = 4
    fe, fc = I.mp_sparse(k, "f")
    ge, gc = I.mp_sparse(k, "g")
    assert len(I.mp_sparse(12, "f")[0]) == 6188 == math.comb(17, 5)
    ex, co, _ = O.laurent_mul(fe, fc, ge, gc)
    rng = np.random.default_rng(99)
    for _ in range(3):
        x, y, z, t, u = (int(v) for v in rng.integers(2, P - 1, size=5))
        bf = (1 + x + y + 2 * z**2 + 3 * t**3 + 5 * u**5) % P
        bg = (1 + u + t + 2 * z**2 + 3 * y**3 + 5 * x**5) % P
        assert O.laurent_eval_modp(ex, co, [x, y, z, t, u]) == pow(bf, k, P) * pow(bg, k, P) % P


def test_schwartz_zippel_random_laurent():
    rng = np.random.default_rng(5)
    a, b = I.config(1, scale=0.2)
    ex, co, _ = O.laurent_mul(a[0], a[1], b[0], b[1])
    for _ in range(3):
        pt = [int(v) for v in rng.integers(2, P - 1, size=3)]
        lhs = O.laurent_eval_modp(ex, co, pt)
        rhs = O.laurent_eval_modp(a[0], a[1], pt) * O.laurent_eval_modp(b[0], b[1], pt) % P
        assert lhs == rhs


# ---------------------------------------------------------------- Poisson pins
def _one(x, j, t, c, nx=1):
    return (np.array([x], dtype=np.int32).reshape(1, nx), np.array([j], dtype=np.int32),
            np.array([t], dtype=np.uint8), np.array([c], dtype=np.float64))


def _pdict(res):
    x, y, t, c, _ = res
    return {(tuple(xx), tuple(yy), int(tt)): cc for xx, yy, tt, cc in zip(x.tolist(), y.tolist(), t, c)}


def test_werner_cos_cos_and_sin_sin():
    cy = _one([0], [1], 0, 1.0)
    sy = _one([0], [1], 1, 1.0)
    cc = _pdict(O.poisson_mul(cy, cy, 1, 1))
    ss = _pdict(O.poisson_mul(sy, sy, 1, 1))
    assert cc == {((0,), (0,), 0): 0.5, ((0,), (2,), 0): 0.5}        # cos^2 = 1/2 + 1/2 cos 2y
    assert ss == {((0,), (0,), 0): 0.5, ((0,), (2,), 0): -0.5}       # sin^2 = 1/2 - 1/2 cos 2y


def test_werner_mixed_drops_sin_zero():
    cy = _one([1], [1], 0, 1.0)
    sy = _one([2], [1], 1, 1.0)
    sc = _pdict(O.poisson_mul(sy, cy, 1, 1))
    cs = _pdict(O.poisson_mul(cy, sy, 1, 1))
    assert sc == {((3,), (2,), 1): 0.5} == cs                       # sin y cos y = 1/2 sin 2y


def test_werner_signs_and_canonical_fold():
    # cos(y1) * sin(y2) = 1/2 sin(y1+y2) - 1/2 sin(y1-y2)
    c1 = (np.zeros((1, 1), np.int32), np.array([[1, 0]], np.int32), np.array([0], np.uint8), np.array([1.0]))
    s2 = (np.zeros((1, 1), np.int32), np.array([[0, 1]], np.int32), np.array([1], np.uint8), np.array([1.0]))
    r = _pdict(O.poisson_mul(c1, s2, 1, 2))
    assert r == {((0,), (1, 1), 1): 0.5, ((0,), (1, -1), 1): -0.5}
    # sin(y2) * cos(y1) = 1/2 sin(y2-y1) + 1/2 sin(y1+y2); sin(-(y1-y2)) folds to -sin(y1-y2)
    r2 = _pdict(O.poisson_mul(s2, c1, 1, 2))
    assert r2 == r
    # sin(y1)*sin(y2) = 1/2 cos(y1-y2) - 1/2 cos(y1+y2)
    s1 = (c1[0], c1[1], np.array([1], np.uint8), c1[3])
    r3 = _pdict(O.poisson_mul(s1, s2, 1, 2))
    assert r3 == {((0,), (1, -1), 0): 0.5, ((0,), (1, 1), 0): -0.5}
    # cos(y2) * cos(y1): cos(y2 - y1) folds to cos(y1 - y2) with the same sign
    c2 = (c1[0], s2[1], np.array([0], np.uint8), c1[3])
    r4 = _pdict(O.poisson_mul(c2, c1, 1, 2))
    assert r4 == {((0,), (1, -1), 0): 0.5, ((0,), (1, 1), 0): 0.5}


@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_chebyshev(n):
    # cos(n y) cos(y) = 1/2 cos((n-1) y) + 1/2 cos((n+1) y)
    r = _pdict(O.poisson_mul(_one([0], [n], 0, 1.0), _one([0], [1], 0, 1.0), 1, 1))
    want = {((0,), (n - 1,), 0): 0.5, ((0,), (n + 1,), 0): 0.5}
    if n == 1:
        want = {((0,), (0,), 0): 0.5, ((0,), (2,), 0): 0.5}
    assert r == want


def _eval_numeric(series, xs, ys):
    x, y, t, c = series[:4]
    xv = np.prod(np.asarray(xs, dtype=np.longdouble)[None, :] ** x.astype(np.longdouble), axis=1)
    ang = (y.astype(np.longdouble) * np.asarray(ys, dtype=np.longdouble)[None, :]).sum(axis=1)
    trig = np.where(t.astype(bool), np.sin(ang), np.cos(ang))
    terms = np.asarray(c, dtype=np.longdouble) * xv * trig
    return terms.sum(), np.abs(terms).sum()


def test_poisson_numeric_evaluation():
    a, b = I.config(4, scale=0.04)          # 200 x 200 terms, N(0,1) * 2^-|j| coefficients
    res = O.poisson_mul(a, b, 3, 6)
    rng = np.random.default_rng(8)
    for _ in range(4):
        xs = rng.uniform(0.5, 1.5, size=3)
        ys = rng.uniform(-np.pi, np.pi, size=6)
        va, sa = _eval_numeric(a, xs, ys)
        vb, sb = _eval_numeric(b, xs, ys)
        vp, sp = _eval_numeric(res, xs, ys)
        assert abs(vp - va * vb) <= 1e-12 * (sa * sb)


def test_poisson_exact_fp2_evaluation():
    nx, ny = 2, 3
    a = I.poisson_random(nx=nx, ny=ny, n=60, xlo=-2, xhi=2, jmax=3, coef="f64int", cfg=90, factor=0)
    b = I.poisson_random(nx=nx, ny=ny, n=50, xlo=-2, xhi=2, jmax=3, coef="f64int", cfg=90, factor=1)
    res = O.poisson_mul(a, b, nx, ny)
    rng = np.random.default_rng(4)
    for _ in range(3):
        xp = [int(v) for v in rng.integers(2, P - 1, size=nx)]
        zp = [tuple(int(v) for v in rng.integers(1, P - 1, size=2)) for _ in range(ny)]
        ea = O.poisson_eval_fp2(a, nx, ny, xp, zp)
        eb = O.poisson_eval_fp2(b, nx, ny, xp, zp)
        assert O.poisson_eval_fp2(res[:4], nx, ny, xp, zp) == O.fp2_mul(ea, eb)


def test_poisson_output_is_canonical_and_sin_zero_free():
    a, b = I.config(4, scale=0.02)
    x, y, t, c, ab = O.poisson_mul(a, b, 3, 6)
    for yy, tt in zip(y, t):
        nz = np.flatnonzero(yy)
        if len(nz) == 0:
            assert tt == 0
        else:
            assert yy[nz[0]] > 0


# ------------------------------------------------------- one-by-one spot checks
def test_laurent_coeff_at_matches_full_product():
    a, b = I.config(1, scale=0.3)
    ex, co, _ = O.laurent_mul(a[0], a[1], b[0], b[1])
    q = np.concatenate([ex[::7], np.array([[40, 40, 40], [-11, 0, 1]], np.int32)])
    got, _, cnt = O.laurent_coeff_at(a[0], a[1], b[0], b[1], q)
    want = list(co[::7]) + [0, 0]
    np.testing.assert_array_equal(got, want)
    assert cnt[-2] == 0


def test_laurent_coeff_at_fateman():
    k = 4
    fe, fc = I.fateman(k)
    ge, gc = I.fateman(k, plus_one=True)
    q = np.array([[0, 0, 0, 0], [1, 2, 3, 2], [8, 0, 0, 0], [2, 2, 2, 2]], np.int32)
    got, _, _ = O.laurent_coeff_at(fe, fc, ge, gc, q)
    for e, c in zip(q, got):
        e = tuple(int(v) for v in e)
        assert int(c) == I.multinomial(2 * k, e) + (I.multinomial(k, e) if sum(e) <= k else 0)


def test_poisson_coeff_at_matches_full_product():
    a, b = I.config(4, scale=0.02)
    x, y, t, c, ab = O.poisson_mul(a, b, 3, 6)
    sel = np.arange(0, len(c), max(1, len(c) // 50))
    got, gab, cnt = O.poisson_coeff_at(a, b, 3, 6, x[sel], y[sel], t[sel])
    np.testing.assert_allclose(got, c[sel], rtol=0, atol=1e-15 * np.max(ab))
    np.testing.assert_allclose(gab, ab[sel], rtol=1e-14)
    # a key that no pair reaches
    got, _, cnt = O.poisson_coeff_at(a, b, 3, 6, [[50, 0, 0]], [[1, 0, 0, 0, 0, 0]], [0])
    assert got[0] == 0 and cnt[0] == 0


# ------------------------------------------------------------------ truncation
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_truncated_equals_brute_force_with_pair_test(seed):
    """Every pair tested against the limit before it contributes (the
    efficient form a multiplier uses), in Python integers mod 2^64, equals the
    oracle's product-then-filter."""
    rng = np.random.default_rng(900 + seed)
    nv = 3
    a = (rng.integers(-3, 5, (40, nv)).astype(np.int32), rng.integers(-50, 50, 40))
    b = (rng.integers(-2, 6, (30, nv)).astype(np.int32), rng.integers(-50, 50, 30))
    w = [int(x) for x in rng.integers(-2, 4, nv)]
    D = int(rng.integers(-3, 12))
    acc = {}
    for ea, ca in zip(a[0].tolist(), a[1].tolist()):
        da = sum(x * y for x, y in zip(w, ea))
        for eb, cb in zip(b[0].tolist(), b[1].tolist()):
            if da + sum(x * y for x, y in zip(w, eb)) > D:
                continue
            k = tuple(x + y for x, y in zip(ea, eb))
            acc[k] = (acc.get(k, 0) + ca * cb) % (1 << 64)
    ref = {k: (v - (1 << 64) if v >= (1 << 63) else v) for k, v in acc.items() if v}
    ex, co, _ = O.laurent_mul_truncated(a[0], a[1], b[0], b[1], w, D)
    got = {tuple(e): int(c) for e, c in zip(ex.tolist(), co.tolist())}
    assert got == ref


@pytest.mark.parametrize("n,m,D", [(5, 4, 6), (7, 7, 3), (6, 2, 8)])
def test_truncated_binomial_closed_form(n, m, D):
    """(1+x+y)^n (1+x+y)^m cut at total degree D: the multinomial coefficients
    of (1+x+y)^(n+m) of degree <= D."""
    def poly(k):
        ex, co = [], []
        for i in range(k + 1):
            for j in range(k + 1 - i):
                ex.append((i, j))
                co.append(math.comb(k, i) * math.comb(k - i, j))
        return np.array(ex, np.int32), np.array(co, np.int64)
    a, b = poly(n), poly(m)
    ex, co, _ = O.laurent_mul_truncated(a[0], a[1], b[0], b[1], [1, 1], D)
    N = n + m
    want = {(i, j): math.comb(N, i) * math.comb(N - i, j)
            for i in range(N + 1) for j in range(N + 1 - i) if i + j <= D}
    assert {tuple(e): int(c) for e, c in zip(ex.tolist(), co.tolist())} == want


def test_truncated_limits():
    rng = np.random.default_rng(77)
    a = (rng.integers(0, 5, (25, 2)).astype(np.int32), rng.integers(1, 9, 25))
    b = (rng.integers(0, 5, (20, 2)).astype(np.int32), rng.integers(1, 9, 20))
    full = O.laurent_mul(a[0], a[1], b[0], b[1])
    top = O.laurent_mul_truncated(a[0], a[1], b[0], b[1], [1, 1], 16)
    assert np.array_equal(full[0], top[0]) and np.array_equal(full[1], top[1])
    none = O.laurent_mul_truncated(a[0], a[1], b[0], b[1], [1, 1], -1)
    assert len(none[1]) == 0
    # weight 0 on a variable: only the other one is cut
    part = O.laurent_mul_truncated(a[0], a[1], b[0], b[1], [0, 1], 3)
    assert (part[0][:, 1] <= 3).all() and part[0][:, 0].max() > 3


# ------------------------------------------------ truncation by harmonic order
def _cos_sum_squared():
    # (cos y1 + cos y2)^2 = 1 + 1/2 cos 2y1 + 1/2 cos 2y2 + cos(y1 + y2) + cos(y1 - y2)
    s = (np.zeros((2, 1), np.int32), np.array([[1, 0], [0, 1]], np.int32),
         np.zeros(2, np.uint8), np.array([1.0, 1.0]))
    return s


@pytest.mark.parametrize("w,H,want", [
    ([1, 2], 3, {(0, 0): 1.0, (2, 0): 0.5, (1, 1): 1.0, (1, -1): 1.0}),
    ([1, 2], 2, {(0, 0): 1.0, (2, 0): 0.5}),
    ([1, 1], 1, {(0, 0): 1.0}),
    ([1, 1], 2, {(0, 0): 1.0, (2, 0): 0.5, (0, 2): 0.5, (1, 1): 1.0, (1, -1): 1.0}),
    ([0, 1], 0, {(0, 0): 1.0, (2, 0): 0.5}),
])
def test_harmonic_truncation_closed_form(w, H, want):
    """(cos y1 + cos y2)^2 cut at weighted harmonic order H: the terms of the
    closed form whose order sum_k w_k |j_k| is at most H."""
    s = _cos_sum_squared()
    x, y, t, c, _ = O.poisson_mul_truncated(s, s, 1, 2, w, H)
    got = {tuple(int(v) for v in j): float(v) for j, v, tt in zip(y, c, t) if v != 0}
    assert (t == 0).all()
    assert got == want


def _werner_pieces(ja, ta, jb, tb, c):
    """The two pieces of one pair (Section 2, with the factor 1/2), each folded
    to canonical form: [(j, is_sin, coefficient)]."""
    d = tuple(p - q for p, q in zip(ja, jb))
    s = tuple(p + q for p, q in zip(ja, jb))
    h = 0.5 * c
    if not ta and not tb:
        raw = [(d, 0, h), (s, 0, h)]
    elif ta and tb:
        raw = [(d, 0, h), (s, 0, -h)]
    elif ta and not tb:
        raw = [(s, 1, h), (d, 1, h)]
    else:
        raw = [(s, 1, h), (d, 1, -h)]
    out = []
    for j, t, v in raw:
        nz = [q for q in j if q != 0]
        if nz and nz[0] < 0:
            j = tuple(-q for q in j)
            if t:
                v = -v
        if t and not nz:
            continue
        out.append((j, t, v))
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_harmonic_truncation_brute_force(seed):
    """Each piece tested against the order limit before it contributes (in
    Python, written from the product-to-sum rule), against the oracle's
    product-then-filter."""
    nx, ny = 1, 3
    a = I.poisson_random(nx=nx, ny=ny, n=30, xlo=-2, xhi=2, jmax=3, coef="f64int", cfg=91 + seed,
                         factor=0)
    b = I.poisson_random(nx=nx, ny=ny, n=25, xlo=-2, xhi=2, jmax=3, coef="f64int", cfg=91 + seed,
                         factor=1)
    w, H = [1, 2, 1], 5 + seed
    acc = {}
    for xa, ja, ta, ca in zip(a[0].tolist(), a[1].tolist(), a[2].tolist(), a[3].tolist()):
        for xb, jb, tb, cb in zip(b[0].tolist(), b[1].tolist(), b[2].tolist(), b[3].tolist()):
            xs = tuple(p + q for p, q in zip(xa, xb))
            for j, t, v in _werner_pieces(ja, ta, jb, tb, ca * cb):
                if sum(wk * abs(q) for wk, q in zip(w, j)) > H:
                    continue
                k = (xs, j, t)
                acc[k] = acc.get(k, 0.0) + v
    want = {k: v for k, v in acc.items() if v != 0}
    x, y, t, c, _ = O.poisson_mul_truncated(a, b, nx, ny, w, H)
    got = {(tuple(xx), tuple(yy), int(tt)): float(cc)
           for xx, yy, tt, cc in zip(x.tolist(), y.tolist(), t.tolist(), c.tolist()) if cc != 0}
    assert got == want   # integer-valued halves: exact in fp64


def test_harmonic_truncation_limits():
    a, b = I.config(4, scale=0.01)
    full = O.poisson_mul(a, b, 3, 6)
    top = O.poisson_mul_truncated(a, b, 3, 6, [1] * 6, 10**6)
    assert all(np.array_equal(u, v) for u, v in zip(full, top))
    assert len(O.poisson_mul_truncated(a, b, 3, 6, [1] * 6, -1)[3]) == 0


# ------------------------------------------------------------ exact (128-bit) products
def _signed128(v):
    v %= 1 << 128
    return v - (1 << 128) if v >= 1 << 127 else v


def _brute_int(ae, ac, be, bc):
    """Schoolbook product in Python integers, reduced to signed 128 bits at
    the end (the exact value whenever it fits)."""
    out = {}
    for e, c in zip(np.asarray(ae).tolist(), np.asarray(ac).tolist()):
        for f, d in zip(np.asarray(be).tolist(), np.asarray(bc).tolist()):
            k = tuple(x + y for x, y in zip(e, f))
            out[k] = out.get(k, 0) + int(c) * int(d)
    out = {k: _signed128(v) for k, v in out.items()}
    return {k: v for k, v in out.items() if v != 0}


@pytest.mark.parametrize("seed,bits", [(0, 63), (1, 63), (2, 58), (3, 58)])
def test_exact_equals_python_integers(seed, bits):
    # Section 5 compares against exact integer arithmetic.  With 63-bit
    # coefficients every product is near 2^126, so sums carry across the
    # 64-bit word boundary and some wrap modulo 2^128; with 58-bit ones the
    # products stay below 2^116 and every sum is the exact integer.
    rng = np.random.default_rng(40 + seed)
    na, nb, nv = 60, 45, 3
    ae = rng.integers(-2, 3, size=(na, nv)).astype(np.int32)
    be = rng.integers(-2, 3, size=(nb, nv)).astype(np.int32)
    hi = 2**bits - 1
    ext = np.array([hi, -hi - 1, -hi, 1, -1, 0], dtype=np.int64)
    ac = np.concatenate([ext, rng.integers(-hi - 1, hi, size=na - 6, dtype=np.int64)])
    bc = np.concatenate([ext[:5], rng.integers(-hi - 1, hi, size=nb - 5, dtype=np.int64)])
    ex, co, ab = O.laurent_mul(ae, ac, be, bc, exact=True)
    assert ab is None and co.shape == (len(ex), 2)
    got = dict(zip(map(tuple, ex.tolist()), O.wide_to_int(co)))
    want = _brute_int(ae, ac, be, bc)
    assert got == want
    if bits == 58:
        assert max(abs(v) for v in want.values()) < 2**127


@pytest.mark.parametrize("k,c", [(3, 3**37), (3, -(3**37)), (4, 7**19)])
def test_exact_scaled_fateman_closed_form(k, c):
    # f = c (1+x+y+z+t)^k, g = f + 1: f g = c^2 (1+...)^(2k) + c (1+...)^k, so
    # each coefficient is c^2 multinomial(2k; e) + c [|e| <= k] multinomial(k; e),
    # with values up to 2^124 (beyond any 64-bit accumulator).
    fe, fc = I.fateman(k)
    fc = fc * c
    gc = fc.copy()
    gc[np.all(fe == 0, axis=1)] += 1
    ex, co, _ = O.laurent_mul(fe, fc, fe, gc, exact=True)
    assert len(ex) == math.comb(2 * k + 4, 4)
    big = 0
    for e, v in zip(ex, O.wide_to_int(co)):
        e = tuple(int(x) for x in e)
        want = c * c * I.multinomial(2 * k, e) + (c * I.multinomial(k, e) if sum(e) <= k else 0)
        assert v == want
        big = max(big, abs(v))
    assert big > 2**100


def test_exact_low_word_and_coeff_at():
    # The low word of the exact sum is the int64 result modulo 2^64, and the
    # one-query-at-a-time form agrees with the full product.
    rng = np.random.default_rng(7)
    ae = rng.integers(-3, 4, size=(80, 2)).astype(np.int32)
    be = rng.integers(-3, 4, size=(70, 2)).astype(np.int32)
    ac = rng.integers(-2**62, 2**62, size=80, dtype=np.int64)
    bc = rng.integers(-2**62, 2**62, size=70, dtype=np.int64)
    ex, co, _ = O.laurent_mul(ae, ac, be, bc, exact=True)
    ex0, co0, _ = O.laurent_mul(ae, ac, be, bc)
    low = {k: int(v) % 2**64 for k, v in zip(map(tuple, ex0.tolist()), co0)}
    for k, v in zip(map(tuple, ex.tolist()), O.wide_to_int(co)):
        assert low.get(k, 0) == v % 2**64
    q = np.concatenate([ex[::5], np.array([[50, 50]], np.int32)])
    got, ab, cnt = O.laurent_coeff_at(ae, ac, be, bc, q, exact=True)
    assert ab is None and cnt[-1] == 0
    assert O.wide_to_int(got) == O.wide_to_int(co[::5]) + [0]
