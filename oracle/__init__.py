"""CPU oracle for sparse Laurent-polynomial and Poisson-series products.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product path never
does, and the two share no code.

The arithmetic lives in ``kp_oracle.cpp`` (std::map over exponent tuples,
written from the paper's definitions: eq. ps_def for the term model, the
schoolbook product of Section 3, and the product-to-sum identities of eq.
werner with their factor 1/2).  This module only marshals numpy arrays in and
out of that library.

Every function here is pinned by ``tests/test_oracle_pins.py``:
  * ``laurent_mul``      -- n-D convolution, Fateman closed form, mod-p
                            evaluation of the Monagan-Pearce benchmark;
  * ``laurent_mul(..., exact=True)`` -- brute force in Python integers, the
                            closed form of scaled Fateman-type products;
  * ``laurent_mul_truncated`` -- brute force with the degree test on each
                            pair, a binomial closed form, the limiting cuts;
  * ``poisson_mul``      -- trigonometric identities, numeric evaluation at
                            random angles, exact evaluation over F_{p^2};
  * ``*_coeff_at``       -- against the full product on random inputs, whose
                            own pins are above, and against closed forms;
  * ``*_eval_*``         -- closed forms of binomial/trigonometric sums.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
P61 = (1 << 61) - 1

_lib = None

_p = C.c_void_p
_i64 = C.c_int64
_i32 = C.c_int
_u64 = C.c_uint64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    lib.oracle_laurent_mul.restype = _p
    lib.oracle_laurent_mul.argtypes = [_i32, _i32, _i64, _p, _p, _i64, _p, _p, _i64, _i64, _i32]
    lib.oracle_laurent_len.restype = _i64
    lib.oracle_laurent_len.argtypes = [_p]
    lib.oracle_laurent_get.restype = None
    lib.oracle_laurent_get.argtypes = [_p, _p, _p, _p]
    lib.oracle_laurent_free.restype = None
    lib.oracle_laurent_free.argtypes = [_p]
    lib.oracle_laurent_coeff_at.restype = None
    lib.oracle_laurent_coeff_at.argtypes = [_i32, _i32, _i64, _p, _p, _i64, _p, _p, _i64, _p,
                                            _p, _p, _p]
    lib.oracle_poisson_mul.restype = _p
    lib.oracle_poisson_mul.argtypes = [_i32, _i32, _i64, _p, _p, _p, _p, _i64, _p, _p, _p, _p,
                                       _i64, _i64, _i32]
    lib.oracle_poisson_len.restype = _i64
    lib.oracle_poisson_len.argtypes = [_p]
    lib.oracle_poisson_get.restype = None
    lib.oracle_poisson_get.argtypes = [_p, _p, _p, _p, _p, _p]
    lib.oracle_poisson_free.restype = None
    lib.oracle_poisson_free.argtypes = [_p]
    lib.oracle_poisson_coeff_at.restype = None
    lib.oracle_poisson_coeff_at.argtypes = [_i32, _i32, _i64, _p, _p, _p, _p, _i64, _p, _p, _p,
                                            _p, _i64, _p, _p, _p, _p, _p, _p]
    lib.oracle_laurent_eval_modp_i64.restype = _u64
    lib.oracle_laurent_eval_modp_i64.argtypes = [_i32, _i64, _p, _p, _p]
    lib.oracle_laurent_eval_modp_f64.restype = _u64
    lib.oracle_laurent_eval_modp_f64.argtypes = [_i32, _i64, _p, _p, _p]
    lib.oracle_poisson_eval_fp2.restype = None
    lib.oracle_poisson_eval_fp2.argtypes = [_i32, _i32, _i64, _p, _p, _p, _p, _p, _p, _p, _p]
    lib.oracle_modp_mul.restype = _u64
    lib.oracle_modp_mul.argtypes = [_u64, _u64]
    lib.oracle_modp_pow.restype = _u64
    lib.oracle_modp_pow.argtypes = [_u64, _u64]
    lib.oracle_fp2_mul.restype = None
    lib.oracle_fp2_mul.argtypes = [_p, _p, _p]
    lib.oracle_hardware_threads.restype = _i32
    lib.oracle_hardware_threads.argtypes = []
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _exps(e, nv=None):
    e = np.ascontiguousarray(e, dtype=np.int32)
    if e.ndim == 1:
        e = e.reshape(-1, 1 if nv is None else nv)
    return e


def _coef(c):
    c = np.asarray(c)
    if c.dtype == np.float64:
        return np.ascontiguousarray(c), 1
    return np.ascontiguousarray(c, dtype=np.int64), 0


def hardware_threads() -> int:
    return int(_load().oracle_hardware_threads())


def laurent_mul(a_exps, a_coef, b_exps, b_coef, row_begin=0, row_end=-1, threads=1,
                exact=False):
    """Product of two Laurent polynomials given as (exponents[n, nv], coef[n]).

    Coefficients are int64 (wrapping mod 2^64) or float64.  With
    ``exact=True`` (int64 factors) every product and sum is formed in signed
    128-bit integers and ``coef`` is int64[m, 2]: the low and the high word of
    each two's complement value (``wide_to_int`` turns them into Python
    integers).  Returns ``(exps[m, nv] int32, coef, abs_sum[m] or None)``
    sorted by exponent tuple.  Integer results omit zero terms; float64
    results keep every touched key (with its sum of |contributions|).
    Only A's rows [row_begin, row_end) take part (for bounded timing samples).
    """
    lib = _load()
    ae, be = _exps(a_exps), _exps(b_exps)
    nv = ae.shape[1]
    assert be.shape[1] == nv
    ac, dt = _coef(a_coef)
    bc, dt2 = _coef(b_coef)
    assert dt == dt2, "both factors need the same coefficient type"
    if exact:
        assert dt == 0, "exact products take int64 coefficients"
        dt = 2
    h = lib.oracle_laurent_mul(nv, dt, ae.shape[0], _ptr(ae), _ptr(ac), be.shape[0], _ptr(be),
                               _ptr(bc), row_begin, row_end, threads)
    if not h:
        raise ValueError("oracle_laurent_mul rejected its arguments")
    try:
        n = lib.oracle_laurent_len(h)
        ex = np.empty((n, nv), dtype=np.int32)
        co = (np.empty((n, 2), dtype=np.int64) if dt == 2 else
              np.empty(n, dtype=np.float64 if dt else np.int64))
        ab = np.empty(n, dtype=np.float64) if dt == 1 else None
        lib.oracle_laurent_get(h, _ptr(ex), _ptr(co), _ptr(ab))
    finally:
        lib.oracle_laurent_free(h)
    return ex, co, ab


def laurent_mul_truncated(a_exps, a_coef, b_exps, b_coef, weights, max_degree, threads=1):
    """Truncated product (Section 3: a series multiplier should truncate): the
    terms of A*B whose weighted degree sum_v weights[v] * e_v is at most
    max_degree.  Definition applied literally: the full product, then the
    filter (variables past len(weights) have weight 0).  Same return layout
    as ``laurent_mul``."""
    ex, co, ab = laurent_mul(a_exps, a_coef, b_exps, b_coef, threads=threads)
    w = np.zeros(ex.shape[1], dtype=np.int64)
    w[:min(len(weights), ex.shape[1])] = np.asarray(weights, dtype=np.int64)[:ex.shape[1]]
    keep = ex.astype(np.int64) @ w <= max_degree
    return ex[keep], co[keep], (ab[keep] if ab is not None else None)


def laurent_coeff_at(a_exps, a_coef, b_exps, b_coef, q_exps, exact=False):
    """Coefficient of each queried monomial of A*B, computed one by one.

    Returns ``(coef[q], abs_sum[q] or None, n_contributions[q])``; with
    ``exact=True`` coef is int64[q, 2] as in ``laurent_mul``.
    """
    lib = _load()
    ae, be = _exps(a_exps), _exps(b_exps)
    nv = ae.shape[1]
    qe = _exps(q_exps, nv)
    ac, dt = _coef(a_coef)
    bc, _ = _coef(b_coef)
    if exact:
        assert dt == 0, "exact products take int64 coefficients"
        dt = 2
    nq = qe.shape[0]
    co = (np.empty((nq, 2), dtype=np.int64) if dt == 2 else
          np.empty(nq, dtype=np.float64 if dt else np.int64))
    ab = np.empty(nq, dtype=np.float64) if dt == 1 else None
    cnt = np.empty(nq, dtype=np.int64)
    lib.oracle_laurent_coeff_at(nv, dt, ae.shape[0], _ptr(ae), _ptr(ac), be.shape[0], _ptr(be),
                                _ptr(bc), nq, _ptr(qe), _ptr(co), _ptr(ab), _ptr(cnt))
    return co, ab, cnt


def wide_to_int(words):
    """Python integers of int64[m, 2] (low word, high word) 128-bit values."""
    w = np.asarray(words, dtype=np.int64).reshape(-1, 2)
    return [int(lo) % (1 << 64) + (int(hi) << 64) for lo, hi in w]


def _series(s, nx, ny):
    x, y, t, c = s
    x = np.ascontiguousarray(x, dtype=np.int32).reshape(-1, nx)
    y = np.ascontiguousarray(y, dtype=np.int32).reshape(-1, ny)
    t = np.ascontiguousarray(t, dtype=np.uint8).reshape(-1)
    c = np.ascontiguousarray(c, dtype=np.float64).reshape(-1)
    n = c.shape[0]
    assert x.shape[0] == n and y.shape[0] == n and t.shape[0] == n
    return x, y, t, c


def poisson_mul(a, b, nx, ny, row_begin=0, row_end=-1, threads=1):
    """Product of two Poisson series, each ``(x[n,nx], y[n,ny], is_sin[n], coef[n])``.

    fp64 only.  Returns ``(x, y, is_sin, coef, abs_sum)`` sorted by key, with
    every touched key (including exact zeros) present.
    """
    lib = _load()
    ax, ay, at, ac = _series(a, nx, ny)
    bx, by, bt, bc = _series(b, nx, ny)
    h = lib.oracle_poisson_mul(nx, ny, ac.shape[0], _ptr(ax), _ptr(ay), _ptr(at), _ptr(ac),
                               bc.shape[0], _ptr(bx), _ptr(by), _ptr(bt), _ptr(bc),
                               row_begin, row_end, threads)
    if not h:
        raise ValueError("oracle_poisson_mul rejected its arguments")
    try:
        n = lib.oracle_poisson_len(h)
        x = np.empty((n, nx), dtype=np.int32)
        y = np.empty((n, ny), dtype=np.int32)
        t = np.empty(n, dtype=np.uint8)
        co = np.empty(n, dtype=np.float64)
        ab = np.empty(n, dtype=np.float64)
        lib.oracle_poisson_get(h, _ptr(x), _ptr(y), _ptr(t), _ptr(co), _ptr(ab))
    finally:
        lib.oracle_poisson_free(h)
    return x, y, t, co, ab


def poisson_mul_truncated(a, b, nx, ny, weights, max_order, threads=1):
    """Truncated Poisson product by the order of the Fourier harmonics (one of
    the truncation criteria Section 3 names): the terms of A*B whose weighted
    harmonic order sum_k weights[k] * |j_k| is at most max_order (weights >= 0;
    trigonometric variables past len(weights) have weight 0).  Definition
    applied literally: the full product, then the filter.  Same return layout
    as ``poisson_mul``."""
    x, y, t, co, ab = poisson_mul(a, b, nx, ny, threads=threads)
    w = np.zeros(ny, dtype=np.int64)
    w[:min(len(weights), ny)] = np.asarray(weights, dtype=np.int64)[:ny]
    keep = np.abs(y.astype(np.int64)) @ w <= max_order
    return x[keep], y[keep], t[keep], co[keep], ab[keep]


def poisson_coeff_at(a, b, nx, ny, qx, qy, qt):
    """Coefficient of each queried (x, j, is_sin) term of A*B, one by one."""
    lib = _load()
    ax, ay, at, ac = _series(a, nx, ny)
    bx, by, bt, bc = _series(b, nx, ny)
    qx = np.ascontiguousarray(qx, dtype=np.int32).reshape(-1, nx)
    qy = np.ascontiguousarray(qy, dtype=np.int32).reshape(-1, ny)
    qt = np.ascontiguousarray(qt, dtype=np.uint8).reshape(-1)
    nq = qt.shape[0]
    co = np.empty(nq, dtype=np.float64)
    ab = np.empty(nq, dtype=np.float64)
    cnt = np.empty(nq, dtype=np.int64)
    lib.oracle_poisson_coeff_at(nx, ny, ac.shape[0], _ptr(ax), _ptr(ay), _ptr(at), _ptr(ac),
                                bc.shape[0], _ptr(bx), _ptr(by), _ptr(bt), _ptr(bc), nq,
                                _ptr(qx), _ptr(qy), _ptr(qt), _ptr(co), _ptr(ab), _ptr(cnt))
    return co, ab, cnt


def laurent_eval_modp(exps, coef, point):
    """sum_t coef_t * prod_k point_k^exps_tk  mod 2^61-1 (exact; point_k != 0)."""
    lib = _load()
    ex = _exps(exps, len(point))
    pt = np.ascontiguousarray([int(p) % P61 for p in point], dtype=np.uint64)
    c, dt = _coef(coef)
    f = lib.oracle_laurent_eval_modp_f64 if dt else lib.oracle_laurent_eval_modp_i64
    return int(f(ex.shape[1], ex.shape[0], _ptr(ex), _ptr(c), _ptr(pt)))


def poisson_eval_fp2(series, nx, ny, xpoint, zpoint):
    """Exact value of a Poisson series over F_{p^2}, p = 2^61-1.

    ``xpoint``: nx nonzero residues for the polynomial variables; ``zpoint``:
    ny nonzero elements (re, im) of F_{p^2} standing for exp(i*y_k).  Returns
    (re, im).  Coefficients must be finite doubles (mapped exactly).
    """
    lib = _load()
    x, y, t, c = _series(series, nx, ny)
    xp = np.ascontiguousarray([int(v) % P61 for v in xpoint] or [1], dtype=np.uint64)
    zr = np.ascontiguousarray([int(z[0]) % P61 for z in zpoint] or [1], dtype=np.uint64)
    zi = np.ascontiguousarray([int(z[1]) % P61 for z in zpoint] or [0], dtype=np.uint64)
    out = np.zeros(2, dtype=np.uint64)
    lib.oracle_poisson_eval_fp2(nx, ny, c.shape[0], _ptr(x), _ptr(y), _ptr(t), _ptr(c),
                                _ptr(xp), _ptr(zr), _ptr(zi), _ptr(out))
    return int(out[0]), int(out[1])


def fp2_mul(a, b):
    lib = _load()
    aa = np.ascontiguousarray([a[0] % P61, a[1] % P61], dtype=np.uint64)
    bb = np.ascontiguousarray([b[0] % P61, b[1] % P61], dtype=np.uint64)
    out = np.zeros(2, dtype=np.uint64)
    lib.oracle_fp2_mul(_ptr(aa), _ptr(bb), _ptr(out))
    return int(out[0]), int(out[1])
