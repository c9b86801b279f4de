"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws terms (exponent tuples, trigonometric multipliers,
cos/sin flags, coefficients).  It holds none of the multiplication's
arithmetic, imports neither the GPU binding nor the oracle, and every array
it returns is plain numpy on the host.

Workloads (the paper's Section 5 benchmarks are closed forms and can be
regenerated exactly; the seeded families below stand in for their shapes):

* ``laurent_box``       -- distinct tuples drawn without replacement from a
                           box (3 variables in [-5, 5]: the 500 x 500 case);
* ``laurent_simplex``   -- distinct tuples from the simplex e >= 0, sum e <= D
                           (4 variables, D = 20, 10,000 terms: the moderately
                           sparse case standing in for Fateman's benchmark);
* ``laurent_sparse``    -- distinct uniform tuples in [0, R]^nv (6 variables,
                           R = 80, 30,000 terms: the highly sparse case
                           standing in for the Monagan-Pearce benchmark);
* ``poisson_random``    -- canonical Poisson terms (3 polynomial variables in
                           [-4, 4], 6 trigonometric multipliers in [-8, 8],
                           half cos and half sin, coefficients
                           N(0,1) * 2^-sum|j|: standing in for ELP3^3, whose
                           data is not available);
* ``fateman`` / ``mp_sparse`` -- the exact factors of Section 5's benchmarks,
                           for any power k;
* ``stream_requests``   -- the mixed request stream of the batching/serving
                           measurements.

Seeds follow ``SeedSequence([10044548, config, factor])``.
"""
from __future__ import annotations

import math
from itertools import product as _iproduct

import numpy as np

SEED_ROOT = 10044548


def rng_for(cfg: int, factor: int, extra: int | None = None) -> np.random.Generator:
    words = [SEED_ROOT, int(cfg), int(factor)]
    if extra is not None:
        words.append(int(extra))
    return np.random.default_rng(np.random.SeedSequence(words))


def _nonzero_ints(rng, lo, hi, n):
    c = rng.integers(lo, hi + 1, size=n, dtype=np.int64)
    while True:
        z = c == 0
        if not z.any():
            return c
        c[z] = rng.integers(lo, hi + 1, size=int(z.sum()), dtype=np.int64)


def _coef(rng, n, kind, lo, hi):
    if kind == "i64":
        return _nonzero_ints(rng, lo, hi, n)
    if kind == "f64":
        return rng.standard_normal(n)
    if kind == "f64int":          # integer-valued doubles: every sum is exact
        return _nonzero_ints(rng, lo, hi, n).astype(np.float64)
    raise ValueError(kind)


def _distinct_uniform(rng, nv, n, lo, hi):
    """n distinct tuples, uniform in [lo, hi]^nv (rejection of duplicates)."""
    width = hi - lo + 1
    if width ** nv < n:
        raise ValueError("box too small for n distinct tuples")
    if width ** nv <= 4 * n or width ** nv <= 1 << 22:
        flat = rng.choice(width ** nv, size=n, replace=False)
        e = np.empty((n, nv), dtype=np.int64)
        for v in range(nv):
            e[:, v] = flat % width
            flat = flat // width
        return (e + lo).astype(np.int32)
    seen = set()
    rows = []
    while len(rows) < n:
        cand = rng.integers(lo, hi + 1, size=(2 * (n - len(rows)) + 16, nv))
        for r in map(tuple, cand):
            if r not in seen:
                seen.add(r)
                rows.append(r)
                if len(rows) == n:
                    break
    return np.asarray(rows, dtype=np.int32)


def laurent_box(nv=3, n=500, lo=-5, hi=5, coef="i64", clo=-100, chi=100, cfg=1, factor=0):
    rng = rng_for(cfg, factor)
    e = _distinct_uniform(rng, nv, n, lo, hi)
    return e, _coef(rng, n, coef, clo, chi)


def simplex_points(nv, deg):
    """All e >= 0 with sum(e) <= deg, in lexicographic order."""
    pts = [p for p in _iproduct(range(deg + 1), repeat=nv) if sum(p) <= deg]
    return np.asarray(pts, dtype=np.int32).reshape(-1, nv)


def laurent_simplex(nv=4, n=10000, deg=20, coef="i64", clo=1, chi=1000, cfg=2, factor=0):
    rng = rng_for(cfg, factor)
    pts = simplex_points(nv, deg)
    if n > len(pts):
        raise ValueError("simplex has fewer points than requested")
    idx = rng.choice(len(pts), size=n, replace=False)
    return pts[idx].copy(), _coef(rng, n, coef, clo, chi)


def laurent_sparse(nv=6, n=30000, hi=80, coef="i64", clo=-1000, chi=1000, cfg=3, factor=0):
    rng = rng_for(cfg, factor)
    e = _distinct_uniform(rng, nv, n, 0, hi)
    return e, _coef(rng, n, coef, clo, chi)


def poisson_random(nx=3, ny=6, n=5000, xlo=-4, xhi=4, jmax=8, coef="f64", clo=-1000, chi=1000,
                   cfg=4, factor=0, scale_by_harmonic=True):
    """Canonical Poisson terms: half cos then half sin, distinct (x, j, t).

    Canonical means the first nonzero trigonometric multiplier is positive;
    sin with the zero multiplier vector is redrawn.
    """
    rng = rng_for(cfg, factor)
    seen = set()
    xs, ys, ts = [], [], []
    for t, count in ((0, n // 2), (1, n - n // 2)):
        got = 0
        while got < count:
            x = rng.integers(xlo, xhi + 1, size=nx)
            j = rng.integers(-jmax, jmax + 1, size=ny)
            nz = np.flatnonzero(j)
            if len(nz) == 0:
                if t == 1:
                    continue
            elif j[nz[0]] < 0:
                j = -j
            key = (tuple(x.tolist()), tuple(j.tolist()), t)
            if key in seen:
                continue
            seen.add(key)
            xs.append(x)
            ys.append(j)
            ts.append(t)
            got += 1
    x = np.asarray(xs, dtype=np.int32).reshape(n, nx)
    y = np.asarray(ys, dtype=np.int32).reshape(n, ny)
    s = np.asarray(ts, dtype=np.uint8)
    c = _coef(rng, n, coef, clo, chi).astype(np.float64)
    if scale_by_harmonic and coef == "f64":
        c = np.ldexp(c, -np.abs(y).sum(axis=1).astype(np.int32))
    return x, y, s, c


# ------------------------------------------------- Section 5 closed forms
def _compositions(total, parts):
    """All tuples of `parts` non-negative ints with sum <= total."""
    if parts == 0:
        yield ()
        return
    for first in range(total + 1):
        for rest in _compositions(total - first, parts - 1):
            yield (first,) + rest


def multinomial(k, powers):
    rem = k - sum(powers)
    out = math.factorial(k) // math.factorial(rem)
    for p in powers:
        out //= math.factorial(p)
    return out


def fateman(k=30, plus_one=False, dtype="i64"):
    """Terms of f = (1 + x + y + z + t)^k (or f + 1), by the multinomial theorem.

    Coefficients are returned as Python-exact int64 when they fit (k <= 30
    does) or as float64 when dtype='f64'.
    """
    exps, coefs = [], []
    for p in _compositions(k, 4):
        exps.append(p)
        c = multinomial(k, p)
        if plus_one and sum(p) == 0:
            c += 1
        coefs.append(c)
    e = np.asarray(exps, dtype=np.int32).reshape(-1, 4)
    if dtype == "f64":
        return e, np.asarray([float(c) for c in coefs], dtype=np.float64)
    return e, np.asarray(coefs, dtype=np.int64)


def mp_sparse(k=12, which="f", dtype="i64"):
    """Terms of (1 + x + y + 2z^2 + 3t^3 + 5u^5)^k ("f") or
    (1 + u + t + 2z^2 + 3y^3 + 5x^5)^k ("g"); variables ordered (x, y, z, t, u)."""
    if which == "f":
        atoms = [(0, 1, 1), (1, 1, 1), (2, 2, 2), (3, 3, 3), (4, 5, 5)]   # (var, exp, mult)
    else:
        atoms = [(4, 1, 1), (3, 1, 1), (2, 2, 2), (1, 3, 3), (0, 5, 5)]
    exps, coefs = [], []
    for p in _compositions(k, 5):
        e = [0] * 5
        c = multinomial(k, p)
        for (var, ex, mul), pw in zip(atoms, p):
            e[var] += ex * pw
            c *= mul ** pw
        exps.append(e)
        coefs.append(c)
    e = np.asarray(exps, dtype=np.int32).reshape(-1, 5)
    if dtype == "f64":
        return e, np.asarray([float(c) for c in coefs], dtype=np.float64)
    return e, np.asarray(coefs, dtype=np.int64)


# ------------------------------------------------------ benchmark configs
def config(cfg: int, dtype: str | None = None, scale: float = 1.0):
    """Factors (A, B) of a numbered configuration; ``scale`` shrinks n."""
    if cfg == 1:
        n = max(1, int(round(500 * scale)))
        kw = dict(coef=dtype or "i64")
        return (laurent_box(n=n, cfg=1, factor=0, **kw), laurent_box(n=n, cfg=1, factor=1, **kw))
    if cfg == 2:
        n = max(1, int(round(10000 * scale)))
        kw = dict(coef=dtype or "i64")
        return (laurent_simplex(n=n, cfg=2, factor=0, **kw),
                laurent_simplex(n=n, cfg=2, factor=1, **kw))
    if cfg == 3:
        n = max(1, int(round(30000 * scale)))
        kw = dict(coef=dtype or "i64")
        return (laurent_sparse(n=n, cfg=3, factor=0, **kw),
                laurent_sparse(n=n, cfg=3, factor=1, **kw))
    if cfg == 4:
        n = max(2, int(round(5000 * scale)))
        kw = dict(coef=dtype or "f64")
        return (poisson_random(n=n, cfg=4, factor=0, **kw),
                poisson_random(n=n, cfg=4, factor=1, **kw))
    raise ValueError(cfg)


def stream_requests(count=2000, seed_cfg=5):
    """Mixed request stream: per request a type in {1,2,3}, 2..6 variables,
    factor sizes log-uniform in [50, 20000], int64 or fp64 coefficients.
    Boxes widen with n so each type keeps its base density.  Returns a list of
    dicts with the two factors and metadata; generation is lazy per request
    through ``request(r)`` to keep memory small."""
    return [request(r, seed_cfg) for r in range(count)]


def request(r: int, seed_cfg: int = 5):
    rng = rng_for(seed_cfg, 0, r)
    typ = int(rng.integers(1, 4))
    nv = int(rng.integers(2, 7))
    n1 = int(round(math.exp(rng.uniform(math.log(50), math.log(20000)))))
    n2 = int(round(math.exp(rng.uniform(math.log(50), math.log(20000)))))
    dt = "i64" if rng.random() < 0.5 else "f64"
    n = max(n1, n2)
    seeds = [int(s) for s in rng.integers(0, 2**31, size=2)]
    if typ == 1:
        h = max(5, math.ceil(((n / 0.376) ** (1.0 / nv) - 1) / 2))
        fa = _box_factor(seeds[0], nv, n1, -h, h, dt, -100, 100)
        fb = _box_factor(seeds[1], nv, n2, -h, h, dt, -100, 100)
    elif typ == 2:
        d = 0
        while math.comb(d + nv, nv) < n / 0.941:
            d += 1
        fa = _simplex_factor(seeds[0], nv, n1, d, dt)
        fb = _simplex_factor(seeds[1], nv, n2, d, dt)
    else:
        rr = max(80, math.ceil((n / 1.06e-7) ** (1.0 / nv)) - 1)
        fa = _box_factor(seeds[0], nv, n1, 0, rr, dt, -1000, 1000)
        fb = _box_factor(seeds[1], nv, n2, 0, rr, dt, -1000, 1000)
    return dict(id=r, type=typ, nv=nv, dtype=dt, a=fa, b=fb)


def _box_factor(seed, nv, n, lo, hi, dt, clo, chi):
    rng = np.random.default_rng(seed)
    e = _distinct_uniform(rng, nv, n, lo, hi)
    return e, _coef(rng, n, dt, clo, chi)


def _simplex_factor(seed, nv, n, deg, dt):
    rng = np.random.default_rng(seed)
    total = math.comb(deg + nv, nv)
    if total <= 4_000_000:
        pts = simplex_points(nv, deg)
        idx = rng.choice(len(pts), size=n, replace=False)
        e = pts[idx].copy()
    else:
        seen, rows = set(), []
        while len(rows) < n:
            c = rng.integers(0, deg + 1, size=(4 * n, nv))
            c = c[c.sum(axis=1) <= deg]
            for r in map(tuple, c):
                if r not in seen:
                    seen.add(r)
                    rows.append(r)
                    if len(rows) == n:
                        break
        e = np.asarray(rows, dtype=np.int32)
    return e, _coef(rng, n, dt, 1, 1000)
