"""Autotuner for the knobs the paper leaves open (Sections 3.1, 3.2): the
dense window size, workgroup size and tasks per compute unit, the global
hash table's load factor and rows per thread, the size and fill of the LDS
tables of grouped products, and the density threshold of the dense/hash
choice (Section 3 leaves it to "an analysis of the densities").  None of them
changes a result; each is picked by timing the library's own multiplies on
seeded products of the benchmark shapes.  Results persist in a JSON cache
keyed by the GPU and the library build, so a process on the same machine
applies them without timing again.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time

import numpy as np

from . import (KP_FLAG_ASYNC, Poly, Workspace, context, encode, laurent_layout, mul_bound,
               mul_laurent_codes, _dt)
from . import inputs as I

DENSE_GRID = [dict(window=w, block=b, tasks_per_cu=t)
              for w, b, t in itertools.product((8192, 16384, 18432), (512, 1024), (1, 2))]
HASH_GRID = [dict(hash_load=l, hash_rows=r)
             for l, r in itertools.product((0.35, 0.5, 0.7), (32, 64, 128))]
BIN_GRID = [dict(hash_bin_slots=s, hash_bin_fill=f)
            for s, f in ((2048, 42), (4096, 42), (4096, 55), (8192, 42))]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_1004_4548_amd",
                             "tune.json")


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


class _Product:
    """A product staged for repeated timing: codes, bounds, buffers."""

    def __init__(self, ctx, a, b):
        import torch
        self.ctx = ctx
        self.pa, self.pb = Poly(_dev(a[0]), _dev(a[1])), Poly(_dev(b[0]), _dev(b[1]))
        self.lay = laurent_layout(self.pa, self.pb, ctx)
        self.ka, _ = encode(self.lay, 0, self.pa.exps, ctx=ctx)
        self.kb, _ = encode(self.lay, 1, self.pb.exps, ctx=ctx)
        self.pairs = len(a[1]) * len(b[1])
        self.ws = Workspace()
        self.out = {}

    def feasible(self, mode):
        from . import KPError
        try:
            mul_bound(self.lay, False, _dt(self.pa.coef), mode, self.pa.coef.shape[0],
                      self.pb.coef.shape[0], self.ctx)
            return True
        except KPError:
            return False

    def seconds(self, mode, reps=5):
        import torch
        _, cap, _ = mul_bound(self.lay, False, _dt(self.pa.coef), mode, self.pa.coef.shape[0],
                              self.pb.coef.shape[0], self.ctx)
        if self.out.get(mode) is None or self.out[mode][0].shape[0] < cap:
            self.out[mode] = (torch.empty(max(cap, 1), dtype=torch.int64, device="cuda"),
                              torch.empty(max(cap, 1), dtype=self.pa.coef.dtype, device="cuda"),
                              torch.empty(1, dtype=torch.int64, device="cuda"))
        f = lambda: mul_laurent_codes(self.lay, self.ka, self.pa.coef, self.kb, self.pb.coef,
                                      mode, self.ctx, self.ws, self.out[mode],
                                      flags=KP_FLAG_ASYNC)
        f()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps


def _search(ctx, prod, mode, grid, reps, fixed=None):
    """Times every candidate (with `fixed` settings held while timing, not
    part of the result) and returns the fastest and the table.  `prod` is a
    product or a list of them, a candidate's time being their sum."""
    prods = prod if isinstance(prod, (list, tuple)) else [prod]
    saved = ctx.tune
    base = {f: getattr(saved, f) for f, _ in type(saved)._fields_}
    table = []
    try:
        for cand in grid:
            ctx.set_tune(**{**base, **(fixed or {}), **cand})
            table.append((sum(p.seconds(mode, reps) for p in prods), cand))
    finally:
        ctx.set_tune(**base)
    table.sort(key=lambda x: x[0])
    return table[0][1], table


def tune_dense(ctx, scale=1.0, reps=5):
    """Window, workgroup and tasks per CU on the 4-variable simplex product."""
    a, b = I.config(2, scale=scale)
    return _search(ctx, _Product(ctx, a, b), "dense", DENSE_GRID, reps)


def tune_hash(ctx, scale=0.2, reps=3):
    """Load factor and rows per thread of the global table (forced while
    timing) on the 6-variable sparse product."""
    a, b = I.config(3, scale=scale)
    return _search(ctx, _Product(ctx, a, b), "hash", HASH_GRID, reps,
                   fixed=dict(hash_partitioned=0))


def tune_bins(ctx, scale=0.5, reps=3):
    """Slots and fill of the grouped products' LDS tables (the grouped layout
    forced while timing), one setting for both groupings: timed on the
    6-variable sparse product (grouped by range; the bins are sized from the
    product count, so the product should be of the size it is tuned for) plus
    the Monagan-Pearce product (many products per term: two-level grouping,
    where small tables lose most)."""
    a, b = I.config(3, scale=scale)
    f, g = I.mp_sparse(12, "f"), I.mp_sparse(12, "g")
    prods = [_Product(ctx, a, b), _Product(ctx, f, g)]
    return _search(ctx, prods, "hash", BIN_GRID, reps, fixed=dict(hash_partitioned=2))


def _crossover(rows, fallback):
    """Threshold on codes per term product between the sparsest product where
    dense mode still wins and the densest sparser one where hash wins."""
    dense_wins = [r for r, td, th in rows if td <= th]
    hash_wins = [r for r, td, th in rows if td > th]
    lo = max(dense_wins) if dense_wins else None
    hi = min([r for r in hash_wins if lo is None or r > lo], default=None)
    if lo is None:
        return 0.0
    if hi is None:
        return max(fallback, lo)
    return float(np.sqrt(lo * hi))


def tune_threshold(ctx, n=2000, reps=3, nvars=(2, 3, 4)):
    """The dense/hash switch: products of n x n terms in boxes of growing
    width, for each number of variables in `nvars`; each shape class gives a
    crossover, and the threshold is their median (the library keeps one).
    Returns the threshold and the rows (codes per pair, dense s, hash s, nv)."""
    rows, per_nv = [], {}
    widths = {2: (30, 45, 70, 100, 150, 220, 330, 500, 750, 1100),
              3: (5, 7, 9, 12, 16, 22, 30, 40, 55, 70, 90),
              4: (4, 5, 7, 9, 12, 16, 22, 30)}
    for nv in nvars:
        mine = []
        for h in widths.get(nv, widths[3]):
            if (2 * h + 1) ** nv < n:
                continue
            a = I.laurent_box(nv=nv, n=n, cfg=7, factor=0, lo=-h, hi=h)
            b = I.laurent_box(nv=nv, n=n, cfg=7, factor=1, lo=-h, hi=h)
            prod = _Product(ctx, a, b)
            if not (prod.feasible("dense") and prod.feasible("hash")):
                continue
            td, th = prod.seconds("dense", reps), prod.seconds("hash", reps)
            mine.append((prod.lay.nkeys / prod.pairs, td, th))
        per_nv[nv] = _crossover(mine, ctx.tune.dense_keys_per_pair)
        rows += [(r, td, th, nv) for r, td, th in mine]
    thr = float(np.median(list(per_nv.values()))) if per_nv else ctx.tune.dense_keys_per_pair
    return thr, rows


def cache_key(device_name, library_path, quick):
    """Key of a tuning result: the GPU, the library build (its SHA-256) and
    the tuning depth."""
    h = hashlib.sha256()
    with open(library_path, "rb") as f:
        for chunk in iter(lambda: f.read(1 << 20), b""):
            h.update(chunk)
    return f"{device_name}|{h.hexdigest()[:16]}|{'quick' if quick else 'full'}"


def load_cache(path):
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(path, key, result):
    d = load_cache(path)
    d[key] = result
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(ctx=None, apply=True, quick=True, cache=DEFAULT_CACHE):
    """Tunes every knob and (when `apply`) sets the context to the result.
    With a `cache` path, a result for this GPU and library build is applied
    from it without timing, and a new result is stored there.  Returns the
    chosen settings and the timing tables."""
    import torch
    from . import LIB_PATH
    ctx = ctx or context()
    key = None
    if cache:
        key = cache_key(torch.cuda.get_device_name(ctx.device), LIB_PATH, quick)
        hit = load_cache(cache).get(key)
        if hit and "chosen" in hit:
            if apply:
                ctx.set_tune(**hit["chosen"])
            return {**hit, "cached": True, "cache_key": key}
    dense, dt = tune_dense(ctx, scale=0.5 if quick else 1.0)
    hashed, ht = tune_hash(ctx, scale=0.1 if quick else 0.3)
    bins, bt = tune_bins(ctx, scale=0.5 if quick else 1.0)
    thr, rows = tune_threshold(ctx, n=1000 if quick else 2000)
    chosen = {**dense, **hashed, **bins, "dense_keys_per_pair": thr}
    if apply:
        ctx.set_tune(**chosen)
    out = {"chosen": chosen,
           "dense_ms": [(round(t * 1e3, 4), c) for t, c in dt],
           "hash_ms": [(round(t * 1e3, 4), c) for t, c in ht],
           "bins_ms": [(round(t * 1e3, 4), c) for t, c in bt],
           "threshold_rows": [(round(r, 3), round(a * 1e3, 4), round(b * 1e3, 4), nv)
                              for r, a, b, nv in rows]}
    if cache:
        save_cache(cache, key, out)
    return {**out, "cached": False, "cache_key": key}
