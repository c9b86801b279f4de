"""Shared helpers of the GPU parity tests (comparison of term sets)."""
import numpy as np


def _col2d(c):
    c = np.asarray(c, dtype=np.int64)
    if c.ndim == 1:
        return c.reshape(-1, 1)
    return c.reshape(c.shape[0], int(np.prod(c.shape[1:])))


def rows_key(*cols):
    """One int64 key per row of the integer columns (mixed radix over their ranges)."""
    cols = [_col2d(c) for c in cols]
    full = np.concatenate(cols, axis=1) if cols else np.zeros((0, 0), np.int64)
    return full


def _as_index(full_a, full_b):
    both = np.concatenate([full_a, full_b], axis=0)
    if both.size == 0:
        return np.zeros(len(full_a), np.int64), np.zeros(len(full_b), np.int64)
    lo = both.min(axis=0)
    w = both.max(axis=0) - lo + 1
    key = np.zeros(len(both), dtype=object if np.prod(w.astype(float)) > 2**62 else np.int64)
    mul = 1
    for v in range(both.shape[1]):
        key = key + (both[:, v] - lo[v]) * mul
        mul *= int(w[v])
    return key[:len(full_a)], key[len(full_a):]


def assert_exact(g_cols, g_coef, o_cols, o_coef, what=""):
    """Bit-exact comparison of two term sets (any order, int64 coefficients)."""
    ga, oa = rows_key(*g_cols), rows_key(*o_cols)
    kg, ko = _as_index(ga, oa)
    assert len(kg) == len(set(kg.tolist())), f"{what}: duplicate keys in GPU result"
    assert len(kg) == len(ko), f"{what}: {len(kg)} GPU terms vs {len(ko)} oracle terms"
    ig, io = np.argsort(kg, kind="stable"), np.argsort(ko, kind="stable")
    np.testing.assert_array_equal(kg[ig], ko[io], err_msg=f"{what}: key sets differ")
    np.testing.assert_array_equal(np.asarray(g_coef)[ig], np.asarray(o_coef)[io],
                                  err_msg=f"{what}: coefficients differ")


def assert_tolerance(g_cols, g_coef, o_cols, o_coef, o_abs, tol=1e-13, what=""):
    """fp64 parity: for every key of the union |gpu - oracle| <= tol * sum|contrib|,
    an absent term counting as 0; a GPU key the oracle never touched fails."""
    ga, oa = rows_key(*g_cols), rows_key(*o_cols)
    kg, ko = _as_index(ga, oa)
    assert len(kg) == len(set(kg.tolist())), f"{what}: duplicate keys in GPU result"
    o_map = {k: i for i, k in enumerate(ko.tolist())}
    g_coef = np.asarray(g_coef, dtype=np.float64)
    o_coef = np.asarray(o_coef, dtype=np.float64)
    o_abs = np.asarray(o_abs, dtype=np.float64)
    seen = np.zeros(len(ko), dtype=bool)
    for i, k in enumerate(kg.tolist()):
        j = o_map.get(k)
        assert j is not None, f"{what}: GPU term {ga[i]} has no contribution in the oracle"
        seen[j] = True
        assert abs(g_coef[i] - o_coef[j]) <= tol * o_abs[j], \
            f"{what}: term {ga[i]}: gpu {g_coef[i]!r} oracle {o_coef[j]!r} abs {o_abs[j]!r}"
    missing = ~seen
    assert np.all(np.abs(o_coef[missing]) <= tol * o_abs[missing]), \
        f"{what}: {int(missing.sum())} oracle terms missing from the GPU result"


# ------------------------------------------------------------------ evaluation of large results
P61 = (1 << 61) - 1


def _mulmod61(a, b):
    """a * b mod 2^61 - 1 for int64 tensors with entries in [0, 2^61 - 1),
    in 64-bit integer arithmetic: 31-bit halves, 2^61 = 1 and 2^62 = 2."""
    m31, m30 = (1 << 31) - 1, (1 << 30) - 1
    ah, al = a >> 31, a & m31
    bh, bl = b >> 31, b & m31
    hh = ah * bh                      # < 2^60, weight 2^62
    mid = ah * bl + al * bh           # < 2^62, weight 2^31
    ll = al * bl                      # < 2^62
    ll = (ll & P61) + (ll >> 61)
    r = 2 * hh + (mid >> 30) + ((mid & m30) << 31) + ll   # < 2^63
    r = (r & P61) + (r >> 61)
    r = (r & P61) + (r >> 61)
    return r - P61 * (r >= P61).to(r.dtype)


def eval_modp_device(exps, coef, point, chunk=1 << 26):
    """sum_t coef_t * prod_v point_v^exps_tv  mod 2^61 - 1 of a device result:
    exps int32 [n, nv] (any sign), coef int64 [n] (signed).  Per-variable
    power tables cover each column's range; negative powers use the inverse."""
    import torch
    n, nv = exps.shape
    dev = exps.device
    tables, lows = [], []
    for v in range(nv):
        lo, hi = (int(exps[:, v].min()), int(exps[:, v].max())) if n else (0, 0)
        x = int(point[v]) % P61
        tables.append(torch.tensor([pow(x, e, P61) if e >= 0 else pow(pow(x, P61 - 2, P61), -e, P61)
                                    for e in range(lo, hi + 1)], dtype=torch.int64, device=dev))
        lows.append(lo)
    hi_sum, lo_sum = 0, 0
    for s in range(0, n, chunk):
        c = torch.remainder(coef[s:s + chunk], P61)
        for v in range(nv):
            idx = exps[s:s + chunk, v].to(torch.int64) - lows[v]
            c = _mulmod61(c, tables[v][idx])
        hi_sum += int((c >> 31).sum())
        lo_sum += int((c & ((1 << 31) - 1)).sum())
    return ((hi_sum << 31) + lo_sum) % P61


def eval_mod2_64_device(exps, coef, point, chunk=1 << 26):
    """The same sum in the ring of integers modulo 2^64 (int64 products and
    sums wrap), for exponents >= 0; returned in [0, 2^64)."""
    import torch
    n, nv = exps.shape
    dev = exps.device
    M = 1 << 64
    tables = []
    for v in range(nv):
        hi = int(exps[:, v].max()) if n else 0
        t = [pow(int(point[v]), e, M) for e in range(hi + 1)]
        tables.append(torch.tensor([x - M if x >= 1 << 63 else x for x in t], dtype=torch.int64,
                                   device=dev))
    total = 0
    for s in range(0, n, chunk):
        c = coef[s:s + chunk].clone()
        for v in range(nv):
            c = c * tables[v][exps[s:s + chunk, v].to(torch.int64)]
        total += int(c.sum())
    return total % M


def parallel_chunks(fn, items, workers=None, parts=64):
    """fn over contiguous chunks of `items` (numpy arrays, first axis) on host
    threads (the oracle's ctypes calls release the GIL); results in order."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    n = len(items[0])
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    bounds = np.linspace(0, n, min(parts, max(n, 1)) + 1).astype(int)
    with ThreadPoolExecutor(workers) as ex:
        futs = [ex.submit(fn, *[it[b0:b1] for it in items])
                for b0, b1 in zip(bounds[:-1], bounds[1:]) if b1 > b0]
        return [f.result() for f in futs]


def adversarial_codes(slots, coef=None):
    """Univariate factors whose product codes, under the two-level hash
    grouping (code times the 64-bit golden-ratio constant), all have their top
    three bits zero: slots + 1000 distinct codes in the first of at most 4
    bins.  A is those exponents (and 0) with coefficients `coef` (ones by
    default), B the constant 1."""
    rng = np.random.default_rng(slots)
    e = np.unique(rng.integers(1, 1 << 31, 1 << 20, dtype=np.int64))
    with np.errstate(over="ignore"):
        h = e.astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    e = e[(h >> np.uint64(61)) == 0][: slots + 999]
    assert len(e) == slots + 999
    c = np.ones(slots + 1000, np.int64) if coef is None else np.asarray(coef, np.int64)
    a = (np.concatenate([[0], e]).astype(np.int32).reshape(-1, 1), c)
    b = (np.zeros((1, 1), np.int32), np.ones(1, np.int64))
    return a, b
