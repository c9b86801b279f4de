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
