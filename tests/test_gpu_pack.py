"""GPU: packed batches (kp_pack): many whole Laurent products in one fixed
sequence of persistent launches over a device task table, eager and as a
replayed HIP graph, against the oracle.  Each case prints what it runs before
touching the GPU."""
import numpy as np
import pytest

import oracle as O
import paper_1004_4548_amd as kp
from paper_1004_4548_amd import inputs as I
from tests.helpers import assert_exact, assert_tolerance

pytestmark = pytest.mark.gpu
TOL = 1e-13


def say(*a):
    print("[case]", *a, flush=True)


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _check(a, b, r, what):
    exps, coef = r.exps.cpu().numpy(), r.coef.cpu().numpy()
    oe, oc, oab = O.laurent_mul(a[0], a[1], b[0], b[1], threads=4)
    if np.asarray(a[1]).dtype == np.float64:
        assert_tolerance([exps], coef, [oe], oc, oab, TOL, what)
    else:
        assert_exact([exps], coef, [oe], oc, what)


def _cases(seed=0):
    """Products of every kind a pack meets: small key spaces (one word per
    code) and sparse ones (hash table), int64 and fp64, one to six variables,
    ragged and tiny sizes, an empty factor, a single term, sums that cancel."""
    rng = np.random.default_rng(seed)
    out = []
    a, b = I.config(1, scale=0.4)
    out.append(("box int64", a, b))
    a, b = I.config(2, scale=0.05 + 0.01 * seed)
    out.append(("simplex int64", a, b))
    out.append(("simplex fp64", (a[0], a[1].astype(np.float64) / 8),
                (b[0], b[1].astype(np.float64))))
    a, b = I.config(3, scale=0.03)
    out.append(("sparse 6 variables int64 (hash table)", a, b))
    out.append(("sparse fp64 (hash table)", (a[0], a[1].astype(np.float64) * 0.75),
                (b[0], b[1].astype(np.float64))))
    n = 257 + seed
    e = rng.integers(-40, 40, (n, 1)).astype(np.int32)
    out.append(("univariate ragged", (e, rng.integers(-9, 9, n)), (e[:37], rng.integers(1, 5, 37))))
    out.append(("single terms", (np.array([[3, -2]], np.int32), np.array([7])),
                (np.array([[-1, 5]], np.int32), np.array([-6]))))
    out.append(("empty factor", (np.zeros((0, 3), np.int32), np.zeros(0, np.int64)),
                (np.array([[1, 2, 3]], np.int32), np.array([2]))))
    x = np.array([[0, 0], [1, 0]], np.int32)   # (1 + x)(1 - x) = 1 - x^2: the x terms cancel
    out.append(("cancelling", (x, np.array([1, 1])), (x, np.array([1, -1]))))
    return [(w, (np.asarray(a[0], np.int32), np.asarray(a[1])),
             (np.asarray(b[0], np.int32), np.asarray(b[1]))) for w, a, b in out]


def _polys(cases):
    return [(kp.Poly(dev(a[0]), dev(a[1])), kp.Poly(dev(b[0]), dev(b[1]))) for _, a, b in cases]


@pytest.mark.parametrize("graph", [False, True])
def test_pack_matches_oracle(graph):
    cases = _cases()
    say("pack of", len(cases), "products", "graph" if graph else "eager")
    pk = kp.Pack(16)
    pk.launch(_polys(cases), graph=graph)
    res = pk.wait()
    for (what, a, b), r in zip(cases, res):
        say("check", what)
        _check(a, b, r, what)


def test_pack_graph_replays_new_batches():
    """One captured graph, replayed for three different batches with eager
    work and synchronisations between the replays: every replay's products
    are the oracle's."""
    import torch
    pk = kp.Pack(16)
    for rep in range(3):
        cases = _cases(seed=rep)[rep:]   # a different number of products each time
        say("graph replay", rep, len(cases), "products")
        pk.launch(_polys(cases), graph=True)
        res = pk.wait()
        for (what, a, b), r in zip(cases, res):
            _check(a, b, r, f"replay {rep}: {what}")
        # eager work of the program's own between replays
        a, b = I.config(1, scale=0.2)
        kp.mul_laurent(kp.Poly(dev(a[0]), dev(a[1])), kp.Poly(dev(b[0]), dev(b[1])))
        torch.cuda.synchronize()


def test_pack_equals_single_calls_on_the_stream():
    """The first requests of the served stream that fit a pack: the same terms
    as one whole-product call each (int64 exactly, fp64 within the
    tolerance against the oracle)."""
    reqs = [I.request(r) for r in range(40)]
    small = [q for q in reqs if len(q["a"][1]) * len(q["b"][1]) <= 2_000_000][:12]
    say("pack of", len(small), "stream requests")
    prods = [(kp.Poly(dev(q["a"][0]), dev(q["a"][1])), kp.Poly(dev(q["b"][0]), dev(q["b"][1])))
             for q in small]
    pk = kp.Pack(16)
    pk.launch(prods, graph=True)
    res = pk.wait()
    for q, (pa, pb), r in zip(small, prods, res):
        one, _ = kp.mul_laurent(pa, pb)
        what = f"request {q['id']} type {q['type']} {q['dtype']}"
        if q["dtype"] == "f64":
            _check(q["a"], q["b"], r, what)
        else:
            assert_exact([r.exps.cpu().numpy()], r.coef.cpu().numpy(), [one.exps.cpu().numpy()],
                         one.coef.cpu().numpy(), what)


def test_pack_errors():
    """Host-detected errors leave the pack usable."""
    pk = kp.Pack(2)
    cases = _cases()[:3]
    say("pack errors")
    with pytest.raises(kp.KPError) as err:
        pk.launch(_polys(cases))
    assert err.value.status == kp.KP_E_ARG
    a, b = cases[0][1], cases[0][2]
    with pytest.raises(ValueError):
        pk.launch([(kp.Poly(dev(a[0]), dev(a[1])), kp.Poly(dev(b[0]), dev(b[1].astype(np.float64))))])
    pk.launch(_polys(cases[:2]))
    with pytest.raises(kp.KPError):   # one batch at a time
        pk.launch(_polys(cases[:2]))
    res = pk.wait()
    for (what, a, b), r in zip(cases[:2], res):
        _check(a, b, r, what)
