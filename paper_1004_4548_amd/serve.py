"""Serving a stream of product requests on one GPU: per-call and batched
execution, closed-loop capacity, and open-loop latency (p50/p99).

A request is a Laurent product given as exponents and coefficients resident
on the device.  Per call, every request runs the whole path alone: min/max of
both factors (one host read), layout, encode, multiply (one host read of the
count), decode.  Batched, a group of requests shares those host reads: one
min/max pass for all factors, encodes queued back to back, all products
queued through one kp_batch launch, one read of all counts, decodes queued,
one synchronisation at the end.  Both orders compute the same products.

Continuous batching: requests arrive at the times of a Poisson process.
Whenever a stream slot is free, the server admits the requests that have
arrived (up to a batch size, and as far as the device memory budget allows,
estimated from each product's output bound and workspace) as one batch on
that slot's stream, without waiting for the batches already on the device:
up to `slots` batches overlap.  A batch completes when its decodes are done;
the latency of a request is its completion time minus its arrival time.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import (KP_FLAG_ASYNC, Batch, Poly, context, decode, encode, layout_product, mul_bound,
               mul_laurent, _boxes, _dt)


@dataclass
class Staged:
    """One request with both factors on the device."""
    rid: int
    a: Poly
    b: Poly
    pairs: int
    meta: dict = field(default_factory=dict)


def stage(requests, device="cuda"):
    """Copy request factors to the device (outside any timed region)."""
    import torch
    out = []
    for r in requests:
        (ea, ca), (eb, cb) = r["a"], r["b"]
        dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(device)
        out.append(Staged(r["id"], Poly(dev(ea), dev(ca)), Poly(dev(eb), dev(cb)),
                          len(ca) * len(cb), {k: r[k] for k in ("type", "nv", "dtype")}))
    return out


def run_per_call(staged, ctx=None):
    """Each request alone, in order; returns (results, seconds per request)."""
    import torch
    ctx = ctx or context()
    res, lat = [], []
    for s in staged:
        t = time.perf_counter()
        p, _ = mul_laurent(s.a, s.b, ctx=ctx)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t)
        res.append(p)
    return res, lat


def _align(n):
    return (n + 255) & ~255


def plan_batch(staged, ctx):
    """Layouts, bounds and buffer sizes of a group of requests (one host read
    of all factor boxes)."""
    vals = []
    for s in staged:
        vals += [s.a.exps, s.b.exps]
    boxes = _boxes(ctx, *vals)
    plans = []
    for i, s in enumerate(staged):
        (amin, amax), (bmin, bmax) = boxes[2 * i], boxes[2 * i + 1]
        lay = layout_product(s.a.nv, 0, amin, amax, bmin, bmax)
        mode, max_out, ws = mul_bound(lay, False, _dt(s.a.coef), "auto", s.a.coef.shape[0],
                                      s.b.coef.shape[0], ctx)
        plans.append((lay, mode, max(max_out, 1), ws))
    return plans


def batch_bytes(staged, plans):
    """Device bytes a batch allocates (workspaces and outputs)."""
    tot = 0
    for s, (lay, mode, cap, ws) in zip(staged, plans):
        tot += _align(ws) + 2 * _align(8 * cap) + _align(4 * s.a.nv * cap)
    return tot


def run_batch(staged, ctx=None, plans=None, graph=False, batch=None):
    """One group of requests through the batched path; returns the products."""
    import torch
    ctx = ctx or context()
    if plans is None:
        plans = plan_batch(staged, ctx)
    dev = staged[0].a.exps.device
    counts = torch.empty(len(staged), dtype=torch.int64, device=dev)
    bt = batch or Batch(len(staged), ctx)
    outs = []
    for i, (s, (lay, mode, cap, ws)) in enumerate(zip(staged, plans)):
        ka, _ = encode(lay, 0, s.a.exps, ctx=ctx, flags=KP_FLAG_ASYNC)
        kb, _ = encode(lay, 1, s.b.exps, ctx=ctx, flags=KP_FLAG_ASYNC)
        oc = torch.empty(cap, dtype=torch.int64, device=dev)
        ov = torch.empty(cap, dtype=s.a.coef.dtype, device=dev)
        wbuf = torch.empty(max(ws, 256), dtype=torch.uint8, device=dev)
        bt.add_laurent(lay, ka, s.a.coef, kb, s.b.coef, (oc, ov, counts[i:i + 1]), wbuf)
        outs.append((lay, oc, ov))
    bt.launch(graph=graph)
    n = counts.cpu().tolist()   # the one read of all counts
    res = []
    for (lay, oc, ov), k in zip(outs, n):
        if k < 0:
            ctx.sync_check()
            raise RuntimeError(f"request failed with status {-k}")
        res.append(Poly(decode(lay, oc[:k], ctx=ctx, flags=KP_FLAG_ASYNC), ov[:k]))
    torch.cuda.synchronize()
    if batch is None:
        del bt
    return res


def groups(staged, plans, max_batch, max_bytes):
    """Consecutive groups of at most max_batch requests and max_bytes."""
    out, cur, cur_plans, used = [], [], [], 0
    for s, p in zip(staged, plans):
        need = batch_bytes([s], [p])
        if cur and (len(cur) == max_batch or used + need > max_bytes):
            out.append((cur, cur_plans))
            cur, cur_plans, used = [], [], 0
        cur.append(s)
        cur_plans.append(p)
        used += need
    if cur:
        out.append((cur, cur_plans))
    return out


class InFlight:
    """A batch on its own stream: multiplies queued, counts on their way to
    pinned host memory; then decodes queued; then done."""

    def __init__(self, staged, plans, stream, ctx):
        import torch
        self.staged, self.stream, self.ctx = staged, stream, ctx
        self.bytes = batch_bytes(staged, plans)
        self.results = None
        dev = staged[0].a.exps.device
        with torch.cuda.stream(stream):
            counts = torch.empty(len(staged), dtype=torch.int64, device=dev)
            self.batch = Batch(len(staged), ctx)
            self.outs = []
            for i, (s, (lay, mode, cap, ws)) in enumerate(zip(staged, plans)):
                ka, _ = encode(lay, 0, s.a.exps, ctx=ctx, flags=KP_FLAG_ASYNC)
                kb, _ = encode(lay, 1, s.b.exps, ctx=ctx, flags=KP_FLAG_ASYNC)
                oc = torch.empty(cap, dtype=torch.int64, device=dev)
                ov = torch.empty(cap, dtype=s.a.coef.dtype, device=dev)
                wbuf = torch.empty(max(ws, 256), dtype=torch.uint8, device=dev)
                self.batch.add_laurent(lay, ka, s.a.coef, kb, s.b.coef,
                                       (oc, ov, counts[i:i + 1]), wbuf)
                self.outs.append((lay, oc, ov))
            self.batch.launch()
            self.counts = torch.empty(len(staged), dtype=torch.int64, pin_memory=True)
            self.counts.copy_(counts, non_blocking=True)
            self.ev = torch.cuda.Event()
            self.ev.record(stream)
        self.phase = 0

    def advance(self):
        """Moves the batch on when its stream has caught up; True when done."""
        import torch
        if not self.ev.query():
            return False
        if self.phase == 0:
            n = self.counts.tolist()
            res = []
            with torch.cuda.stream(self.stream):
                for (lay, oc, ov), k in zip(self.outs, n):
                    if k < 0:
                        self.ctx.sync_check()
                        raise RuntimeError(f"request failed with status {-k}")
                    res.append(Poly(decode(lay, oc[:k], ctx=self.ctx, flags=KP_FLAG_ASYNC),
                                    ov[:k]))
                self.ev = torch.cuda.Event()
                self.ev.record(self.stream)
            self.results = res
            self.batch = None
            self.phase = 1
            return False
        return True


def _plan_on(staged, ctx, stream):
    import torch
    with torch.cuda.stream(stream):
        return plan_batch(staged, ctx)


def serve_stream(staged, arrivals, ctx=None, max_batch=16, max_bytes=48 << 30, slots=3):
    """Continuous batching: requests arriving at `arrivals` (seconds from
    start) are admitted as soon as a stream slot and memory allow, while
    earlier batches are still running; up to `slots` batches overlap on the
    device.  Returns (latencies, completion order, results, wall time)."""
    import torch
    ctx = ctx or context()
    streams = [torch.cuda.Stream() for _ in range(slots)]
    free = list(range(slots))
    inflight = []   # (InFlight, slot, first, last)
    lat = np.zeros(len(staged))
    results = [None] * len(staged)
    used = 0
    nxt = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while nxt < len(staged) or inflight:
        now = time.perf_counter() - t0
        for item in list(inflight):
            f, slot, i0, i1 = item
            if f.advance():
                done = time.perf_counter() - t0
                lat[i0:i1] = done - arrivals[i0:i1]
                results[i0:i1] = f.results
                used -= f.bytes
                free.append(slot)
                inflight.remove(item)
        admitted = False
        if free and nxt < len(staged) and arrivals[nxt] <= now:
            end = nxt
            while end < len(staged) and end - nxt < max_batch and arrivals[end] <= now:
                end += 1
            slot = free[0]
            plans = _plan_on(staged[nxt:end], ctx, streams[slot])
            # admit the longest prefix that fits the memory left (at least one
            # request when nothing else is in flight)
            take, need = 0, 0
            for s, p in zip(staged[nxt:end], plans):
                b = batch_bytes([s], [p])
                if take and used + need + b > max_bytes:
                    break
                if not take and inflight and used + b > max_bytes:
                    break
                take += 1
                need += b
            if take:
                free.pop(0)
                f = InFlight(staged[nxt:nxt + take], plans[:take], streams[slot], ctx)
                used += f.bytes
                inflight.append((f, slot, nxt, nxt + take))
                nxt += take
                admitted = True
        if not admitted and inflight:
            time.sleep(0)   # let the device catch up
        elif not admitted and nxt < len(staged):
            wait = arrivals[nxt] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.0005))
    torch.cuda.synchronize()
    return lat, results, time.perf_counter() - t0


def closed_loop(staged, ctx=None, max_batch=16, max_bytes=48 << 30, slots=3):
    """Batched capacity: every request available at once; seconds."""
    _, _, wall = serve_stream(staged, np.zeros(len(staged)), ctx, max_batch, max_bytes, slots)
    return wall


def open_loop(staged, rate, ctx=None, max_batch=16, max_bytes=48 << 30, slots=3,
              seed=10044548):
    """Continuous batching under Poisson arrivals at `rate` requests/s.
    Returns per-request latencies (s) and the wall time."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(staged)))
    lat, _, wall = serve_stream(staged, arrivals, ctx, max_batch, max_bytes, slots)
    return lat, wall


def percentiles(lat):
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(np.mean(lat) * 1e3)}
