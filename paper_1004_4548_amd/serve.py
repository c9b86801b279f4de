"""Serving a stream of product requests on one GPU: per-call and batched
execution, closed-loop capacity, and open-loop latency (p50/p99).

A request is a Laurent product given as exponents and coefficients resident
on the device.  Per call, every request runs the whole path alone: min/max of
both factors (one host read), layout, encode, multiply (one host read of the
count), decode.  Batched, a group of requests shares those host reads: one
min/max pass for all factors, encodes queued back to back, all products
queued through one kp_batch launch, one read of all counts, decodes queued,
one synchronisation at the end.  Both orders compute the same products.

Products of at most `pack_pairs` term pairs (most of the stream) go into a
kp_pack: one host wait for all their factor boxes, then a fixed sequence of
persistent launches over a device task table, replayed from a HIP graph that
is captured once per stream slot, and one wait for all their counts.  Larger
products take the per-product kernels through kp_batch in the same batch.

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

from . import (KP_FLAG_ASYNC, Batch, Pack, Poly, context, decode, encode, layout_product,
               mul_bound, mul_laurent, _boxes, _dt)

# products of at most this many term pairs are computed in a pack
PACK_PAIRS = 1 << 22


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


def run_per_call(staged, ctx=None, keep=True):
    """Each request alone, in order; returns (results, seconds per request).
    keep=False drops each result once it is complete (a stream's results
    need not fit the device together)."""
    import torch
    ctx = ctx or context()
    res, lat = [], []
    for s in staged:
        t = time.perf_counter()
        p, _ = mul_laurent(s.a, s.b, ctx=ctx)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t)
        res.append(p if keep else None)
    return res, lat


def _align(n):
    return (n + 255) & ~255


def plan_batch(staged, ctx):
    """Layouts, bounds and buffer sizes of a group of requests (one host read
    of all factor boxes)."""
    if not staged:
        return []
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
    """Device bytes a batch allocates (workspaces and outputs) for products
    planned one by one."""
    tot = 0
    for s, (lay, mode, cap, ws) in zip(staged, plans):
        tot += _align(ws) + 2 * _align(8 * cap) + _align(4 * s.a.nv * cap)
    return tot


def pack_bytes(s):
    """A bound on the device bytes of one product in a pack: its result
    (at most one term per pair: exponents and coefficient), codes and
    accumulator (at most 8 words per result term: a hash table of up to four
    times the bound, two words a slot, or one word per code up to twice that
    many slots)."""
    na, nb = s.a.coef.shape[0], s.b.coef.shape[0]
    return _align(s.pairs * (4 * s.a.nv + 8 + 64)) + _align(8 * (na + nb)) + 4096


class SlotMemory:
    """Device memory of one stream slot, reused by its batches: every batch
    carves its buffers from one allocation, replaced by a larger one only when
    a batch needs more (a stream of products of very uneven sizes would
    otherwise fragment the allocator's cache).  Views are valid until the
    slot's next batch."""

    def __init__(self, device, nbytes=0):
        import torch
        self.device, self.off = device, 0
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device) if nbytes else None

    def ensure(self, nbytes):
        import torch
        if self.buf is None or self.buf.numel() < nbytes:
            old = 0 if self.buf is None else self.buf.numel()
            self.buf = None
            self.buf = torch.empty(max(nbytes + (nbytes >> 2), 2 * old) + (64 << 20),
                                   dtype=torch.uint8, device=self.device)
        self.off = 0

    def take(self, n, dtype):
        import torch
        nbytes = _align(n * torch.empty((), dtype=dtype).element_size())
        if self.off + nbytes > self.buf.numel():
            raise RuntimeError("slot memory: the batch needs more than it planned")
        v = self.buf[self.off:self.off + nbytes].view(dtype)[:n]
        self.off += nbytes
        return v


def split(staged, pack_pairs):
    """Indices of the requests computed in a pack and of the others."""
    small = [i for i, s in enumerate(staged) if s.pairs <= pack_pairs]
    large = [i for i, s in enumerate(staged) if s.pairs > pack_pairs]
    return small, large


def request_bytes(s, plan, pack_pairs):
    return pack_bytes(s) if s.pairs <= pack_pairs else batch_bytes([s], [plan])


class InFlight:
    """A batch on its own stream: the small products in the slot's pack, the
    others through kp_batch, their counts on the way to pinned host memory;
    then the large products' decodes; then done."""

    def __init__(self, staged, plans, stream, ctx, pack, pack_pairs=PACK_PAIRS, graph=True,
                 mem=None):
        import torch
        self.staged, self.stream, self.ctx, self.pack, self.mem = staged, stream, ctx, pack, mem
        self.small, self.large = split(staged, pack_pairs)
        self.bytes = sum(request_bytes(s, p, pack_pairs) for s, p in zip(staged, plans))
        self.results = None
        dev = staged[0].a.exps.device
        new = self._new = (mem.take if mem is not None else
                           (lambda n_, dt: torch.empty(n_, dtype=dt, device=dev)))
        with torch.cuda.stream(stream):
            need = 0
            if self.small:
                _, need = pack.plan([(staged[i].a, staged[i].b) for i in self.small],
                                    graph=graph, stream=stream)
            if mem is not None:
                for i in self.large:
                    s, (lay, mode, cap, ws) = staged[i], plans[i]
                    need += (2 * _align(8 * cap) + _align(max(ws, 256)) +
                             _align(4 * lay.nx * cap))
                mem.ensure(need)
            if self.small:
                pack.run(alloc=mem.take if mem is not None else None)
            self.outs = []
            if self.large:
                counts = torch.empty(len(self.large), dtype=torch.int64, device=dev)
                self.batch = Batch(len(self.large), ctx)
                for j, i in enumerate(self.large):
                    s, (lay, mode, cap, ws) = staged[i], plans[i]
                    ka, _ = encode(lay, 0, s.a.exps, ctx=ctx, flags=KP_FLAG_ASYNC)
                    kb, _ = encode(lay, 1, s.b.exps, ctx=ctx, flags=KP_FLAG_ASYNC)
                    oc = new(cap, torch.int64)
                    ov = new(cap, s.a.coef.dtype)
                    wbuf = new(max(ws, 256), torch.uint8)
                    self.batch.add_laurent(lay, ka, s.a.coef, kb, s.b.coef,
                                           (oc, ov, counts[j:j + 1]), wbuf)
                    self.outs.append((lay, oc, ov))
                self.batch.launch()
                self.counts = torch.empty(len(self.large), dtype=torch.int64, pin_memory=True)
                self.counts.copy_(counts, non_blocking=True)
            self.ev = torch.cuda.Event()
            self.ev.record(stream)
        self.phase = 0

    def advance(self):
        """Moves the batch on when its stream has caught up; True when done."""
        import torch
        if not self.ev.query() or (self.small and not self.pack.ready()):
            return False
        if self.phase == 0:
            res = [None] * len(self.staged)
            if self.small:
                for i, r in zip(self.small, self.pack.wait()):
                    res[i] = r
            if self.large:
                n = self.counts.tolist()
                with torch.cuda.stream(self.stream):
                    for i, (lay, oc, ov), k in zip(self.large, self.outs, n):
                        if k < 0:
                            self.ctx.sync_check()
                            raise RuntimeError(f"request failed with status {-k}")
                        x = self._new(k * lay.nx, torch.int32).view(k, lay.nx)
                        res[i] = Poly(decode(lay, oc[:k], ctx=self.ctx, flags=KP_FLAG_ASYNC,
                                             out=x), ov[:k])
                    self.ev = torch.cuda.Event()
                    self.ev.record(self.stream)
                self.batch = None
            self.results = res
            self.phase = 1
            return False
        return True


def run_batch(staged, ctx=None, pack_pairs=PACK_PAIRS, graph=True):
    """One group of requests through the batched path; returns the products."""
    import torch
    ctx = ctx or context()
    small, large = split(staged, pack_pairs)
    plans = [None] * len(staged)
    for i, p in zip(large, plan_batch([staged[i] for i in large], ctx)):
        plans[i] = p
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    f = InFlight(staged, plans, stream, ctx, Pack(max(len(small), 1), ctx), pack_pairs, graph)
    while not f.advance():
        pass
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    return f.results


def groups(staged, plans, max_batch, max_bytes, pack_pairs=PACK_PAIRS):
    """Consecutive groups of at most max_batch requests and max_bytes."""
    out, cur, cur_plans, used = [], [], [], 0
    for s, p in zip(staged, plans):
        need = request_bytes(s, p, pack_pairs)
        if cur and (len(cur) == max_batch or used + need > max_bytes):
            out.append((cur, cur_plans))
            cur, cur_plans, used = [], [], 0
        cur.append(s)
        cur_plans.append(p)
        used += need
    if cur:
        out.append((cur, cur_plans))
    return out


def _plan_on(staged, ctx, stream, pack_pairs=PACK_PAIRS):
    """Plans of the requests that do not go into a pack (None for the others)."""
    import torch
    _, large = split(staged, pack_pairs)
    plans = [None] * len(staged)
    with torch.cuda.stream(stream):
        for i, p in zip(large, plan_batch([staged[i] for i in large], ctx)):
            plans[i] = p
    return plans


class Server:
    """The resources of a serving loop, kept from one run to the next: a
    stream, a pack (its graph captured at the slot's first batch) and a
    reusable device buffer per slot (allocating and freeing device memory
    takes far longer than most products)."""

    def __init__(self, slots=3, max_batch=16, ctx=None, device=None, slot_bytes=24 << 30):
        import torch
        self.ctx = ctx or context()
        self.max_batch = max_batch
        self.slot_bytes = slot_bytes
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.packs = [Pack(max_batch, self.ctx) for _ in range(slots)]
        dev = device or torch.device("cuda", torch.cuda.current_device())
        self.mems = [SlotMemory(dev, slot_bytes) for _ in range(slots)]


def serve_stream(staged, arrivals, ctx=None, max_batch=16, max_bytes=72 << 30, slots=3,
                 pack_pairs=PACK_PAIRS, graph=True, keep=True, server=None):
    """Continuous batching: requests arriving at `arrivals` (seconds from
    start) are admitted as soon as a stream slot and memory allow, while
    earlier batches are still running; up to `slots` batches overlap on the
    device, each slot with a pack of its own (its graph captured at the
    slot's first batch).  Returns (latencies, results, wall time); keep=False
    drops each batch's results once complete, and each slot then carves its
    buffers from one reused allocation (the `server`'s, when given)."""
    import torch
    ctx = ctx or context()
    if server is None or len(server.streams) != slots or server.max_batch < max_batch:
        server = Server(slots, max_batch, ctx, slot_bytes=0 if keep else 24 << 30)
    streams, packs = server.streams, server.packs
    mems = [None] * slots if keep else server.mems
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
                if keep:
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
            plans = _plan_on(staged[nxt:end], ctx, streams[slot], pack_pairs)
            # admit the longest prefix that fits the memory left (at least one
            # request when nothing else is in flight), and the slot's buffer
            # when the slot carves one
            cap = server.slot_bytes if mems[slot] is not None and server.slot_bytes else max_bytes
            take, need = 0, 0
            for s, p in zip(staged[nxt:end], plans):
                b = request_bytes(s, p, pack_pairs)
                if take and (used + need + b > max_bytes or need + b > cap):
                    break
                if not take and inflight and used + b > max_bytes:
                    break
                take += 1
                need += b
            if take:
                free.pop(0)
                f = InFlight(staged[nxt:nxt + take], plans[:take], streams[slot], ctx,
                             packs[slot], pack_pairs, graph, mems[slot])
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


def closed_loop(staged, ctx=None, max_batch=16, max_bytes=72 << 30, slots=3,
                pack_pairs=PACK_PAIRS, server=None):
    """Batched capacity: every request available at once; seconds."""
    _, _, wall = serve_stream(staged, np.zeros(len(staged)), ctx, max_batch, max_bytes, slots,
                              pack_pairs, keep=False, server=server)
    return wall


def open_loop(staged, rate, ctx=None, max_batch=16, max_bytes=72 << 30, slots=3,
              seed=10044548, pack_pairs=PACK_PAIRS, server=None):
    """Continuous batching under Poisson arrivals at `rate` requests/s.
    Returns per-request latencies (s) and the wall time."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(staged)))
    lat, _, wall = serve_stream(staged, arrivals, ctx, max_batch, max_bytes, slots, pack_pairs,
                                keep=False, server=server)
    return lat, wall


def percentiles(lat):
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(np.mean(lat) * 1e3)}
