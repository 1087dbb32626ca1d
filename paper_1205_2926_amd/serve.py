"""Continuous-batching server for exact polynomial products on one GPU.

Requests (pairs of uint32 coefficient arrays) arrive over time.  One engine
loop on the host:

* admits waiting requests in arrival order while their device memory fits the
  HBM budget (operands, product and the plan's workspace, all carved out of one
  arena allocated up front, so the budget can never be exceeded) and their
  operands and product fit the pinned host staging buffer;
* launches each admitted group as one batch (``hntt_polymul_plan_*``: three
  primes + CRT) on the next idle HIP stream, so batches that are admitted
  while others are still on the GPU run concurrently with them;
* retires batches as their completion events fire, copies results back (into
  buffers the client provides, when it does), frees their memory, and admits
  whatever now fits.

Operands and products travel through a pinned staging buffer unless the
client brings them in pinned host memory itself (``Request.pinned``): then
they are copied between its buffers and the device directly, and the host
moves no data at all.

Twiddle tables stay resident on the context across batches.  A request's
result never depends on what it was batched with: every product is computed
independently (checked by the tests: alone vs in the mix, bit for bit).
Latency is arrival -> result on the host (stamped after the copy out of
staging); ``run`` reports p50/p99, products/s, the most batches that were on
the GPU at once, the fraction of the run during which any batch was in flight,
and the fractions during which product kernels, copies in and copies out ran
(from events around each phase on the batch's stream), with the host<->device
bytes per second.
"""
from __future__ import annotations

import bisect
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
import torch

from . import hntt

_ALIGN = 256


def _up(x: int, a: int = _ALIGN) -> int:
    return (x + a - 1) // a * a


class Arena:
    """First-fit allocator of byte ranges inside one device buffer."""

    def __init__(self, nbytes: int):
        self.size = nbytes
        self.free = [(0, nbytes)]  # sorted (offset, length)
        self.used = 0
        self.peak = 0

    def alloc(self, nbytes: int):
        nbytes = _up(nbytes)
        for i, (off, ln) in enumerate(self.free):
            if ln >= nbytes:
                if ln == nbytes:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + nbytes, ln - nbytes)
                self.used += nbytes
                self.peak = max(self.peak, self.used)
                return off
        return None

    def release(self, off: int, nbytes: int):
        nbytes = _up(nbytes)
        self.used -= nbytes
        i = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(i, (off, nbytes))
        # merge with neighbours
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    a: np.ndarray           # uint32 coefficients
    b: np.ndarray
    out: np.ndarray = None  # optional client buffer (uint64, >= nout words) that receives the product
    result: np.ndarray = None
    admitted: float = None
    finished: float = None
    batch: int = -1
    # optional pinned host tensors of the client (int32 operands, int64 product) that a,
    # b and out are views of: the server then copies straight between them and the device
    pinned: tuple = None

    def __post_init__(self):
        if self.out is not None and not (isinstance(self.out, np.ndarray) and self.out.dtype == np.uint64
                                         and self.out.ndim == 1 and self.out.size >= self.nout
                                         and self.out.flags.c_contiguous and self.out.flags.writeable):
            raise ValueError("out must be a writable contiguous uint64 array of at least na + nb - 1 words")
        if self.pinned is not None:
            ta, tb, to = self.pinned
            ok = all(isinstance(t, torch.Tensor) and t.device.type == "cpu" and t.is_pinned() and t.is_contiguous()
                     and t.dim() == 1 for t in (ta, tb, to))
            ok = ok and ta.dtype == tb.dtype == torch.int32 and to.dtype == torch.int64
            ok = ok and ta.numel() == self.a.size and tb.numel() == self.b.size and to.numel() >= self.nout
            ok = ok and self.out is not None and np.shares_memory(self.out, to.numpy())
            if not ok:
                raise ValueError("pinned must be (a, b, out) pinned contiguous host tensors (int32, int32, int64) "
                                 "that a, b and out are views of")

    @property
    def direct(self) -> bool:
        return self.pinned is not None

    @property
    def nout(self) -> int:
        return self.a.size + self.b.size - 1

    def io_bytes(self) -> int:
        """Operands and product, each 256-byte aligned (the same on the device and in staging)."""
        return _up(4 * self.a.size) + _up(4 * self.b.size) + _up(8 * self.nout)

    def staging_bytes(self) -> int:
        return 0 if self.direct else self.io_bytes()

    def workspace_bound(self) -> int:
        """Upper bound of this product's share of a plan workspace: six padded residue arrays,
        its pair record, chunk lists and nine transform entries (hntt_polymul_workspace_size
        of a group is at most the sum of these plus _GROUP_SLACK)."""
        n = max(self.a.size, self.b.size)
        L = 1 << max(1, (n - 1).bit_length() + 1)
        chunks = -(-L // 1024) + -(-self.nout // 1024)
        return 24 * L + 48 + 8 * chunks + 9 * 16

    def device_bytes(self) -> int:
        return self.io_bytes() + self.workspace_bound()


_GROUP_SLACK = 5 * _ALIGN  # alignment of the five regions of a plan workspace


@dataclass
class _Batch:
    bid: int
    reqs: list
    dev_off: int
    dev_bytes: int
    host_off: int
    host_bytes: int
    out_offs: list
    stream: torch.cuda.Stream
    event: torch.cuda.Event
    plan: object
    start: torch.cuda.Event
    k0: torch.cuda.Event   # after the copies in, before the product kernels
    k1: torch.cuda.Event   # after the product kernels, before the copies out
    h2d_bytes: int
    d2h_bytes: int


class PolymulServer:
    """Serve exact polynomial products within `hbm_budget` bytes of device memory.

    Operands and products travel through one pinned host staging buffer
    (`host_staging` bytes, default min(budget, 1 GiB)): a batch's operands are packed
    into it and sent with one host-to-device copy, and its products come back with
    one device-to-host copy, so no per-request allocation happens while serving."""

    def __init__(self, ctx: hntt.Context, hbm_budget: int, streams: int = 4, max_batch: int = 64,
                 plain: bool = False, host_staging: int = None, copy_threads: int = 8):
        self.ctx = ctx
        self.budget = _up(hbm_budget)
        self.arena_t = torch.empty(self.budget, dtype=torch.uint8, device="cuda")
        self.arena = Arena(self.budget)
        staging = _up(host_staging if host_staging is not None else min(self.budget, 1 << 30))
        self.host_t = torch.empty(staging, dtype=torch.uint8, pin_memory=True)
        self.host_np = self.host_t.numpy()
        self.harena = Arena(staging)
        self.streams = [torch.cuda.Stream() for _ in range(streams)]  # default priority
        self.max_batch = max_batch
        self.plain = plain
        self.inflight: list[_Batch] = []
        self.max_inflight = 0
        self.busy_spans: list[tuple[float, float]] = []  # (start, end) ms of each batch on the GPU
        self.kernel_spans: list[tuple[float, float]] = []  # (start, end) ms of each batch's product kernels
        self.in_spans: list[tuple[float, float]] = []      # (start, end) ms of each batch's copies in
        self.out_spans: list[tuple[float, float]] = []     # (start, end) ms of each batch's copies out
        self.h2d_bytes = 0
        self.d2h_bytes = 0
        self.t_ref = None                                  # timing event at the start of run()
        self.nbatches = 0
        self.rejected: list[Request] = []
        # host copies into and out of the staging buffer run on a few threads (numpy
        # releases the GIL for plain copies)
        self.pool = ThreadPoolExecutor(max_workers=copy_threads)

    def _fits_alone(self, r: Request) -> bool:
        return r.device_bytes() + _GROUP_SLACK <= self.budget and r.staging_bytes() <= self.harena.size

    def _launch(self, reqs, now) -> bool:
        # device layout: staged operands | direct operands | staged products | direct products;
        # the staging buffer mirrors the staged parts (operands, then products)
        staged = [r for r in reqs if not r.direct]
        direct = [r for r in reqs if r.direct]
        st_in = sum(_up(4 * r.a.size) + _up(4 * r.b.size) for r in staged)
        st_out = sum(_up(8 * r.nout) for r in staged)
        all_in = st_in + sum(_up(4 * r.a.size) + _up(4 * r.b.size) for r in direct)
        io_bytes = sum(r.io_bytes() for r in reqs)
        dev_bytes = io_bytes + sum(r.workspace_bound() for r in reqs) + _GROUP_SLACK
        host_bytes = st_in + st_out
        doff = self.arena.alloc(dev_bytes)
        if doff is None:
            return False
        hoff = 0
        if host_bytes:
            hoff = self.harena.alloc(host_bytes)
            if hoff is None:
                self.arena.release(doff, dev_bytes)
                return False
        busy = {id(b.stream) for b in self.inflight}
        stream = next(s for s in self.streams if id(s) not in busy)
        pairs, outs, out_offs, copies, direct_in = [], [], {}, [], []
        cur, ocur = 0, all_in
        for r in staged + direct:
            na, nb = r.a.size, r.b.size
            da = self.arena_t[doff + cur:doff + cur + 4 * na].view(torch.int32)
            if r.direct:
                direct_in.append((da, r.pinned[0]))
            else:
                copies.append((hoff + cur, r.a))
            cur += _up(4 * na)
            db = self.arena_t[doff + cur:doff + cur + 4 * nb].view(torch.int32)
            if r.direct:
                direct_in.append((db, r.pinned[1]))
            else:
                copies.append((hoff + cur, r.b))
            cur += _up(4 * nb)
            do = self.arena_t[doff + ocur:doff + ocur + 8 * r.nout].view(torch.int64)
            pairs.append((da, db))
            outs.append(do)
            out_offs[id(r)] = ocur - all_in + st_in  # staging offset of a staged product
            ocur += _up(8 * r.nout)

        def pack(job):
            off, src = job
            self.host_np[off:off + 4 * src.size].view(np.uint32)[:] = src

        if copies:
            list(self.pool.map(pack, copies))
        ws = self.arena_t[doff + io_bytes:doff + dev_bytes]
        # the plan is built on the host before anything is queued, so that the phase spans
        # below hold GPU work only
        plan = self.ctx.polymul_plan(pairs, outs, plain=self.plain, graph=False, workspace=ws, stream=stream)
        with torch.cuda.stream(stream):
            start = torch.cuda.Event(enable_timing=True)
            start.record(stream)
            if st_in:
                self.arena_t[doff:doff + st_in].copy_(self.host_t[hoff:hoff + st_in], non_blocking=True)
            for dst, src in direct_in:
                dst.copy_(src, non_blocking=True)
            k0 = torch.cuda.Event(enable_timing=True)
            k0.record(stream)
            plan.execute(stream=stream)
            k1 = torch.cuda.Event(enable_timing=True)
            k1.record(stream)
            if st_out:
                self.host_t[hoff + st_in:hoff + host_bytes].copy_(self.arena_t[doff + all_in:doff + all_in + st_out],
                                                                  non_blocking=True)
            for r, do in zip(staged + direct, outs):
                if r.direct:
                    r.pinned[2][:r.nout].copy_(do, non_blocking=True)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
        order = staged + direct
        for r in order:
            r.admitted = now
            r.batch = self.nbatches
        self.inflight.append(_Batch(self.nbatches, order, doff, dev_bytes, hoff, host_bytes,
                                    [out_offs[id(r)] for r in order], stream, ev, plan, start, k0, k1,
                                    all_in, sum(8 * r.nout for r in order)))
        self.max_inflight = max(self.max_inflight, len(self.inflight))
        self.nbatches += 1
        return True

    def _retire(self, t0: float) -> int:
        done = 0
        for bt in list(self.inflight):
            if bt.event.query():
                def unpack(job, base=bt.host_off):
                    r, o = job
                    if r.direct:  # already in the client's pinned buffer
                        r.result = r.out[:r.nout]
                        return
                    src = self.host_np[base + o:base + o + 8 * r.nout].view(np.uint64)
                    if r.out is not None:  # into the client's buffer: no allocation here
                        np.copyto(r.out[:r.nout], src)
                        r.result = r.out[:r.nout]
                    else:
                        r.result = src.copy()

                list(self.pool.map(unpack, zip(bt.reqs, bt.out_offs)))
                finished = time.perf_counter() - t0  # the results are on the host now
                for r in bt.reqs:
                    r.finished = finished
                if self.t_ref is not None:
                    t = [self.t_ref.elapsed_time(e) for e in (bt.start, bt.k0, bt.k1, bt.event)]
                    self.busy_spans.append((t[0], t[3]))
                    self.in_spans.append((t[0], t[1]))
                    self.kernel_spans.append((t[1], t[2]))
                    self.out_spans.append((t[2], t[3]))
                self.h2d_bytes += bt.h2d_bytes
                self.d2h_bytes += bt.d2h_bytes
                bt.plan.destroy()
                self.arena.release(bt.dev_off, bt.dev_bytes)
                if bt.host_bytes:
                    self.harena.release(bt.host_off, bt.host_bytes)
                self.inflight.remove(bt)
                done += len(bt.reqs)
        return done

    @staticmethod
    def _union_ms(spans) -> float:
        """Length of the union of (start, end) intervals."""
        total, end = 0.0, None
        for a, b in sorted(spans):
            if end is None or a > end:
                total += b - a
                end = b
            elif b > end:
                total += b - end
                end = b
        return total

    def run(self, requests: list[Request], time_limit: float = 600.0) -> dict:
        """Serve `requests` (arrival in seconds from now); returns throughput and latency statistics."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending: deque = deque()
        nxt = 0
        finished = 0
        self.busy_spans, self.kernel_spans, self.in_spans, self.out_spans = [], [], [], []
        self.h2d_bytes = self.d2h_bytes = 0
        self.t_ref = torch.cuda.Event(enable_timing=True)
        self.t_ref.record(torch.cuda.current_stream())
        t0 = time.perf_counter()
        while finished + len(self.rejected) < len(reqs):
            now = time.perf_counter() - t0
            if now > time_limit:
                raise TimeoutError("serving run exceeded its time limit")
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                r = reqs[nxt]
                if not self._fits_alone(r):
                    self.rejected.append(r)  # can never fit: refuse instead of waiting forever
                else:
                    pending.append(r)
                nxt += 1
            finished += self._retire(t0)
            # admission: the longest arrival-ordered prefix of the queue that fits now
            while pending and len(self.inflight) < len(self.streams):
                group, dev, host = [], _GROUP_SLACK, 0
                dev_free = self.budget - self.arena.used
                host_free = self.harena.size - self.harena.used
                while pending and len(group) < self.max_batch:
                    r = pending[0]
                    if dev + r.device_bytes() > dev_free or host + r.staging_bytes() > host_free:
                        break
                    dev += r.device_bytes()
                    host += r.staging_bytes()
                    group.append(pending.popleft())
                if not group or not self._launch(group, now):
                    for r in reversed(group):
                        pending.appendleft(r)
                    break
            if not self.inflight and not pending and nxt < len(reqs):
                wait = reqs[nxt].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.001))
        wall = time.perf_counter() - t0
        torch.cuda.synchronize()
        inflight_ms = self._union_ms(self.busy_spans)
        wall_ms = wall * 1e3
        frac = {k: self._union_ms(sp) / wall_ms if wall > 0 else 0.0
                for k, sp in (("kernel_frac", self.kernel_spans), ("h2d_frac", self.in_spans),
                              ("d2h_frac", self.out_spans))}
        lat = np.array([r.finished - r.arrival for r in reqs if r.result is not None])
        return {
            "requests": len(reqs),
            "completed": int(lat.size),
            "rejected": len(self.rejected),
            "batches": self.nbatches,
            "wall_s": wall,
            "products_per_s": lat.size / wall if wall > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "mean_ms": float(lat.mean() * 1e3) if lat.size else None,
            "max_inflight": self.max_inflight,
            # share of the wall time with at least one batch between its first copy in and
            # its last copy out (copies and waits on the stream included)
            "inflight_frac": inflight_ms / wall_ms if wall > 0 else 0.0,
            # shares of the wall time with at least one batch in each phase: product kernels,
            # copies in, copies out (a phase's span on a stream includes waits for a copy engine)
            **frac,
            # operand and product bytes moved between host and device, per second of wall time
            "h2d_GBs": self.h2d_bytes / wall / 1e9 if wall > 0 else 0.0,
            "d2h_GBs": self.d2h_bytes / wall / 1e9 if wall > 0 else 0.0,
            "peak_bytes": self.arena.peak,
            "budget_bytes": self.budget,
            "host_staging_bytes": self.harena.size,
        }

    def close(self):
        """Release the device arena and the pinned staging buffer (in-flight batches first)."""
        if self.inflight:
            torch.cuda.synchronize()
            self._retire(time.perf_counter())
        self.pool.shutdown()
        self.arena_t = None
        self.host_t = None
        self.host_np = None


def make_requests(seed: int, count: int, rate_per_s: float, lo_bits: float = 10, hi_bits: float = 20,
                  client_out: bool = False, pinned: bool = False):
    """Poisson arrivals of products with log-uniform lengths (see workloads.poisson_requests).
    client_out: each request carries a result buffer that the client allocated and touched
    beforehand (as a client reusing its buffers would have), so that the server's unpacking
    is one copy per product and no page faults.
    pinned: the client keeps operands and result buffer in pinned host memory (as a client
    that reuses pinned buffers would), so the server copies straight to and from them."""
    from .workloads import poisson_requests
    reqs = []
    for i, (t, a, b) in enumerate(poisson_requests(seed, count, rate_per_s, lo_bits, hi_bits)):
        out, pin = None, None
        if pinned:
            ta = torch.from_numpy(a.view(np.int32)).pin_memory()
            tb = torch.from_numpy(b.view(np.int32)).pin_memory()
            to = torch.zeros(a.size + b.size - 1, dtype=torch.int64).pin_memory()
            a, b, out = ta.numpy().view(np.uint32), tb.numpy().view(np.uint32), to.numpy().view(np.uint64)
            pin = (ta, tb, to)
        elif client_out:
            out = np.empty(a.size + b.size - 1, np.uint64)
            out.fill(0)
        reqs.append(Request(i, t, a, b, out, pinned=pin))
    return reqs
