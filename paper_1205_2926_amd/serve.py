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

Twiddle tables stay resident on the context across batches.  A request's
result never depends on what it was batched with: every product is computed
independently (checked by the tests: alone vs in the mix, bit for bit).
Latency is arrival -> result on the host; ``run`` reports p50/p99 and products/s.
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

    def __post_init__(self):
        if self.out is not None and not (isinstance(self.out, np.ndarray) and self.out.dtype == np.uint64
                                         and self.out.ndim == 1 and self.out.size >= self.nout
                                         and self.out.flags.c_contiguous and self.out.flags.writeable):
            raise ValueError("out must be a writable contiguous uint64 array of at least na + nb - 1 words")

    @property
    def nout(self) -> int:
        return self.a.size + self.b.size - 1

    def io_bytes(self) -> int:
        """Operands and product, each 256-byte aligned (the same on the device and in staging)."""
        return _up(4 * self.a.size) + _up(4 * self.b.size) + _up(8 * self.nout)

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
        self.nbatches = 0
        self.rejected: list[Request] = []
        # host copies into and out of the staging buffer run on a few threads (numpy
        # releases the GIL for plain copies)
        self.pool = ThreadPoolExecutor(max_workers=copy_threads)

    def _fits_alone(self, r: Request) -> bool:
        return r.device_bytes() + _GROUP_SLACK <= self.budget and r.io_bytes() <= self.harena.size

    def _launch(self, reqs, now) -> bool:
        io = [r.io_bytes() for r in reqs]
        in_bytes = sum(_up(4 * r.a.size) + _up(4 * r.b.size) for r in reqs)
        host_bytes = sum(io)
        dev_bytes = host_bytes + sum(r.workspace_bound() for r in reqs) + _GROUP_SLACK
        doff = self.arena.alloc(dev_bytes)
        if doff is None:
            return False
        hoff = self.harena.alloc(host_bytes)
        if hoff is None:
            self.arena.release(doff, dev_bytes)
            return False
        busy = {id(b.stream) for b in self.inflight}
        stream = next(s for s in self.streams if id(s) not in busy)
        # layout (same relative offsets on both sides): all operands, then all products
        pairs, outs, out_offs, copies = [], [], [], []
        cur, ocur = 0, in_bytes
        for r in reqs:
            na, nb = r.a.size, r.b.size
            copies.append((hoff + cur, r.a))
            da = self.arena_t[doff + cur:doff + cur + 4 * na].view(torch.int32)
            cur += _up(4 * na)
            copies.append((hoff + cur, r.b))
            db = self.arena_t[doff + cur:doff + cur + 4 * nb].view(torch.int32)
            cur += _up(4 * nb)
            do = self.arena_t[doff + ocur:doff + ocur + 8 * r.nout].view(torch.int64)
            pairs.append((da, db))
            outs.append(do)
            out_offs.append(ocur)
            ocur += _up(8 * r.nout)

        def pack(job):
            off, src = job
            self.host_np[off:off + 4 * src.size].view(np.uint32)[:] = src

        list(self.pool.map(pack, copies))
        ws = self.arena_t[doff + host_bytes:doff + dev_bytes]
        with torch.cuda.stream(stream):
            self.arena_t[doff:doff + in_bytes].copy_(self.host_t[hoff:hoff + in_bytes], non_blocking=True)
            plan = self.ctx.polymul_plan(pairs, outs, plain=self.plain, graph=False, workspace=ws, stream=stream)
            plan.execute(stream=stream)
            self.host_t[hoff + in_bytes:hoff + host_bytes].copy_(self.arena_t[doff + in_bytes:doff + host_bytes],
                                                                 non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        for r in reqs:
            r.admitted = now
            r.batch = self.nbatches
        self.inflight.append(_Batch(self.nbatches, reqs, doff, dev_bytes, hoff, host_bytes, out_offs, stream, ev,
                                    plan))
        self.nbatches += 1
        return True

    def _retire(self, now) -> int:
        done = 0
        for bt in list(self.inflight):
            if bt.event.query():
                def unpack(job, base=bt.host_off):
                    r, o = job
                    src = self.host_np[base + o:base + o + 8 * r.nout].view(np.uint64)
                    if r.out is not None:  # into the client's buffer: no allocation here
                        np.copyto(r.out[:r.nout], src)
                        r.result = r.out[:r.nout]
                    else:
                        r.result = src.copy()

                list(self.pool.map(unpack, zip(bt.reqs, bt.out_offs)))
                for r in bt.reqs:
                    r.finished = now
                bt.plan.destroy()
                self.arena.release(bt.dev_off, bt.dev_bytes)
                self.harena.release(bt.host_off, bt.host_bytes)
                self.inflight.remove(bt)
                done += len(bt.reqs)
        return done

    def run(self, requests: list[Request], time_limit: float = 600.0) -> dict:
        """Serve `requests` (arrival in seconds from now); returns throughput and latency statistics."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending: deque = deque()
        nxt = 0
        finished = 0
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
            finished += self._retire(now)
            # admission: the longest arrival-ordered prefix of the queue that fits now
            while pending and len(self.inflight) < len(self.streams):
                group, dev, host = [], _GROUP_SLACK, 0
                dev_free = self.budget - self.arena.used
                host_free = self.harena.size - self.harena.used
                while pending and len(group) < self.max_batch:
                    r = pending[0]
                    if dev + r.device_bytes() > dev_free or host + r.io_bytes() > host_free:
                        break
                    dev += r.device_bytes()
                    host += r.io_bytes()
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
            "peak_bytes": self.arena.peak,
            "budget_bytes": self.budget,
            "host_staging_bytes": self.harena.size,
        }

    def close(self):
        """Release the device arena and the pinned staging buffer (in-flight batches first)."""
        if self.inflight:
            torch.cuda.synchronize()
            self._retire(0.0)
        self.pool.shutdown()
        self.arena_t = None
        self.host_t = None
        self.host_np = None


def make_requests(seed: int, count: int, rate_per_s: float, lo_bits: float = 10, hi_bits: float = 20,
                  client_out: bool = False):
    """Poisson arrivals of products with log-uniform lengths (see workloads.poisson_requests).
    client_out: each request carries a result buffer that the client allocated and touched
    beforehand (as a client reusing its buffers would have), so that the server's unpacking
    is one copy per product and no page faults."""
    from .workloads import poisson_requests
    reqs = []
    for i, (t, a, b) in enumerate(poisson_requests(seed, count, rate_per_s, lo_bits, hi_bits)):
        out = None
        if client_out:
            out = np.empty(a.size + b.size - 1, np.uint64)
            out.fill(0)
        reqs.append(Request(i, t, a, b, out))
    return reqs
