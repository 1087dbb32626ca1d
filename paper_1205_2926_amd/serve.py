"""Continuous-batching server for exact polynomial products on one GPU.

Requests (pairs of uint32 coefficient arrays) arrive over time.  One engine
loop on the host:

* admits waiting requests in arrival order while their device memory fits the
  HBM budget (operands, product and the plan's workspace, all carved out of one
  arena allocated up front, so the budget can never be exceeded);
* launches each admitted group as one batch (``hntt_polymul_plan_*``: three
  primes + CRT) on the next idle HIP stream, so batches that are admitted
  while others are still on the GPU run concurrently with them;
* retires batches as their completion events fire, copies results back, frees
  their memory, and admits whatever now fits.

Twiddle tables stay resident on the context across batches.  A request's
result never depends on what it was batched with: every product is computed
independently (checked by the tests: alone vs in the mix, bit for bit).
Latency is arrival -> result on the host; ``run`` reports p50/p99 and products/s.
"""
from __future__ import annotations

import bisect
import time
from collections import deque
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
    result: np.ndarray = None
    admitted: float = None
    finished: float = None
    batch: int = -1

    @property
    def nout(self) -> int:
        return self.a.size + self.b.size - 1

    def operand_bytes(self) -> int:
        return _up(4 * self.a.size) + _up(4 * self.b.size) + _up(8 * self.nout)


@dataclass
class _Batch:
    bid: int
    reqs: list
    offset: int
    nbytes: int
    stream: torch.cuda.Stream
    event: torch.cuda.Event
    plan: object
    outs_host: list
    keep: list = field(default_factory=list)


class PolymulServer:
    """Serve exact polynomial products within `hbm_budget` bytes of device memory."""

    def __init__(self, ctx: hntt.Context, hbm_budget: int, streams: int = 4, max_batch: int = 64,
                 plain: bool = False):
        self.ctx = ctx
        self.budget = _up(hbm_budget)
        self.arena_t = torch.empty(self.budget, dtype=torch.uint8, device="cuda")
        self.arena = Arena(self.budget)
        self.streams = [torch.cuda.Stream() for _ in range(streams)]  # default priority
        self.max_batch = max_batch
        self.plain = plain
        self.inflight: list[_Batch] = []
        self.nbatches = 0
        self.rejected: list[Request] = []

    def request_bytes(self, reqs) -> int:
        ws = hntt.polymul_workspace_size([(r.a.size, r.b.size) for r in reqs])
        return sum(r.operand_bytes() for r in reqs) + _up(ws)

    def _view(self, off: int, nbytes: int, dtype) -> torch.Tensor:
        return self.arena_t[off:off + nbytes].view(dtype)

    def _launch(self, reqs, now):
        nbytes = self.request_bytes(reqs)
        off = self.arena.alloc(nbytes)
        if off is None:
            return False
        busy = {id(b.stream) for b in self.inflight}
        stream = next(s for s in self.streams if id(s) not in busy)
        pairs, outs, outs_host, keep = [], [], [], []
        cur = off
        with torch.cuda.stream(stream):
            for r in reqs:
                da = self._view(cur, 4 * r.a.size, torch.int32)
                cur += _up(4 * r.a.size)
                db = self._view(cur, 4 * r.b.size, torch.int32)
                cur += _up(4 * r.b.size)
                do = self._view(cur, 8 * r.nout, torch.int64)
                cur += _up(8 * r.nout)
                ha = torch.from_numpy(r.a.view(np.int32)).pin_memory()
                hb = torch.from_numpy(r.b.view(np.int32)).pin_memory()
                da.copy_(ha, non_blocking=True)
                db.copy_(hb, non_blocking=True)
                pairs.append((da, db))
                outs.append(do)
                keep += [ha, hb]
            ws_bytes = off + nbytes - cur
            ws = self._view(cur, ws_bytes, torch.uint8)
            plan = self.ctx.polymul_plan(pairs, outs, plain=self.plain, graph=False, workspace=ws, stream=stream)
            plan.execute(stream=stream)
            for do in outs:
                ho = torch.empty(do.numel(), dtype=torch.int64, pin_memory=True)
                ho.copy_(do, non_blocking=True)
                outs_host.append(ho)
            ev = torch.cuda.Event()
            ev.record(stream)
        for r in reqs:
            r.admitted = now
            r.batch = self.nbatches
        self.inflight.append(_Batch(self.nbatches, reqs, off, nbytes, stream, ev, plan, outs_host, keep))
        self.nbatches += 1
        return True

    def _retire(self, now) -> int:
        done = 0
        for bt in list(self.inflight):
            if bt.event.query():
                for r, ho in zip(bt.reqs, bt.outs_host):
                    r.result = ho.numpy().view(np.uint64).copy()
                    r.finished = now
                bt.plan.destroy()
                self.arena.release(bt.offset, bt.nbytes)
                self.inflight.remove(bt)
                done += len(bt.reqs)
        return done

    def run(self, requests: list[Request], time_limit: float = 600.0) -> dict:
        """Serve `requests` (sorted by arrival, seconds from now); returns latency statistics."""
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
                if self.request_bytes([r]) > self.budget:
                    self.rejected.append(r)  # can never fit: refuse instead of waiting forever
                else:
                    pending.append(r)
                nxt += 1
            finished += self._retire(now)
            # admission: the longest arrival-ordered prefix of the queue that fits now
            while pending and len(self.inflight) < len(self.streams):
                group = []
                while pending and len(group) < self.max_batch:
                    cand = group + [pending[0]]
                    if self.request_bytes(cand) > self.budget - self.arena.used:
                        break
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
        }


def make_requests(seed: int, count: int, rate_per_s: float, lo_bits: float = 10, hi_bits: float = 20):
    """Poisson arrivals of products with log-uniform lengths (see workloads.poisson_requests)."""
    from .workloads import poisson_requests
    return [Request(i, t, a, b) for i, (t, a, b) in enumerate(poisson_requests(seed, count, rate_per_s, lo_bits,
                                                                              hi_bits))]
