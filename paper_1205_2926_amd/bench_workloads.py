"""Measurements of the non-headline workloads for ``bench.py --workload ...``.

single1k  one forward NTT of 1024 residues (latency, lazy and plain)
u64       8 NTTs of length 2^22 over the 62-bit prime, forward + inverse, lazy vs plain vs Montgomery
bigmul    16 products of 2^20-limb (32 Mbit) integers, three primes + device carry scan
pointwise c = a b mod p over 64 x 2^20 u32 words (HBM roofline of the standalone product)
table1    host CPU: Algorithm 2 vs Algorithm 3, one transform of 2^11 over the 62-bit prime
          (the design of the paper's Table 1), time per butterfly on one core
polymul   4096 products with log-uniform lengths 2^8..2^16, three primes + CRT, one graph launch
          (each length class a parallel branch of the graph)
serving   Poisson stream of products (lengths 2^10..2^20), rate swept up to saturation
Each returns one JSON-able dict.  Inputs are the seeded synthetic workloads of
``workloads.py``; results are checked before the numbers are reported, with
checks that need neither the library nor the test oracle: round trips,
products of whole integers in CPython (a product polynomial with coefficients
below 2^64 is the base-2^64 digit string of A(2^64) * B(2^64)), compared
exactly or modulo two 61-bit primes, and numpy's own modular product.
"""
from __future__ import annotations

import hashlib
import json
import os
import random
import sys
import time

import numpy as np
import torch

from . import autotune, hntt
from .workloads import BATCH8_4M_U64, SINGLE_1K, polymul_pairs


def _as_int(words: np.ndarray, digit_bytes: int) -> int:
    """The integer whose base-2^(8 digit_bytes) digits, least significant first, are `words`."""
    return int.from_bytes(np.ascontiguousarray(words, dtype=f"<u{digit_bytes}").tobytes(), "little")


_M61 = (2305843009213693951, 2305843009213693921)


def _product_ok(a: np.ndarray, b: np.ndarray, c: np.ndarray) -> bool:
    """Whether c holds the coefficients of a * b.  With a, b < 2^20 and at most 2^20 terms
    every coefficient of the product is below 2^60, so C(2^64) = A(2^64) * B(2^64) as
    integers.  Short products compare that identity exactly; long ones compare it modulo two
    61-bit primes and compare the lowest 512 coefficients exactly (CPython's product of
    64-Mbit integers would take tens of seconds)."""
    if c.size != a.size + b.size - 1:
        return False
    A, B, C = _as_int(a, 8), _as_int(b, 8), _as_int(c, 8)
    if c.size <= 1 << 13:
        return C == A * B
    low = (1 << (64 * 512)) - 1
    return (all(C % m == (A % m) * (B % m) % m for m in _M61)
            and C & low == ((A & low) * (B & low)) & low)


def _events_ms(fn, reps):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_TRAFFIC = os.path.join(_ROOT, "profiles", "hbm_traffic_workloads.json")
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12  # 256 CUs x 64 int32 lanes x 2.4 GHz


def _counters(workload):
    """The committed rocprofv3 figures of a workload (HBM bytes and VALU instructions per batch
    or per launch), or None when the kernel sources changed since they were taken."""
    try:
        rec = json.load(open(_TRAFFIC))
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(_ROOT, f), "rb").read())
    except (OSError, ValueError, KeyError):
        return None
    return rec["workloads"].get(workload) if h.hexdigest() == rec["source_sha256"] else None


def _batch_roofline(workload, ms, butterflies):
    """Roofline of a whole product batch: the algorithmic VALU work (9 int32 operations per
    butterfly of Algorithm 3, the CRT and products not counted) against the int32 VALU peak,
    and the HBM bytes the committed counters recorded for one batch against the 8 TB/s peak;
    `bound` is the larger fraction (HBM only when the counters are current)."""
    alu = butterflies * 9 / (ms * 1e-3) / 1e12
    rec = _counters(workload)
    out = {"bound": "alu", "achieved": alu, "peak": VALU_PEAK_TOPS, "unit": "Tops/s", "frac": alu / VALU_PEAK_TOPS,
           "traffic": None, "basis": "butterflies x 9 int32 ops per batch / batch time"}
    if rec:
        gbs = rec["bytes_per_batch"] / (ms * 1e-3) / 1e9
        out["traffic"] = rec["bytes_per_batch"]
        out["hbm"] = {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                      "basis": "counted HBM bytes per batch (FETCH_SIZE, WRITE_SIZE) / batch time"}
        out["valu_issue"] = rec["valu_insts_per_batch"] / (256 * 2.4e9 * ms * 1e-3)
        if gbs / HBM_PEAK_GBS > out["frac"]:
            out.update({"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "basis": out["hbm"]["basis"]})
    return out


def _u64_roofline(ms, cfg):
    """HBM roofline of the 64-bit batch: four passes per forward+inverse step, each reading and
    writing every 8-byte word once (the traffic of this two-pass design), over the step time;
    `traffic` is what the committed counters recorded for the four launches."""
    words = cfg.batch << cfg.log2_len
    alg = 4 * words * 16
    gbs = alg / (ms * 1e-3) / 1e9
    rec = _counters("u64")
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": sum(rec["bytes_per_launch"].values()) if rec else None,
            "basis": "4 passes x (8 B read + 8 B written) per word per step / step time"}


def _policies(args, all_policies):
    """The butterfly policies to measure: lazy only under --no-plain (which also drops the
    Montgomery comparison), else all of them."""
    return all_policies[:1] if args.no_plain else all_policies


def _ratios(res, key):
    return {f"lazy_over_{k}": res[k][key] / res["lazy"][key] for k in res if k != "lazy"}


def _time_plan(make_plan, count, args):
    """Batch time of a product plan over max(3, steps/2) executions after one untimed one, and
    how they were enqueued: one graph launch, or kernel by kernel (with the reason when
    recording the graph failed).  A second plan of the same batch without the graph gives the
    kernel-by-kernel time beside it."""
    res = {}
    for graph in (True, False):
        plan = make_plan(graph)
        plan.execute()
        torch.cuda.synchronize()
        ms = _events_ms(plan.execute, max(3, args.steps // 2))
        mode = plan.exec_mode
        plan.destroy()
        if graph:
            res = {"ms_per_batch": ms, "products_per_s": count / (ms / 1e3), "executed_as": mode}
        else:
            res["direct"] = {"ms_per_batch": ms, "executed_as": mode}
    return res


def _schedules(tuned):
    if tuned is not None:
        return {"schedules": {f"2^{l}": {k: v[k] for k in ("row_log2", "g_cols", "g_rows")}
                              for l, v in tuned["classes"].items()}, "tuned": True}
    return {"tuned": False}


def single1k(args):
    cfg = SINGLE_1K
    ctx = hntt.Context(0)
    w = hntt.root_of_unity(cfg.p, cfg.log2_len)
    x_np = cfg.data()
    x = torch.from_numpy(x_np.view(np.int32)).cuda()
    out = {"metric": "single forward NTT latency", "unit": "us", "workload": "1 x 2^10, p=998244353, u32"}
    for plain in (False, True):
        for _ in range(20):
            ctx.ntt_forward(x, cfg.p, w, plain=plain)
            ctx.ntt_inverse(x, cfg.p, w, plain=plain)
        fwd = _events_ms(lambda: ctx.ntt_forward(x, cfg.p, w, plain=plain), 200) * 1e3
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(200):
            ctx.ntt_forward(x, cfg.p, w, plain=plain)
            torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / 200 * 1e6
        out["plain" if plain else "lazy"] = {"device_us": fwd, "host_roundtrip_us": wall}
        x.copy_(torch.from_numpy(x_np.view(np.int32)))
        ctx.ntt_forward(x, cfg.p, w, plain=plain)
        ctx.ntt_inverse(x, cfg.p, w, plain=plain)
        assert np.array_equal(x.cpu().numpy().view(np.uint32), x_np), "single 1K round trip mismatch"
    ctx.close()
    return out


def u64(args):
    cfg = BATCH8_4M_U64
    ctx = hntt.Context(0)
    l, p = cfg.log2_len, cfg.p
    w = hntt.root_of_unity(p, l)
    x_np = cfg.data()
    x = torch.from_numpy(x_np.view(np.int64)).cuda()
    res = {}
    for policy in _policies(args, ("lazy", "plain", "mont")):
        kw = {"plain": policy == "plain", "mont": policy == "mont"}
        if not args.no_tune:
            autotune.tune(ctx, x, p, w, policy=policy)
        # untimed round trips first: a schedule from the tuning cache skips the tuner's trials,
        # which would otherwise have built this policy's tables and warmed the GPU
        autotune.warm(ctx, x, p, w, policy, 0.5)
        ms = _events_ms(lambda: (ctx.ntt_forward(x, p, w, **kw), ctx.ntt_inverse(x, p, w, **kw)), args.steps)
        res[policy] = {"ms_per_step": ms, "butterflies_per_s": 2 * cfg.butterflies / (ms / 1e3),
                       "schedule": ctx.get_plan(l, 64)}
    assert np.array_equal(x.cpu().numpy().view(np.uint64), x_np), "u64 round trip mismatch"
    ctx.close()
    return {"metric": "NTT butterflies/s, 64-bit words", "unit": "butterflies/s",
            "value": res["lazy"]["butterflies_per_s"], "workload": "8 x 2^22 forward+inverse, p=2^62-ish, u64",
            "p": p, **res, **_ratios(res, "ms_per_step"), "roofline": _u64_roofline(res["lazy"]["ms_per_step"], cfg)}


def polymul(args):
    pairs = polymul_pairs(seed=4, pairs=4096)
    ctx = hntt.Context(0)
    dpairs = [(torch.from_numpy(a.view(np.int32)).cuda(), torch.from_numpy(b.view(np.int32)).cuda())
              for a, b in pairs]
    outs = [torch.empty(a.size + b.size - 1, dtype=torch.int64, device="cuda") for a, b in pairs]
    # butterflies: per product, 6 forward and 3 inverse transforms of length L = 2 nextpow2(n)
    bfly = 0
    words = 0
    for a, b in pairs:
        n = max(a.size, b.size)
        l = (n - 1).bit_length() + 1
        bfly += 9 * l * (1 << (l - 1))
        words += 1 << l
    res = {}
    for policy in _policies(args, ("lazy", "plain")):
        plain = policy == "plain"
        # each policy gets its own per-class schedules, timed on this batch's own plan
        tuned = None if args.no_tune else autotune.tune_polymul(ctx, dpairs, outs, plain=plain)
        res[policy] = _time_plan(lambda graph: ctx.polymul_plan(dpairs, outs, plain=plain, graph=graph),
                                 len(pairs), args)
        res[policy]["butterflies_per_s"] = bfly / (res[policy]["ms_per_batch"] / 1e3)
        res[policy].update(_schedules(tuned))
    rr = random.Random(7)
    for i in rr.sample(range(len(pairs)), 64):
        assert _product_ok(*pairs[i], outs[i].cpu().numpy().view(np.uint64)), "polymul result mismatch"
    ctx.close()
    return {"metric": "exact polynomial products/s (3 primes + CRT, one graph launch)", "unit": "products/s",
            "value": res["lazy"]["products_per_s"],
            "workload": "4096 pairs, n log-uniform 2^8..2^16, coefficients < 2^20", "sum_padded_len": words,
            "butterflies_per_batch": bfly, **res, **_ratios(res, "ms_per_batch"),
            "roofline": _batch_roofline("polymul", res["lazy"]["ms_per_batch"], bfly)}


def serving(args):
    """Continuous batching of exact products (Poisson arrivals), for two kinds of client: one
    that keeps operands and result buffers in pinned host memory (the server copies straight
    to and from them: the reported value) and one with pageable buffers (through the server's
    pinned staging).  Saturation throughput is the highest achieved rate while the offered
    rate grows by 1.5x steps (from the rate of a burst queued at time 0) until the server falls
    behind; the offered rate is then swept over fractions of it, reporting achieved products/s,
    arrival-to-result p50/p99, the fraction of the wall time with a batch in flight (copies in,
    kernels, copies out), the fractions with product kernels, copies in and copies out running,
    the host<->device bytes per second, and the most batches in flight at once."""
    from .serve import PolymulServer, make_requests
    ctx = hntt.Context(0)
    budget = 8 << 30
    keys = ("offered_rate", "products_per_s", "p50_ms", "p99_ms", "inflight_frac", "kernel_frac", "h2d_frac",
            "d2h_frac", "h2d_GBs", "d2h_GBs", "max_inflight")

    def serve(reqs):
        srv = PolymulServer(ctx, budget)
        try:
            return srv.run(reqs)
        finally:
            srv.close()

    def at_rate(rate, pinned, seed=5):
        count = int(min(800, max(60, rate * 0.5)))
        reqs = make_requests(seed=seed, count=count, rate_per_s=rate, client_out=True, pinned=pinned)
        st = serve(reqs)
        st.update({"offered_rate": rate})
        return st, reqs

    def client(pinned, sweep_fracs):
        burst = serve(make_requests(seed=5, count=400, rate_per_s=1e9, client_out=True, pinned=pinned))
        # saturation: raise the offered rate until the server falls behind (achieved < 90% offered)
        rate, probes = burst["products_per_s"], []
        for _ in range(10):
            st, _ = at_rate(rate, pinned)
            probes.append({k: st[k] for k in keys})
            print(f"serving {'pinned' if pinned else 'pageable'} probe {probes[-1]}", file=sys.stderr, flush=True)
            if st["products_per_s"] < 0.9 * rate:
                break
            rate *= 1.5
        mu = max(p["products_per_s"] for p in probes)
        sweep, reqs = [], []
        for frac in sweep_fracs:
            st, reqs = at_rate(frac * mu, pinned)
            st.update({"offered_fraction": frac})
            sweep.append(st)
            print(f"serving {'pinned' if pinned else 'pageable'} at {frac} of saturation: "
                  f"{ {k: st[k] for k in keys} }", file=sys.stderr, flush=True)
        # every coefficient of a tenth of the last run's results
        for r in reqs[:: max(1, len(reqs) // 10)]:
            assert _product_ok(r.a, r.b, r.result[: r.nout]), "served product mismatch"
        return {"products_per_s": mu,
                "burst": {k: burst[k] for k in ("requests", "products_per_s", "p50_ms", "p99_ms", "batches",
                                                "inflight_frac", "kernel_frac", "h2d_frac", "d2h_frac",
                                                "h2d_GBs", "d2h_GBs", "max_inflight")},
                "saturation_probes": probes,
                "sweep": [{k: st[k] for k in ("offered_fraction", *keys, "mean_ms", "requests", "batches",
                                              "peak_bytes")} for st in sweep]}

    # warm the twiddle tables of every length class
    serve(make_requests(seed=50, count=40, rate_per_s=1e9))
    pinned = client(True, (0.1, 0.25, 0.5, 0.75, 0.9, 1.0, 1.2))
    staged = client(False, () if args.no_plain else (0.1, 0.5, 1.0))
    ctx.close()
    return {"metric": "serving: products/s at saturation, p50/p99 latency vs offered rate", "unit": "products/s",
            "value": pinned["products_per_s"],
            "workload": "Poisson stream, n log-uniform 2^10..2^20, 3 primes + CRT, budget 8 GiB; value: client "
                        "buffers in pinned host memory",
            "pinned_client": pinned, "pageable_client": staged,
            "pinned_over_pageable": pinned["products_per_s"] / staged["products_per_s"]}


def bigmul(args):
    """Large-integer products: 16 pairs of 2^20-limb (32 Mbit) integers, uniform limbs,
    one plan replayed as a HIP graph; checked by residues modulo two 61-bit primes and by the
    low 1000 limbs, both from CPython integers; Python's integer product timed beside it on a
    smaller sample."""
    import time as _time
    n, count = 1 << 20, 16
    gen = np.random.Generator(np.random.PCG64(7))
    pairs = [(gen.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32),
              gen.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)) for _ in range(count)]
    ctx = hntt.Context(0)
    dpairs = [(torch.from_numpy(a.view(np.int32)).cuda(), torch.from_numpy(b.view(np.int32)).cuda()) for a, b in pairs]
    outs = [torch.empty(2 * n, dtype=torch.int32, device="cuda") for _ in range(count)]
    res = {}
    for policy in _policies(args, ("lazy", "plain")):
        plain = policy == "plain"
        tuned = None if args.no_tune else autotune.tune_polymul(ctx, dpairs, outs, plain=plain, big=True)
        res[policy] = _time_plan(lambda graph: ctx.bigmul_plan(dpairs, outs, plain=plain, graph=graph), count, args)
        res[policy].update(_schedules(tuned))
    for i in (0, count - 1):
        a, b = (_as_int(v, 4) for v in pairs[i])
        c = _as_int(outs[i].cpu().numpy().view(np.uint32), 4)
        for m in _M61:
            assert c % m == (a % m) * (b % m) % m, "bigmul mismatch"
        low = (1 << (32 * 1000)) - 1
        assert c & low == ((a & low) * (b & low)) & low, "bigmul low limbs"
    ctx.close()
    ns = 1 << 19
    a, b = _as_int(pairs[0][0][:ns], 4), _as_int(pairs[0][1][:ns], 4)
    t0 = _time.perf_counter()
    _ = a * b
    cpu_s = _time.perf_counter() - t0
    bfly = count * 9 * 21 * (1 << 20)  # 9 transforms of 2^21 words per product, 21 x 2^20 butterflies each
    return {"metric": "large-integer products/s, 2^20-limb (32 Mbit) operands", "unit": "products/s",
            "roofline": _batch_roofline("bigmul", res["lazy"]["ms_per_batch"], bfly),
            "value": res["lazy"]["products_per_s"], "workload": "16 products of 2^20 x 2^20 base-2^32 limbs",
            **res, **_ratios(res, "ms_per_batch"),
            "cpu_python_int": {"seconds": cpu_s, "sample": "one product of 2^19 x 2^19 limbs (16 Mbit operands), "
                               "CPython integer multiplication, 1 core"}}


def table1(args):
    """Same-host counterpart of Table 1 (no GPU): one-core transforms of length 2^11 over the
    62-bit prime with Algorithm 2 and Algorithm 3 butterflies, time per butterfly."""
    from . import cpu
    from .workloads import G62, P62, uniform_residues
    w = hntt.root_of_unity(P62, 11)
    x = uniform_residues(8, 1 << 11, P62, np.uint64)
    r = cpu.run(x, P62, w, reps=20000)
    return {"metric": "ns per butterfly, one CPU core, L = 2^11, 62-bit p (Table 1 design)", "unit": "ns",
            "value": r["alg3"]["ns_per_butterfly"], **r,
            "paper_table1_cycles": {"Westmere": {"alg2": 10.1, "alg3": 6.9}, "Sandy Bridge": {"alg2": 9.1, "alg3": 5.9},
                                    "Piledriver": {"alg2": 13.9, "alg3": 12.0}}}


def pointwise(args):
    """hntt_pointwise_mul over 64 x 2^20 u32 residues (two reads and one write of 4 bytes per
    word): achieved bandwidth against the 8 TB/s HBM peak; the first 2^16 words checked against
    numpy's modular product."""
    from .workloads import P30, uniform_residues
    n = 64 << 20
    a_np = uniform_residues(9, n, P30, np.uint32)
    b_np = uniform_residues(10, n, P30, np.uint32)
    ctx = hntt.Context(0)
    a = torch.from_numpy(a_np.view(np.int32)).cuda()
    b = torch.from_numpy(b_np.view(np.int32)).cuda()
    c = torch.empty_like(a)
    for _ in range(3):
        ctx.pointwise_mul(a, b, c, P30)
    ms = _events_ms(lambda: ctx.pointwise_mul(a, b, c, P30), max(10, args.steps))
    got = c[: 1 << 16].cpu().numpy().view(np.uint32).astype(np.uint64)
    want = a_np[: 1 << 16].astype(np.uint64) * b_np[: 1 << 16].astype(np.uint64) % np.uint64(P30)
    assert np.array_equal(got, want), "pointwise mismatch"
    ctx.close()
    gbs = 12 * n / (ms / 1e3) / 1e9
    return {"metric": "pointwise product bandwidth, 64 x 2^20 u32 words", "unit": "GB/s", "value": gbs,
            "ms_per_call": ms, "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                                            "frac": gbs / 8000.0}}
