#!/usr/bin/env python3
"""Throughput of the lazy-butterfly NTT on one MI355X.

Workload: 64 forward + inverse NTTs of length 2^20 over p = 998244353 on 32-bit
words (omega = 3^((p-1)/2^20)), uniform residues from seed 2, already resident
in HBM.  One step = the forward transform of the whole batch followed by the
inverse (so every step starts from the same data).  The same steps are timed
again with the fully reducing (plain) butterflies of Algorithm 2 and with the
Montgomery butterflies of Algorithm 5 under the same kernel template.

Reported: butterflies/s (batch * l * L/2 per direction, counted as the paper
does) for the round trip and for each direction (median, min and max over the
steps), the roofline of the dominant kernel (HIP-event durations of the launches
inside the timed region), the HBM fraction read two ways (compulsory bytes, and
the bytes the rocprofv3 counters recorded) against both the 8 TB/s peak and a
plain device copy measured in the same process, the VALU issue rate of the
dominant kernel, the lazy/plain and lazy/Montgomery ratios, and the CPU oracle
timed on a bounded sample on the host cores (batch-parallel, and one transform
on one thread).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0               # MI355X HBM3E
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12  # 256 CUs x 64 int32 lanes/clk x 2.4 GHz = 39.3 Tops/s
# int32 VALU operations per butterfly on gfx950 (Algorithm 3: add, sub+min for the
# conditional -2p, sub+add for T, mul_hi, 2x mul_lo, sub; Algorithm 2: 12).  Only the
# paper's butterflies count as algorithmic work; the split-twiddle products of the
# two-pass decomposition are overhead of this implementation and are not counted.
OPS_BFLY = {"lazy": 9, "plain": 12}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-sample", type=int, default=128,
                    help="transforms (forward + inverse, length 2^20) in the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-mont", action="store_true", help="skip the Montgomery-butterfly (Algorithm 5) comparison")
    ap.add_argument("--no-tune", action="store_true", help="use the built-in schedule instead of the autotuner's")
    ap.add_argument("--clock-warm", type=float, default=0.5,
                    help="seconds of untimed round trips before each policy's warm-up steps, so that the "
                         "timed steps run at working clocks also when the schedule comes from the cache")
    ap.add_argument("--workload", default="batch64",
                    choices=["batch64", "single1k", "u64", "polymul", "serving", "bigmul", "table1", "pointwise"],
                    help="batch64 (default, the headline line); the others print their own JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy three times (reference for HBM byte counters)")
    return ap.parse_args()


def copy_calibration():
    """A plain device copy of known size: 1 GiB read + 1 GiB written per launch, three launches."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": src.numel() * 4, "copy_bytes_written_per_launch": dst.numel() * 4,
                      "launches": 3}))


def copy_bandwidth(reps: int = 10) -> float:
    """GB/s of a plain 1 GiB device-to-device copy (bytes read + bytes written over the
    median launch time): the practical HBM ceiling next to the 8 TB/s peak."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for i in range(reps):
        dst.copy_(src)
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(reps))[reps // 2]
    nbytes = 2 * src.numel() * 4
    del src, dst
    torch.cuda.empty_cache()
    return nbytes / (ms * 1e-3) / 1e9


def direction_times(ctx, x, p, w, policy, steps):
    """Per-step forward, inverse and round-trip times (ms) from events on the stream the
    library launches on (torch's current stream), in a run of its own."""
    import torch
    kw = {"plain": policy == "plain", "mont": policy == "mont"}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps + 1)]
    ev[0].record()
    for i in range(steps):
        ctx.ntt_forward(x, p, w, **kw)
        ev[2 * i + 1].record()
        ctx.ntt_inverse(x, p, w, **kw)
        ev[2 * i + 2].record()
    torch.cuda.synchronize()
    fwd = [ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(steps)]
    inv = [ev[2 * i + 1].elapsed_time(ev[2 * i + 2]) for i in range(steps)]
    return {"forward": fwd, "inverse": inv, "round_trip": [a + b for a, b in zip(fwd, inv)]}


def summarize_ms(ms, bfly):
    import statistics
    med = statistics.median(ms)
    return {"butterflies_per_s": bfly / (med * 1e-3), "median_ms": med, "min_ms": min(ms), "max_ms": max(ms)}


def pass_butterflies(name: str, batch: int, l: int) -> int:
    """Radix-2 butterflies in one launch of the named pass (kernel name ends in _n<log2 sub-length>)."""
    n = int(name.rsplit("_n", 1)[1])
    return batch * n * ((1 << l) // 2)


def time_steps(ctx, x, p, w, policy, steps, warmup):
    import torch
    kw = {"plain": policy == "plain", "mont": policy == "mont"}
    for _ in range(warmup):
        ctx.ntt_forward(x, p, w, **kw)
        ctx.ntt_inverse(x, p, w, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.ntt_forward(x, p, w, **kw)
        ctx.ntt_inverse(x, p, w, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # The same K steps again with a HIP event pair on the library's stream around every
    # launch, for the per-kernel durations.  The event packets add a few microseconds
    # per launch, so the step time above is taken without them.
    ctx.trace_reset()
    ctx.trace(True)
    for _ in range(steps):
        ctx.ntt_forward(x, p, w, **kw)
        ctx.ntt_inverse(x, p, w, **kw)
    torch.cuda.synchronize()
    ctx.trace(False)
    kernels = ctx.trace_read()
    return (t1 - t0) / steps, kernels


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_64x2^20_u32.json")


def measured_counter(kernel: str, field: str = "bytes_per_launch"):
    """A per-launch figure for `kernel` from the committed rocprofv3 counters (HBM bytes, or VALU
    wave instructions with field="valu_insts_per_launch"), or None when the kernel sources
    changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return rec.get(field, {}).get(kernel)


CPU_SHARE_PER_GPU = 16


def cpu_baseline(cfg, w, x_np, sample):
    import numpy as np
    import oracle
    orc = oracle.Oracle()
    # one thread per core of this GPU's share of the host: 16 cores per GPU (the share a
    # one-GPU job may occupy), fewer if the process may run on fewer
    allowed = len(os.sched_getaffinity(0))
    cores = min(CPU_SHARE_PER_GPU, allowed)
    l, p = cfg.log2_len, cfg.p
    rows = [x_np[i % x_np.shape[0]].astype(np.uint64) for i in range(sample)]

    def work(a):
        orc.lib.oracle_ntt_forward(oracle._ptr(a), l, p, w)
        f = a.copy()
        orc.lib.oracle_ntt_inverse(oracle._ptr(a), l, p, w)
        return f

    one = rows[0].copy()
    t0 = time.perf_counter()
    work(one)
    single = time.perf_counter() - t0
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        fwd = list(ex.map(work, rows))
    wall = time.perf_counter() - t0
    bfly = sample * 2 * l * (1 << (l - 1))
    return {"value": bfly / wall, "unit": "butterflies/s", "cores": cores, "kind": "oracle",
            "sample": f"{sample} of the 64 transforms (length 2^20), forward + inverse, one transform per "
                      f"thread, {cores} threads, {wall:.2f} s wall", "wall_s": wall,
            "single_thread": {"value": 2 * l * (1 << (l - 1)) / single, "unit": "butterflies/s",
                              "sample": "one transform, forward + inverse, on one thread", "wall_s": single},
            "cpu_model": cpu_model(), "host_cores_total": os.cpu_count(), "host_cores_allowed": allowed,
            "cores_note": f"{cores} threads: the CPU share of one GPU on this host "
                          f"({os.cpu_count()} logical cores in total, {allowed} allowed to this process)"}, fwd, rows


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: every transform batch here fits one MI355X and this build has no "
              "multi-GPU path (independent batches would shard by descriptor with no communication). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload != "batch64":
        from paper_1205_2926_amd import bench_workloads
        print(json.dumps(getattr(bench_workloads, args.workload)(args)))
        return

    import numpy as np
    import torch

    from paper_1205_2926_amd import hntt
    from paper_1205_2926_amd.workloads import BATCH64_1M

    cfg = BATCH64_1M
    l, p = cfg.log2_len, cfg.p
    w = hntt.root_of_unity(p, l)
    x_np = cfg.data()
    x = torch.from_numpy(x_np.view(np.int32)).cuda()
    ctx = hntt.Context(0)

    # correctness gate on the benchmark's own launches: the round trip is exact
    ctx.ntt_forward(x, p, w)
    fwd0 = x[0].cpu().numpy().view(np.uint32).copy()
    ctx.ntt_inverse(x, p, w)
    assert np.array_equal(x.cpu().numpy().view(np.uint32), x_np), "round trip mismatch"

    bfly_step = 2 * cfg.butterflies
    copy_gbs = copy_bandwidth()
    res = {}
    schedules = {}
    from paper_1205_2926_amd import autotune
    policies = ["lazy"] + ([] if args.no_plain else ["plain"]) + ([] if args.no_mont else ["mont"])
    for policy in policies:
        if args.no_tune:
            ctx.set_tuning(l, cfg.word_bits)
        else:  # each butterfly gets its own best schedule (cached per GPU and shape)
            autotune.tune(ctx, x, p, w, policy=policy)
        schedules[policy] = ctx.get_plan(l, cfg.word_bits)
        autotune.warm(ctx, x, p, w, policy, args.clock_warm)
        sec, kernels = time_steps(ctx, x, p, w, policy, args.steps, args.warmup)
        res[policy] = (sec, kernels)
    # the other policies once more under the lazy schedule: the butterflies alone compared
    same = {}
    sched = schedules["lazy"]
    ctx.set_tuning(l, cfg.word_bits, sched["g_cols"], sched["g_rows"], sched["batch_chunk"], sched["row_log2"],
                   sched["g_rows_inv"])
    for policy in policies[1:]:
        same[policy] = time_steps(ctx, x, p, w, policy, args.steps, args.warmup)[0]
    # forward and inverse apart, per step, under the lazy schedule
    dirs = direction_times(ctx, x, p, w, "lazy", args.steps)
    assert np.array_equal(x.cpu().numpy().view(np.uint32), x_np), "data changed across steps"

    sec, kernels = res["lazy"]
    value = bfly_step / sec
    # roofline of the dominant kernel (largest total time in the timed region)
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    avg_s = kernels[dom]["total_ms"] / kernels[dom]["launches"] / 1e3
    bfly = pass_butterflies(dom, cfg.batch, l)
    bytes_alg = 2 * (cfg.word_bits // 8) * cfg.batch * (1 << l)
    ops_alg = bfly * OPS_BFLY["lazy"]
    hbm = {"bound": "hbm", "achieved": bytes_alg / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    alu = {"bound": "alu", "achieved": ops_alg / avg_s / 1e12, "peak": VALU_PEAK_TOPS, "unit": "Tops/s"}
    for r in (hbm, alu):
        r["frac"] = r["achieved"] / r["peak"]
    roof = dict(max((hbm, alu), key=lambda r: r["frac"]))
    roof.update({"kernel": dom, "avg_launch_ms": avg_s * 1e3, "traffic": measured_counter(dom),
                 "algorithmic_bytes": bytes_alg, "algorithmic_ops": ops_alg,
                 "other": (alu if roof["bound"] == "hbm" else hbm)})

    # HBM read two ways (compulsory bytes; bytes the rocprofv3 counters recorded for these
    # kernels), each against the 8 TB/s peak and against the copy measured above
    step_bytes = {"compulsory": 2 * bytes_alg}
    per_launch = {k: measured_counter(k) for k in kernels}
    step_bytes["measured"] = (None if None in per_launch.values() else
                              sum(per_launch[k] * v["launches"] for k, v in kernels.items()) / args.steps)
    hbm_read = {"copy_GBs": copy_gbs, "peak_GBs": HBM_PEAK_GBS}
    for kind, b in step_bytes.items():
        hbm_read[kind] = None if b is None else {
            "bytes_per_step": b, "GBs": b / sec / 1e9,
            "frac_of_peak": b / sec / 1e9 / HBM_PEAK_GBS, "frac_of_copy": b / sec / 1e9 / copy_gbs}
    insts = measured_counter(dom, "valu_insts_per_launch")
    valu = {"kernel": dom, "wave_insts_per_launch": insts,
            "issue_frac": None if insts is None else insts / (256 * 2.4e9 * avg_s),
            "definition": "wave64 VALU instructions (SQ_INSTS_VALU) / (256 CUs x 1 per clock x 2.4 GHz "
                          "x average launch time)"}

    out = {
        "metric": "NTT butterflies/s + %HBM roofline (L=2^20x64, 30-bit p), lazy vs plain",
        "value": value,
        "unit": "butterflies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic: uniform residues in [0,p) from numpy PCG64 seed 2",
        "config": {"workload": "64 forward+inverse NTTs, L=2^20, p=998244353, 32-bit words, lazy butterflies",
                   "batch": cfg.batch, "log2_len": l, "p": p, "omega": w, "word_bits": cfg.word_bits},
        "roofline": roof,
        "hbm_frac_compulsory": (2 * bytes_alg) / sec / 1e9 / HBM_PEAK_GBS,
        "hbm": hbm_read,
        "valu": valu,
        "directions": {k: summarize_ms(v, cfg.butterflies * (2 if k == "round_trip" else 1))
                       for k, v in dirs.items()},
        "kernels_ms": {k: v["total_ms"] / v["launches"] for k, v in kernels.items()},
        "schedule": schedules.get("lazy"),
    }
    for other in ("plain", "mont"):
        if other in res:
            psec, pk = res[other]
            out[other] = {"value": bfly_step / psec, "ms_per_step": psec * 1e3, "schedule": schedules[other],
                          "kernels_ms": {k: v["total_ms"] / v["launches"] for k, v in pk.items()}}
            out[f"lazy_over_{other}"] = psec / sec
            out[f"lazy_over_{other}_same_schedule"] = same[other] / sec
    if not args.no_cpu_baseline:
        cb, fwd, rows = cpu_baseline(cfg, w, x_np, args.cpu_sample)
        assert np.array_equal(fwd[0], fwd0.astype(np.uint64)), "GPU forward differs from the oracle"
        out["cpu_baseline"] = cb
        out["gpu_over_cpu"] = value / cb["value"]
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
