"""Host-side logic of bench.py: the one-GPU rule, the committed counter record and the
summaries it prints (no GPU needed)."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_pass_butterflies(bench):
    # a ten-stage pass over 64 transforms of length 2^20 runs 64 * 10 * 2^19 butterflies
    assert bench.pass_butterflies("cols_inv_lazy_u32_n10", 64, 20) == 64 * 10 * (1 << 19)


def test_summaries_use_the_median(bench):
    s = bench.summarize_ms([3.0, 1.0, 2.0], 1000)
    assert (s["median_ms"], s["min_ms"], s["max_ms"]) == (2.0, 1.0, 3.0)
    assert s["butterflies_per_s"] == pytest.approx(1000 / 2e-3)


def test_counter_record_matches_the_kernel_sources(bench):
    # the committed rocprofv3 record is only used while the sources it was taken on are unchanged
    for k in ("cols_fwd_lazy_u32_n10", "cols_inv_lazy_u32_n10", "rows_fwd_lazy_u32_n10", "rows_inv_lazy_u32_n10"):
        b = bench.measured_counter(k)
        v = bench.measured_counter(k, "valu_insts_per_launch")
        if b is None:
            pytest.skip("kernel sources changed since the counters were taken")
        # at least the compulsory bytes (read and write 64 x 2^20 words of 4 bytes)
        assert b >= 2 * 4 * 64 * (1 << 20)
        assert v > 0
    assert bench.measured_counter("no_such_kernel") is None


def test_counter_record_is_dropped_when_sources_change(bench, tmp_path, monkeypatch):
    import json
    rec = json.load(open(bench.TRAFFIC_FILE))
    rec["source_sha256"] = "0" * 64
    f = tmp_path / "rec.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_counter("cols_inv_lazy_u32_n10") is None


def test_workload_product_check_accepts_products_and_rejects_corruption():
    # the check the workload benchmarks run on GPU results, exercised here on the oracle's
    # schoolbook products (one short enough for the exact comparison, one long one)
    import numpy as np
    import oracle
    from paper_1205_2926_amd import bench_workloads as bw
    orc = oracle.Oracle()
    rng = np.random.Generator(np.random.PCG64(21))
    short = (rng.integers(0, 1 << 20, 300).astype(np.uint32), rng.integers(0, 1 << 20, 200).astype(np.uint32))
    long_ = (rng.integers(0, 1 << 20, 9000).astype(np.uint32), rng.integers(0, 1 << 20, 5000).astype(np.uint32))
    cases = [(short, orc.schoolbook(*short)),
             (long_, orc.schoolbook(*long_))]
    for (a, b), c in cases:
        c = np.asarray(c, dtype=np.uint64)
        assert bw._product_ok(a, b, c)
        for k in (0, c.size // 2, c.size - 1):
            bad = c.copy()
            bad[k] += np.uint64(1)
            assert not bw._product_ok(a, b, bad)
        assert not bw._product_ok(a, b, c[:-1])


def test_polymul_tuning_cache_key_follows_length_classes():
    # the cached schedule of a product batch is reused only for a batch with the same
    # number of products in every length class, of the same kind and policy
    import torch
    from paper_1205_2926_amd import autotune
    t = lambda n: torch.empty(n, dtype=torch.int32)
    a = [(t(100), t(3)), (t(1000), t(1000)), (t(129), t(1))]
    b = [(t(1), t(70)), (t(513), t(600)), (t(200), t(65))]  # same classes (2^8, 2^11, 2^9)
    c = [(t(100), t(3)), (t(1000), t(1000)), (t(1000), t(1))]
    assert autotune._poly_key(a, False, False) == autotune._poly_key(b, False, False)
    assert autotune._poly_key(a, False, False) != autotune._poly_key(c, False, False)
    assert autotune._poly_key(a, False, False) != autotune._poly_key(a, True, False)
    assert autotune._poly_key(a, False, False) != autotune._poly_key(a, False, True)
