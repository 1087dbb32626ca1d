"""The serving loop: continuous batching within an HBM budget, results identical alone and in the mix."""
import random

import numpy as np
import pytest
import torch  # noqa: F401  (pinned host tensors)

import oracle
from paper_1205_2926_amd import hntt
from paper_1205_2926_amd.serve import PolymulServer, Request, make_requests

pytestmark = pytest.mark.gpu
M61 = (1 << 61) - 1


@pytest.fixture(scope="module")
def ctx():
    c = hntt.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle()


def _check(orc, r, full=False):
    assert r.result is not None and r.result.size == r.nout
    if full:
        np.testing.assert_array_equal(r.result, orc.schoolbook(r.a, r.b))
        return
    rr = random.Random(r.rid)
    for k in (0, r.nout - 1, rr.randrange(r.nout)):
        assert int(r.result[k]) == orc.product_coeff(r.a, r.b, k), (r.rid, k)
    x = rr.randrange(1, M61)
    assert orc.poly_eval(r.result, x, M61) == orc.poly_eval(r.a, x, M61) * orc.poly_eval(r.b, x, M61) % M61


def _alone(ctx, reqs, budget):
    """Serve each request by itself (one server, one request per run) and return the results."""
    srv = PolymulServer(ctx, budget, streams=1, max_batch=1)
    try:
        out = []
        for r in reqs:
            alone = Request(r.rid, 0.0, r.a.copy(), r.b.copy())
            st = srv.run([alone], time_limit=60)
            assert st["completed"] == 1
            out.append(alone.result)
        return out
    finally:
        srv.close()


def test_mixed_stream_within_budget_and_alone_equals_mix(ctx, orc):
    """A Poisson stream of mixed sizes through a budget that forces waiting: every request
    completes, memory never exceeds the budget, several batches are on the GPU at once, and
    each result equals the oracle and, bit for bit, the same request served alone."""
    print("serve: mixed stream", flush=True)
    reqs = make_requests(seed=5, count=48, rate_per_s=4000.0, lo_bits=10, hi_bits=16)
    budget = 24 << 20
    srv = PolymulServer(ctx, budget, streams=3, max_batch=8)
    try:
        stats = srv.run(reqs, time_limit=120)
    finally:
        srv.close()
    assert stats["completed"] == len(reqs) and stats["rejected"] == 0
    assert stats["peak_bytes"] <= budget
    assert stats["batches"] > 1
    assert stats["max_inflight"] >= 2, stats  # continuous batching: batches overlap on the device
    assert 0.0 < stats["inflight_frac"] <= 1.0
    assert 0.0 < stats["kernel_frac"] <= stats["inflight_frac"] + 1e-6
    for k in ("h2d_frac", "d2h_frac"):
        assert 0.0 < stats[k] <= stats["inflight_frac"] + 1e-6
    assert stats["h2d_GBs"] > 0.0 and stats["d2h_GBs"] > 0.0
    for r in reqs:
        _check(orc, r, full=r.nout < 3000)
    for r, res in zip(reqs, _alone(ctx, reqs, budget)):
        np.testing.assert_array_equal(res, r.result, err_msg=f"request {r.rid}")


def test_alone_equals_mix_up_to_2e20(ctx, orc):
    """A mix whose sizes reach n = 2^20 coefficients (the top of the serving workload):
    every request, served alone, gives the same bits as in the mix."""
    print("serve: mix up to 2^20", flush=True)
    reqs = make_requests(seed=8, count=10, rate_per_s=2000.0, lo_bits=10, hi_bits=20)
    reqs[-1] = Request(reqs[-1].rid, reqs[-1].arrival, np.arange(1 << 20, dtype=np.uint32) % (1 << 20),
                       np.full(1 << 20, (1 << 20) - 1, np.uint32))
    budget = 1 << 30
    srv = PolymulServer(ctx, budget, streams=3, max_batch=4)
    try:
        stats = srv.run(reqs, time_limit=120)
    finally:
        srv.close()
    assert stats["completed"] == len(reqs)
    assert max(r.a.size for r in reqs) == 1 << 20
    for r in reqs:
        _check(orc, r, full=r.nout < 3000)
    for r, res in zip(reqs, _alone(ctx, reqs, budget)):
        np.testing.assert_array_equal(res, r.result, err_msg=f"request {r.rid} (n={r.a.size})")


def test_request_larger_than_budget_is_rejected(ctx, orc):
    big = Request(0, 0.0, np.ones(1 << 16, np.uint32), np.ones(1 << 16, np.uint32))
    small = Request(1, 0.0, np.arange(100, dtype=np.uint32), np.arange(50, dtype=np.uint32))
    srv = PolymulServer(ctx, 1 << 20, streams=2)
    try:
        stats = srv.run([big, small], time_limit=60)
    finally:
        srv.close()
    assert stats["rejected"] == 1 and srv.rejected[0] is big
    _check(orc, small, full=True)


def test_large_requests_up_to_2e20(ctx, orc):
    """The largest requests of the serving workload (n up to 2^20 coefficients)."""
    reqs = make_requests(seed=6, count=6, rate_per_s=1000.0, lo_bits=19, hi_bits=20)
    srv = PolymulServer(ctx, 1 << 30, streams=2, max_batch=2)
    try:
        stats = srv.run(reqs, time_limit=120)
    finally:
        srv.close()
    assert stats["completed"] == len(reqs)
    for r in reqs:
        _check(orc, r)


def test_client_result_buffers(ctx, orc):
    """Requests that bring their own result buffers get the same products, written in place."""
    reqs = make_requests(seed=7, count=12, rate_per_s=4000.0, lo_bits=10, hi_bits=15, client_out=True)
    ref = make_requests(seed=7, count=12, rate_per_s=4000.0, lo_bits=10, hi_bits=15)
    for rs in (reqs, ref):
        srv = PolymulServer(ctx, 64 << 20, streams=2, max_batch=4)
        try:
            srv.run(rs, time_limit=60)
        finally:
            srv.close()
    for r, q in zip(reqs, ref):
        assert np.shares_memory(r.result, r.out)
        np.testing.assert_array_equal(r.result, q.result)
        _check(orc, r, full=r.nout < 3000)


def test_pinned_client_buffers_mixed_with_staged(ctx, orc):
    """Requests whose operands and result buffers are pinned host memory are copied straight
    to and from the device; mixed in one stream with staged requests, every product equals
    the staged path's, bit for bit."""
    print("serve: pinned client buffers", flush=True)
    pinned = make_requests(seed=9, count=16, rate_per_s=8000.0, lo_bits=10, hi_bits=17, pinned=True)
    staged = make_requests(seed=9, count=16, rate_per_s=8000.0, lo_bits=10, hi_bits=17)
    mix = [p if i % 2 else s for i, (p, s) in enumerate(zip(pinned, staged))]
    srv = PolymulServer(ctx, 256 << 20, streams=3, max_batch=6)
    try:
        stats = srv.run(mix, time_limit=60)
    finally:
        srv.close()
    assert stats["completed"] == len(mix)
    ref = make_requests(seed=9, count=16, rate_per_s=8000.0, lo_bits=10, hi_bits=17)
    for r, res in zip(ref, _alone(ctx, ref, 256 << 20)):
        r.result = res
    for r, q in zip(mix, ref):
        if r.direct:
            assert np.shares_memory(r.result, r.pinned[2].numpy())
        np.testing.assert_array_equal(r.result, q.result, err_msg=f"request {r.rid}")
        _check(orc, r, full=r.nout < 3000)


def test_pinned_request_checks():
    a = np.arange(10, dtype=np.uint32)
    with pytest.raises(ValueError):
        Request(0, 0.0, a, a, np.zeros(19, np.uint64), pinned=(None, None, None))
