"""The serving loop: continuous batching within an HBM budget, results identical alone and in the mix."""
import random

import numpy as np
import pytest

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


def test_mixed_stream_within_budget_and_alone_equals_mix(ctx, orc):
    """A Poisson stream of mixed sizes through a budget that forces waiting: every request
    completes, memory never exceeds the budget, several batches overlap, and each result
    equals the oracle and, bit for bit, the same request served alone."""
    reqs = make_requests(seed=5, count=48, rate_per_s=4000.0, lo_bits=10, hi_bits=16)
    budget = 24 << 20
    srv = PolymulServer(ctx, budget, streams=3, max_batch=8)
    stats = srv.run(reqs, time_limit=120)
    assert stats["completed"] == len(reqs) and stats["rejected"] == 0
    assert stats["peak_bytes"] <= budget
    assert stats["batches"] > 1
    for r in reqs:
        _check(orc, r, full=r.nout < 3000)
    for r in reqs[:: 7]:
        alone = Request(r.rid, 0.0, r.a, r.b)
        PolymulServer(ctx, budget, streams=1, max_batch=1).run([alone], time_limit=60)
        np.testing.assert_array_equal(alone.result, r.result)


def test_request_larger_than_budget_is_rejected(ctx, orc):
    big = Request(0, 0.0, np.ones(1 << 16, np.uint32), np.ones(1 << 16, np.uint32))
    small = Request(1, 0.0, np.arange(100, dtype=np.uint32), np.arange(50, dtype=np.uint32))
    srv = PolymulServer(ctx, 1 << 20, streams=2)
    stats = srv.run([big, small], time_limit=60)
    assert stats["rejected"] == 1 and srv.rejected[0] is big
    _check(orc, small, full=True)


def test_large_requests_up_to_2e20(ctx, orc):
    """The largest requests of the serving workload (n up to 2^20 coefficients)."""
    reqs = make_requests(seed=6, count=6, rate_per_s=1000.0, lo_bits=19, hi_bits=20)
    srv = PolymulServer(ctx, 1 << 30, streams=2, max_batch=2)
    stats = srv.run(reqs, time_limit=120)
    assert stats["completed"] == len(reqs)
    for r in reqs:
        _check(orc, r)


def test_client_result_buffers(ctx, orc):
    """Requests that bring their own result buffers get the same products, written in place."""
    reqs = make_requests(seed=7, count=12, rate_per_s=4000.0, lo_bits=10, hi_bits=15, client_out=True)
    ref = make_requests(seed=7, count=12, rate_per_s=4000.0, lo_bits=10, hi_bits=15)
    PolymulServer(ctx, 64 << 20, streams=2, max_batch=4).run(reqs, time_limit=60)
    PolymulServer(ctx, 64 << 20, streams=2, max_batch=4).run(ref, time_limit=60)
    for r, q in zip(reqs, ref):
        assert np.shares_memory(r.result, r.out)
        np.testing.assert_array_equal(r.result, q.result)
        _check(orc, r, full=r.nout < 3000)
