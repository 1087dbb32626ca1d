"""Three-prime polynomial products on the GPU against the oracle (exact integers)."""
import random

import numpy as np
import pytest
import torch

import oracle
from paper_1205_2926_amd import hntt
from paper_1205_2926_amd.workloads import CRT_PRIMES, polymul_pairs, rng
from tests.gpu_util import dev, host

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


def _run(ctx, pairs, plain=False, graph=True):
    dpairs = [(dev(a), dev(b)) for a, b in pairs]
    outs = [torch.empty(a.size + b.size - 1, dtype=torch.int64, device="cuda") for a, b in pairs]
    ctx.polymul_crt(dpairs, outs, plain=plain, graph=graph)
    return [host(o, np.uint64) for o in outs]


def test_small_products_exact(ctx, orc):
    """Ragged and extreme shapes, full 32-bit coefficients where the product still fits 64 bits."""
    r = rng(40)
    shapes = [(1, 1), (1, 9), (9, 1), (2, 2), (3, 1000), (1000, 3), (64, 64), (100, 37), (2049, 2048), (4096, 4097),
              (5000, 17)]
    pairs = []
    for na, nb in shapes:
        bits = 20 if max(na, nb) > 8 else 30
        pairs.append((r.integers(0, 1 << bits, size=na, dtype=np.uint32), r.integers(0, 1 << bits, size=nb,
                                                                                    dtype=np.uint32)))
    pairs.append((np.full(7, (1 << 32) - 1, np.uint32), np.full(3, (1 << 31) - 1, np.uint32)))
    got = _run(ctx, pairs)
    for (a, b), g in zip(pairs, got):
        np.testing.assert_array_equal(g, orc.schoolbook(a, b), err_msg=f"{a.size}x{b.size}")


@pytest.mark.parametrize("plain", [False, True], ids=["lazy", "plain"])
def test_uneven_batch_one_call(ctx, orc, plain):
    """A few hundred products with log-uniform lengths 2^8..2^16 in one call (graph replay):
    whole products against the oracle's three-prime CRT for a spread of lengths, single
    coefficients against the definition for every product, and evaluation at a random
    point mod 2^61-1 (Schwartz-Zippel) for every product."""
    pairs = polymul_pairs(seed=41, pairs=300)
    got = _run(ctx, pairs, plain=plain)
    order = sorted(range(len(pairs)), key=lambda i: pairs[i][0].size)
    for i in order[:: max(1, len(order) // 12)]:
        a, b = pairs[i]
        np.testing.assert_array_equal(got[i], orc.polymul_exact(a, b, CRT_PRIMES), err_msg=f"pair {i}")
    rr = random.Random(42)
    for i, ((a, b), g) in enumerate(zip(pairs, got)):
        for k in (0, g.size - 1, rr.randrange(g.size)):
            assert int(g[k]) == orc.product_coeff(a, b, k), (i, k)
        x = rr.randrange(1, M61)
        assert orc.poly_eval(g, x, M61) == orc.poly_eval(a, x, M61) * orc.poly_eval(b, x, M61) % M61, i


def test_uneven_batch_4096_pairs(ctx, orc):
    """The full uneven workload: 4096 pairs, n log-uniform in 2^8..2^16, coefficients below
    2^20, three primes + CRT in one graph launch.  Checked by evaluation at a random point
    for every product, sampled coefficients, and whole products for a subset."""
    pairs = polymul_pairs(seed=4, pairs=4096)
    got = _run(ctx, pairs)
    rr = random.Random(43)
    for i, ((a, b), g) in enumerate(zip(pairs, got)):
        x = rr.randrange(1, M61)
        assert orc.poly_eval(g, x, M61) == orc.poly_eval(a, x, M61) * orc.poly_eval(b, x, M61) % M61, i
        k = rr.randrange(g.size)
        assert int(g[k]) == orc.product_coeff(a, b, k), (i, k)
    for i in range(0, 4096, 512):
        a, b = pairs[i]
        np.testing.assert_array_equal(got[i], orc.polymul_exact(a, b, CRT_PRIMES), err_msg=f"pair {i}")


def test_graph_replays_match_eager(ctx, orc):
    """A recorded plan replayed several times, with eager work and synchronisation between
    replays, gives the eager (non-graph) result every time."""
    pairs = polymul_pairs(seed=44, pairs=64, lo_bits=8, hi_bits=14)
    dpairs = [(dev(a), dev(b)) for a, b in pairs]
    outs_e = [torch.empty(a.size + b.size - 1, dtype=torch.int64, device="cuda") for a, b in pairs]
    ctx.polymul_crt(dpairs, outs_e, graph=False)
    eager = [host(o, np.uint64) for o in outs_e]
    outs = [torch.zeros_like(o) for o in outs_e]
    plan = ctx.polymul_plan(dpairs, outs)
    try:
        assert plan.exec_mode == "not executed"
        for rep in range(4):
            for o in outs:
                o.zero_()
            plan.execute()
            assert plan.exec_mode == "graph"  # one graph launch, not the kernel-by-kernel fallback
            torch.cuda.synchronize()
            scratch = torch.arange(1 << 20, device="cuda").sum()  # unrelated eager work between replays
            assert int(scratch) == (1 << 20) * ((1 << 20) - 1) // 2
            for o, e in zip(outs, eager):
                np.testing.assert_array_equal(host(o, np.uint64), e, err_msg=f"replay {rep}")
    finally:
        plan.destroy()
    a, b = pairs[5]
    np.testing.assert_array_equal(eager[5], orc.polymul_exact(a, b, CRT_PRIMES))


def test_plan_exec_mode_reports_direct_launches(ctx, orc):
    """A plan made without the graph, or executed while launches are traced, reports that its
    kernels were launched one by one, and gives the same products."""
    pairs = polymul_pairs(seed=46, pairs=8, lo_bits=8, hi_bits=12)
    dpairs = [(dev(a), dev(b)) for a, b in pairs]
    outs = [torch.empty(a.size + b.size - 1, dtype=torch.int64, device="cuda") for a, b in pairs]
    plan = ctx.polymul_plan(dpairs, outs, graph=False)
    try:
        plan.execute()
        assert plan.exec_mode == "direct"
    finally:
        plan.destroy()
    direct = [host(o, np.uint64) for o in outs]
    plan = ctx.polymul_plan(dpairs, outs)
    try:
        ctx.trace(True)
        plan.execute()
        torch.cuda.synchronize()
        ctx.trace(False)
        assert plan.exec_mode == "direct"  # tracing times each launch, so the graph is not used
        plan.execute()
        torch.cuda.synchronize()
        assert plan.exec_mode == "graph"
    finally:
        ctx.trace(False)
        ctx.trace_reset()
        plan.destroy()
    for o, d, (a, b) in zip(outs, direct, pairs):
        np.testing.assert_array_equal(host(o, np.uint64), d)
        np.testing.assert_array_equal(d, orc.polymul_exact(a, b, CRT_PRIMES))


def test_plan_with_caller_workspace(ctx, orc):
    pairs = polymul_pairs(seed=45, pairs=16, lo_bits=10, hi_bits=13)
    dpairs = [(dev(a), dev(b)) for a, b in pairs]
    outs = [torch.empty(a.size + b.size - 1, dtype=torch.int64, device="cuda") for a, b in pairs]
    probe = ctx.polymul_plan(dpairs, outs, graph=False)
    need = probe.workspace_bytes
    probe.destroy()
    ws = torch.empty(need // 8 + 64, dtype=torch.int64, device="cuda")
    plan = ctx.polymul_plan(dpairs, outs, workspace=ws)
    plan.execute()
    got = [host(o, np.uint64) for o in outs]
    plan.destroy()
    for (a, b), g in zip(pairs, got):
        np.testing.assert_array_equal(g, orc.polymul_exact(a, b, CRT_PRIMES))
    small = torch.empty(need // 16, dtype=torch.int64, device="cuda")
    with pytest.raises(hntt.HnttError):
        ctx.polymul_plan(dpairs, outs, workspace=small)
