"""Large-integer multiplication on the GPU (three-prime product + device carry scan)
against the oracle: long multiplication for small operands, Python's integer product
for larger ones, residues modulo 61-bit primes for the largest."""
import random

import numpy as np
import pytest
import torch

import oracle
from paper_1205_2926_amd import hntt
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu
ALL = 0xFFFFFFFF


@pytest.fixture(scope="module")
def ctx():
    c = hntt.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle()


def _limbs(r, n, hi=1 << 32):
    return np.array([r.randrange(hi) for _ in range(n)], np.uint32)


def _run(ctx, pairs, plain=False, graph=True):
    dpairs = [(dev(a), dev(b)) for a, b in pairs]
    outs = [torch.empty(a.size + b.size, dtype=torch.int32, device="cuda") for a, b in pairs]
    ctx.bigmul(dpairs, outs, plain=plain, graph=graph)
    return [host(o, np.uint32) for o in outs]


@pytest.mark.parametrize("plain", [False, True], ids=["lazy", "plain"])
def test_small_shapes_against_long_multiplication(ctx, orc, plain):
    r = random.Random(60)
    shapes = [(1, 1), (1, 9), (9, 1), (2, 2), (3, 1000), (1000, 3), (64, 64), (100, 37), (1025, 1023),
              (2049, 2048), (4096, 4097), (5000, 17)]
    pairs = [(_limbs(r, na), _limbs(r, nb)) for na, nb in shapes]
    got = _run(ctx, pairs, plain=plain)
    for (a, b), g in zip(pairs, got):
        np.testing.assert_array_equal(g, orc.bigmul_schoolbook(a, b), err_msg=f"{a.size}x{b.size}")


def test_carry_chains(ctx, orc):
    """Operands that make long runs of all-ones limbs and carries crossing many chunks:
    (beta^n - 1)^2, a (beta^m - 1) for random a, alternating limbs, zeros and ones."""
    r = random.Random(61)
    cases = []
    for n in (1, 5, 1000, 1 << 14):
        ones = np.full(n, ALL, np.uint32)
        cases.append((ones, ones))
    for na, m in ((3000, 5000), (70000, 9000)):
        cases.append((_limbs(r, na), np.full(m, ALL, np.uint32)))
    alt = np.array([ALL, 0] * 5000, np.uint32)
    cases.append((alt, alt[::-1].copy()))
    cases.append((np.zeros(4000, np.uint32), _limbs(r, 3000)))
    cases.append((np.array([1], np.uint32), _limbs(r, 7777)))
    got = _run(ctx, cases)
    for (a, b), g in zip(cases, got):
        np.testing.assert_array_equal(g, orc.bigmul(a, b), err_msg=f"{a.size}x{b.size}")
    n = 1 << 14
    want = np.array([1] + [0] * (n - 1) + [ALL - 1] + [ALL] * (n - 1), np.uint32)
    np.testing.assert_array_equal(got[3], want)


def test_uneven_batch_one_call(ctx, orc):
    """A batch of products with log-uniform limb counts 2^4..2^16 in one call (graph replay),
    each against Python's integer product."""
    r = random.Random(62)
    pairs = []
    for i in range(40):
        na = int(2 ** r.uniform(4, 16))
        nb = int(2 ** r.uniform(4, 16)) if i % 3 else na
        pairs.append((_limbs(r, na), _limbs(r, nb)))
    got = _run(ctx, pairs)
    for i, ((a, b), g) in enumerate(zip(pairs, got)):
        np.testing.assert_array_equal(g, orc.bigmul(a, b), err_msg=f"product {i}")
    again = _run(ctx, pairs, graph=False)
    for g, h in zip(got, again):
        np.testing.assert_array_equal(g, h)


def test_largest_operands(ctx, orc):
    """Operands of 2^22 limbs (128 Mbit each), the largest the three primes support:
    residues modulo three 61-bit primes and the low 2000 limbs against the oracle."""
    r = random.Random(63)
    n = 1 << 22
    gen = np.random.Generator(np.random.PCG64(64))
    a = gen.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    b = gen.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    b[-5:] = ALL
    (g,) = _run(ctx, [(a, b)])
    for m in (2305843009213693951, 2305843009213693921, 2305843009213693907):
        assert orc.limbs_mod(g, m) == orc.limbs_mod(a, m) * orc.limbs_mod(b, m) % m, m
    k = 2000
    np.testing.assert_array_equal(g[:k], orc.bigmul(a[:k], b[:k])[:k])
    assert g[-1] != 0 or g[-2] != 0


def test_plan_with_caller_workspace_and_replays(ctx, orc):
    r = random.Random(65)
    pairs = [(_limbs(r, 3000 + 17 * i), _limbs(r, 2000 + 31 * i)) for i in range(6)]
    dpairs = [(dev(a), dev(b)) for a, b in pairs]
    outs = [torch.zeros(a.size + b.size, dtype=torch.int32, device="cuda") for a, b in pairs]
    need = hntt.bigmul_workspace_size([(a.size, b.size) for a, b in pairs])
    ws = torch.empty(need // 8 + 64, dtype=torch.int64, device="cuda")
    plan = ctx.bigmul_plan(dpairs, outs, workspace=ws)
    try:
        assert plan.workspace_bytes == need
        for rep in range(3):
            for o in outs:
                o.zero_()
            plan.execute()
            torch.cuda.synchronize()
            for (a, b), o in zip(pairs, outs):
                np.testing.assert_array_equal(host(o, np.uint32), orc.bigmul(a, b), err_msg=f"replay {rep}")
    finally:
        plan.destroy()
