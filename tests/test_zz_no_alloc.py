"""The allocation-free product entry point (hntt_polymul_crt_static) against the
allocating one (hntt_polymul_crt): bit-identical products on two calls in a row on
one stream, the second smaller; oversized batches and batches whose tables are not
resident are refused on the host."""
import numpy as np
import pytest
import torch

import oracle
from paper_1205_2926_amd import hntt
from paper_1205_2926_amd.workloads import rng
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _pairs(seed, count, lo, hi):
    r = rng(seed)
    out = []
    for _ in range(count):
        n = int(2 ** r.uniform(lo, hi))
        out.append((r.integers(0, 1 << 20, size=n, dtype=np.uint32),
                    r.integers(0, 1 << 20, size=max(1, n - int(r.integers(0, 3))), dtype=np.uint32)))
    return out


def _dev_batch(pairs):
    dpairs = [(dev(a), dev(b)) for a, b in pairs]
    outs = [torch.full((a.size + b.size - 1,), -1, dtype=torch.int64, device="cuda") for a, b in pairs]
    return dpairs, outs


@pytest.mark.parametrize("plain", [False, True], ids=["lazy", "plain"])
def test_static_matches_allocating_entry_point(plain):
    print(f"no-alloc products, plain={plain}", flush=True)
    ctx = hntt.Context(0)
    try:
        big = _pairs(900, 24, 3, 14)     # padded lengths 2^4 .. 2^15
        small = _pairs(901, 6, 1, 10)    # the second call: fewer, shorter products
        # reference results (and resident tables for every padded length) from the allocating call
        refs = []
        for pairs in (big, small):
            dp, outs = _dev_batch(pairs)
            ctx.polymul_crt(dp, outs, plain=plain)
            refs.append([host(o, np.uint64) for o in outs])
        # two static calls in a row on one stream, no synchronisation between them
        dp1, o1 = _dev_batch(big)
        dp2, o2 = _dev_batch(small)
        ctx.polymul_crt_static(dp1, o1, plain=plain)
        ctx.polymul_crt_static(dp2, o2, plain=plain)
        torch.cuda.synchronize()
        for ref, outs in zip(refs, (o1, o2)):
            for i, (r, o) in enumerate(zip(ref, outs)):
                np.testing.assert_array_equal(host(o, np.uint64), r, err_msg=f"product {i}")
        # the first batch again after the smaller one: the workspace keeps no stale state that matters
        dp3, o3 = _dev_batch(big)
        ctx.polymul_crt_static(dp3, o3, plain=plain)
        for i, (r, o) in enumerate(zip(refs[0], o3)):
            np.testing.assert_array_equal(host(o, np.uint64), r, err_msg=f"repeat product {i}")
        # and against the oracle's exact product for a few
        orc = oracle.Oracle()
        for i in (0, 5, 11):
            a, b = big[i]
            np.testing.assert_array_equal(refs[0][i], orc.schoolbook(a, b), err_msg=f"oracle {i}")
    finally:
        ctx.close()


def test_static_refuses_on_the_host():
    print("no-alloc refusals", flush=True)
    ctx = hntt.Context(0)
    try:
        # tables of this length are not resident on a fresh context: refused, nothing enqueued
        a = torch.ones(300, dtype=torch.int32, device="cuda")
        out = torch.full((599,), -7, dtype=torch.int64, device="cuda")
        with pytest.raises(hntt.HnttError) as ei:
            ctx.polymul_crt_static([(a, a)], [out])
        assert ei.value.status == hntt.EUNSUPPORTED
        assert "not resident" in ctx.last_error()
        assert int(out[0]) == -7
        # after the allocating call has built them, the same product goes through
        ctx.polymul_crt([(a, a)], [out])
        want = host(out, np.uint64).copy()
        out.fill_(-7)
        ctx.polymul_crt_static([(a, a)], [out])
        np.testing.assert_array_equal(host(out, np.uint64), want)
        # a batch above the static workspace is refused before the device is touched
        n = 1 << 19  # padded length 2^20: 24 MiB of residues per product, two products
        lens = [(n, n), (n, n)]
        assert hntt.polymul_workspace_size(lens) > hntt.STATIC_SCRATCH_BYTES
        big = torch.zeros(n, dtype=torch.int32, device="cuda")
        outs = [torch.zeros(2 * n - 1, dtype=torch.int64, device="cuda") for _ in lens]
        with pytest.raises(hntt.HnttError) as ei:
            ctx.polymul_crt_static([(big, big)] * 2, outs)
        assert ei.value.status == hntt.ENOMEM
        assert "static workspace" in ctx.last_error()
    finally:
        ctx.close()
