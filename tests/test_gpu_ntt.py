"""HIP transforms against the CPU oracle, element by element (bit-exact: this is exact
integer work, so every fully reduced output must equal the oracle's)."""
import random

import numpy as np
import pytest
import torch

import oracle
from paper_1205_2926_amd import hntt
from paper_1205_2926_amd.workloads import (BATCH8_4M_U64, BATCH64_1M, CRT_PRIMES, G30, G62, P30, P62, SINGLE_1K,
                                           uniform_residues)
from tests.gpu_util import dev, host, rev
from tests.oracle_pins import naive_dft, to_bitrev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = hntt.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle()


def _np_dtype(wb):
    return np.uint32 if wb == 32 else np.uint64


def _omega(orc, p, g, l):
    w = orc.root_of_unity(p, g, l)
    assert w == hntt.root_of_unity(p, l)
    return w


POLICIES = ["lazy", "plain", "mont"]  # Algorithms 3/4, 2, and 5 (with its inverse counterpart)


def _kw(policy):
    return {"plain": policy == "plain", "mont": policy == "mont"}


# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("policy", POLICIES)
def test_single_1k(ctx, orc, policy):
    """One forward NTT of 1024 residues mod 998244353 with omega = 3^((p-1)/1024):
    bit-exact against the oracle and the naive DFT, output bit-reversed in [0,p)."""
    cfg = SINGLE_1K
    x = cfg.data()[0]
    w = _omega(orc, cfg.p, cfg.g, cfg.log2_len)
    assert w == 258648936
    t = dev(x)
    ctx.ntt_forward(t, cfg.p, w, **_kw(policy))
    got = host(t, np.uint32)
    ref = orc.forward(x, cfg.log2_len, cfg.p, w)
    np.testing.assert_array_equal(got.astype(np.uint64), ref)
    assert got.tolist() == to_bitrev(naive_dft(x.tolist(), cfg.p, w))
    ctx.ntt_inverse(t, cfg.p, w, **_kw(policy))
    np.testing.assert_array_equal(host(t, np.uint32), x)


LENGTHS_32 = [(l, P30, G30) for l in range(1, 24)] + [(24, 167772161, 3)]
LENGTHS_64 = [(l, P62, G62) for l in range(1, 23)]


@pytest.mark.parametrize("policy", POLICIES)
@pytest.mark.parametrize("wb,l,p,g", [(32, *c) for c in LENGTHS_32] + [(64, *c) for c in LENGTHS_64],
                         ids=lambda v: str(v))
def test_every_length(ctx, orc, wb, l, p, g, policy):
    """Forward and inverse at every length from 2 up to the two-pass limit, several
    tiles and ragged batch sizes, against the oracle."""
    batch = 3 if l <= 14 else 1
    w = _omega(orc, p, g, l)
    x = uniform_residues(100 + l, (batch, 1 << l), p, _np_dtype(wb))
    t = dev(x)
    ctx.ntt_forward(t, p, w, **_kw(policy))
    np.testing.assert_array_equal(host(t, _np_dtype(wb)).astype(np.uint64), orc.forward(x, l, p, w))
    y = uniform_residues(200 + l, (batch, 1 << l), p, _np_dtype(wb))
    u = dev(y)
    ctx.ntt_inverse(u, p, w, **_kw(policy))
    np.testing.assert_array_equal(host(u, _np_dtype(wb)).astype(np.uint64), orc.inverse(y, l, p, w))
    ctx.ntt_forward(u, p, w, **_kw(policy))
    np.testing.assert_array_equal(host(u, _np_dtype(wb)), y)


def _sampled_points(orc, x, got, l, p, w, per_row, seed):
    r = random.Random(seed)
    for b in range(x.shape[0]):
        for j in [0, (1 << l) - 1] + [r.randrange(1 << l) for _ in range(per_row - 2)]:
            assert int(got[b, rev(j, l)]) == orc.dft_point(x[b], l, p, w, j), (b, j)


def test_headline_batch64_lazy_vs_plain(ctx, orc):
    """64 forward+inverse NTTs of length 2^20 mod 998244353 (the benchmark's workload, same
    launches): lazy, plain and Montgomery agree bit for bit, whole transforms match the
    oracle on a subset, every transform matches the definition at sampled outputs, and the
    round trip returns the input exactly."""
    cfg = BATCH64_1M
    x = cfg.data()
    l, p = cfg.log2_len, cfg.p
    w = _omega(orc, p, cfg.g, l)
    assert w == 565042129
    t_lazy, t_plain, t_mont = dev(x), dev(x), dev(x)
    ctx.ntt_forward(t_lazy, p, w)
    ctx.ntt_forward(t_plain, p, w, plain=True)
    ctx.ntt_forward(t_mont, p, w, mont=True)
    got = host(t_lazy, np.uint32)
    np.testing.assert_array_equal(got, host(t_plain, np.uint32))
    np.testing.assert_array_equal(got, host(t_mont, np.uint32))
    for b in (0, 17, 63):
        np.testing.assert_array_equal(got[b].astype(np.uint64), orc.forward(x[b], l, p, w))
    _sampled_points(orc, x, got, l, p, w, per_row=3, seed=5)
    ctx.ntt_inverse(t_lazy, p, w)
    ctx.ntt_inverse(t_plain, p, w, plain=True)
    ctx.ntt_inverse(t_mont, p, w, mont=True)
    np.testing.assert_array_equal(host(t_lazy, np.uint32), x)
    np.testing.assert_array_equal(host(t_plain, np.uint32), x)
    np.testing.assert_array_equal(host(t_mont, np.uint32), x)


def test_u64_batch8(ctx, orc):
    """8 NTTs of length 2^22 over the 62-bit prime on 64-bit words."""
    cfg = BATCH8_4M_U64
    x = cfg.data()
    l, p = cfg.log2_len, cfg.p
    w = _omega(orc, p, cfg.g, l)
    assert w == 3217870244631358983
    t = dev(x)
    tp = dev(x)
    tm = dev(x)
    ctx.ntt_forward(t, p, w)
    ctx.ntt_forward(tp, p, w, plain=True)
    ctx.ntt_forward(tm, p, w, mont=True)
    got = host(t, np.uint64)
    np.testing.assert_array_equal(got, host(tp, np.uint64))
    np.testing.assert_array_equal(got, host(tm, np.uint64))
    np.testing.assert_array_equal(got[0], orc.forward(x[0], l, p, w))
    _sampled_points(orc, x, got, l, p, w, per_row=2, seed=6)
    ctx.ntt_inverse(t, p, w)
    np.testing.assert_array_equal(host(t, np.uint64), x)
    ctx.ntt_inverse(tm, p, w, mont=True)
    np.testing.assert_array_equal(host(tm, np.uint64), x)


def test_mixed_batch_one_call(ctx, orc):
    """One call with descriptors of different primes, lengths and word sizes."""
    specs = [(P30, G30, 20, 32), (754974721, 11, 9, 32), (167772161, 3, 13, 32), (P62, G62, 16, 64),
             (P30, G30, 20, 32), (P62, G62, 3, 64), (167772161, 3, 1, 32)]
    xs, ts, descs = [], [], (hntt.Desc * len(specs))()
    for i, (p, g, l, wb) in enumerate(specs):
        x = uniform_residues(300 + i, 1 << l, p, _np_dtype(wb))
        t = dev(x)
        xs.append(x)
        ts.append(t)
        descs[i] = hntt.Desc(p, _omega(orc, p, g, l), t.data_ptr(), l, wb)
    ctx.ntt_descs("hntt_ntt_forward", descs)
    for (p, g, l, wb), x, t in zip(specs, xs, ts):
        np.testing.assert_array_equal(host(t, _np_dtype(wb)).astype(np.uint64),
                                      orc.forward(x, l, p, _omega(orc, p, g, l)))


@pytest.mark.parametrize("policy", POLICIES)
@pytest.mark.parametrize("wb,l,batch", [(32, 12, 131), (32, 14, 70), (64, 13, 66)], ids=str)
def test_batches_above_one_launch(ctx, orc, wb, l, batch, policy):
    """Batches larger than one launch takes (64 transforms) run as several launches with a
    ragged last one: every transform equal to its own single-transform call, and a spread of
    them (first and last of each launch) against the oracle."""
    p, g = (P30, G30) if wb == 32 else (P62, G62)
    dt = _np_dtype(wb)
    w = _omega(orc, p, g, l)
    x = uniform_residues(500 + l, (batch, 1 << l), p, dt)
    t = dev(x)
    ctx.ntt_forward(t, p, w, **_kw(policy))
    got = host(t, dt)
    for b in sorted({0, 63, 64, 127, 128, batch - 1} & set(range(batch))):
        np.testing.assert_array_equal(got[b].astype(np.uint64), orc.forward(x[b], l, p, w), err_msg=str(b))
    for b in range(batch):
        one = dev(x[b])
        ctx.ntt_forward(one, p, w, **_kw(policy))
        np.testing.assert_array_equal(host(one, dt), got[b], err_msg=str(b))
    ctx.ntt_inverse(t, p, w, **_kw(policy))
    np.testing.assert_array_equal(host(t, dt), x)


@pytest.mark.parametrize("wb,l", [(32, 10), (32, 16), (64, 13)], ids=str)
def test_validate_flag(ctx, orc, wb, l):
    """HNTT_VALIDATE: in-range batches transform as without it; a batch with a word at or above
    p fails with EINVAL naming the first such descriptor, and no array is changed."""
    p, g = (P30, G30) if wb == 32 else (P62, G62)
    dt = _np_dtype(wb)
    w = _omega(orc, p, g, l)
    x = uniform_residues(600 + l, (3, 1 << l), p, dt)
    for inverse in (False, True):
        fn = ctx.ntt_inverse if inverse else ctx.ntt_forward
        a, b = dev(x), dev(x)
        fn(a, p, w)
        fn(b, p, w, validate=True)
        np.testing.assert_array_equal(host(b, dt), host(a, dt))
        for bad_rows, bad_value, first in (([1, 2], p, 1), ([2], (1 << wb) - 1, 2), ([0], p + 5, 0)):
            y = x.copy()
            for r in bad_rows:
                y[r, (r * 7919) % (1 << l)] = dt(bad_value)
            t = dev(y)
            with pytest.raises(hntt.HnttError) as err:
                fn(t, p, w, validate=True)
            assert err.value.status == hntt.EINVAL and f"descriptor {first}" in str(err.value)
            np.testing.assert_array_equal(host(t, dt), y)
    # the pointwise product checks both operands
    a, b = dev(x[0]), dev(x[1])
    c = dev(x[2])
    ctx.pointwise_mul(a, b, c, p, validate=True)
    np.testing.assert_array_equal(host(c, dt).astype(np.uint64), orc.pointwise(x[0], x[1], p))
    yb = x[1].copy()
    yb[-1] = dt(p)
    c = dev(x[2])
    with pytest.raises(hntt.HnttError) as err:
        ctx.pointwise_mul(a, dev(yb), c, p, validate=True)
    assert err.value.status == hntt.EINVAL
    np.testing.assert_array_equal(host(c, dt), x[2])


@pytest.mark.parametrize("l", [5, 12, 20])
def test_closed_forms_and_extremes(ctx, orc, l):
    p, g = P30, G30
    L = 1 << l
    w = _omega(orc, p, g, l)
    cases = {
        "zeros": np.zeros(L, np.uint32),
        "all_p_minus_1": np.full(L, p - 1, np.uint32),
        "delta0": np.eye(1, L, 0, dtype=np.uint32)[0],
        "ones": np.ones(L, np.uint32),
    }
    for name, x in cases.items():
        for policy in POLICIES:
            t = dev(x)
            ctx.ntt_forward(t, p, w, **_kw(policy))
            got = host(t, np.uint32)
            np.testing.assert_array_equal(got.astype(np.uint64), orc.forward(x, l, p, w), err_msg=name)
            if name == "delta0":
                assert np.all(got == 1)
            if name == "ones":
                assert got[0] == L % p and not np.any(got[1:])


@pytest.mark.parametrize("policy", ["lazy", "mont"])
def test_lazy_accepts_redundant_inputs(ctx, orc, policy):
    """Algorithms 3 and 5 take inputs in [0,2p) and the inverse butterflies in [0,4p):
    redundant representatives give the same fully reduced result."""
    p, l = P30, 20
    w = _omega(orc, p, G30, l)
    x = uniform_residues(7, 1 << l, p, np.uint32)
    rng = np.random.Generator(np.random.PCG64(8))
    red = (x.astype(np.uint64) + p * rng.integers(0, 2, size=x.size, dtype=np.uint64)).astype(np.uint32)
    t = dev(red)
    ctx.ntt_forward(t, p, w, **_kw(policy))
    np.testing.assert_array_equal(host(t, np.uint32).astype(np.uint64), orc.forward(x, l, p, w))
    red4 = (x.astype(np.uint64) + p * rng.integers(0, 4, size=x.size, dtype=np.uint64)).astype(np.uint32)
    u = dev(red4)
    ctx.ntt_inverse(u, p, w, **_kw(policy))
    np.testing.assert_array_equal(host(u, np.uint32).astype(np.uint64), orc.inverse(x, l, p, w))


@pytest.mark.parametrize("policy", ["lazy", "mont"])
@pytest.mark.parametrize("l", [10, 20])
def test_no_normalize_ranges(ctx, orc, l, policy):
    """Without the final reduction the lazy forward result lies in [0,2p) and the inverse
    in [0,4p) (Theorems 2, 3 and 4), congruent to the oracle's."""
    p = P30
    w = _omega(orc, p, G30, l)
    x = uniform_residues(9, 1 << l, p, np.uint32)
    t = dev(x)
    ctx.ntt_forward(t, p, w, normalize=False, **_kw(policy))
    got = host(t, np.uint32).astype(np.uint64)
    assert got.max() < 2 * p
    np.testing.assert_array_equal(got % p, orc.forward(x, l, p, w))
    u = dev(x)
    ctx.ntt_inverse(u, p, w, normalize=False, **_kw(policy))
    got = host(u, np.uint32).astype(np.uint64)
    assert got.max() < 4 * p
    np.testing.assert_array_equal(got % p, orc.inverse(x, l, p, w))


def test_deterministic(ctx):
    p, l = P30, 20
    w = hntt.root_of_unity(p, l)
    x = uniform_residues(10, (4, 1 << l), p, np.uint32)
    a, b = dev(x), dev(x)
    ctx.ntt_forward(a, p, w)
    ctx.ntt_forward(b, p, w)
    assert torch.equal(a, b)


# ---------------------------------------------------------------------------------------------
_KIND = {"alg2_plain_fwd": 0, "alg3_lazy_fwd": 1, "alg4_lazy_inv": 2, "plain_inv": 3, "alg5_mont_fwd": 4,
         "mont_inv": 5}


@pytest.mark.parametrize("kind", list(_KIND))
@pytest.mark.parametrize("wb,p", [(32, P30), (32, 167772161), (64, P62)], ids=["p30", "p28", "p62"])
def test_butterfly_theorems(ctx, kind, wb, p):
    """Each device butterfly against its algorithm's stated output range and congruences
    (Theorems 1-4), with exact Python integers, on random and edge operands."""
    k = _KIND[kind]
    beta = 1 << wb
    in_bound = {0: p, 1: 2 * p, 2: 4 * p, 3: p, 4: 2 * p, 5: 4 * p}[k]
    out_bound = {0: p, 1: 2 * p, 2: 4 * p, 3: p, 4: 2 * p, 5: 4 * p}[k]
    r = random.Random(k * 7 + wb)
    g = G62 if wb == 64 else hntt.primitive_root(p)
    omega = pow(g, (p - 1) >> 10, p)
    edges = sorted(e for e in {0, 1, p - 1, p, 2 * p - 1, 3 * p, in_bound - 1} if e < in_bound)
    xs, ys, ws = [], [], []
    for X in edges:
        for Y in edges:
            for W in (1, p - 1, omega):
                xs.append(X)
                ys.append(Y)
                ws.append(W)
    for _ in range(4000):
        xs.append(r.randrange(in_bound))
        ys.append(r.randrange(in_bound))
        ws.append(r.randrange(1, p))
    if k >= 4:  # Algorithm 5 inputs: W' = W beta mod p and J = p^-1 mod beta
        wargs = [(W * beta) % p for W in ws]
        wps = [pow(p, -1, beta)] * len(ws)
    else:
        wargs = ws
        wps = [(W * beta) // p for W in ws]
    dt = _np_dtype(wb)
    X, Y, W, WP = (dev(np.array(v, dtype=dt)) for v in (xs, ys, wargs, wps))
    XO, YO = torch.empty_like(X), torch.empty_like(Y)
    ctx.debug_butterfly(k, p, X, Y, W, WP, XO, YO)
    xo = host(XO, dt).tolist()
    yo = host(YO, dt).tolist()
    for i in range(len(xs)):
        a, b, w_ = xs[i], ys[i], ws[i]
        assert 0 <= xo[i] < out_bound and 0 <= yo[i] < out_bound, (kind, a, b, w_, xo[i], yo[i])
        if k in (0, 1, 4):
            assert xo[i] % p == (a + b) % p and yo[i] % p == w_ * (a - b) % p, (kind, a, b, w_)
        else:
            assert xo[i] % p == (a + w_ * b) % p and yo[i] % p == (a - w_ * b) % p, (kind, a, b, w_)


@pytest.mark.parametrize("wb,p", [(32, P30), (32, 754974721), (32, 167772161), (64, P62)])
def test_pointwise_mul(ctx, orc, wb, p):
    n = (1 << 18) + 77
    dt = _np_dtype(wb)
    a = uniform_residues(11, n, p, dt)
    b = uniform_residues(12, n, p, dt)
    a[:3] = [0, p - 1, p - 1]
    b[:3] = [p - 1, p - 1, 0]
    ta, tb = dev(a), dev(b)
    tc = torch.empty_like(ta)
    ctx.pointwise_mul(ta, tb, tc, p)
    np.testing.assert_array_equal(host(tc, dt).astype(np.uint64), orc.pointwise(a, b, p))
    tc2 = torch.zeros_like(ta)
    ctx.pointwise_mul(ta[1:], tb[1:], tc2[1:], p)  # operands not 16-byte aligned: word-by-word path
    np.testing.assert_array_equal(host(tc2, dt)[1:].astype(np.uint64), orc.pointwise(a[1:], b[1:], p))
    ctx.pointwise_mul(ta, tb, ta, p)  # in place
    np.testing.assert_array_equal(host(ta, dt).astype(np.uint64), orc.pointwise(a, b, p))


@pytest.mark.parametrize("policy", ["lazy", "mont"])
@pytest.mark.parametrize("wb,l", [(32, 20), (32, 13), (64, 22), (64, 15)])
def test_schedule_independence(ctx, orc, wb, l, policy):
    """Every legal schedule gives bit-identical results (a cross-schedule check that would
    expose LDS races or indexing mistakes tied to one tile shape)."""
    from paper_1205_2926_amd.autotune import candidates, splits
    p, g = (P30, G30) if wb == 32 else (P62, G62)
    w = _omega(orc, p, g, l)
    dt = _np_dtype(wb)
    batch = 12
    x = uniform_residues(400 + l, (batch, 1 << l), p, dt)
    ref = None
    cands = candidates(ctx, l, wb, batch)
    assert len(cands) >= 4
    picks = cands[:: max(1, len(cands) // 10)]
    # every split of the stages between the passes, whatever the stride above lands on
    for c in sorted({k["row_log2"] for k in cands}):
        picks.append(next(k for k in cands if k["row_log2"] == c))
    assert len({k["row_log2"] for k in picks}) == len(splits(ctx, l, wb)) and (l <= 12 or len(splits(ctx, l, wb)) >= 2)
    # the inverse row pass with another group than the forward one
    if l > 12:
        d = dict(picks[0])
        for gi in (d["g_rows"] // 2, d["g_rows"] * 2):
            try:
                ctx.set_tuning(l, wb, d["g_cols"], d["g_rows"], d["batch_chunk"], d["row_log2"], gi)
            except hntt.HnttError:
                continue
            picks.append({**d, "g_rows_inv": gi})
    for cand in picks:
        ctx.set_tuning(l, wb, cand["g_cols"], cand["g_rows"], cand["batch_chunk"], cand["row_log2"],
                       cand.get("g_rows_inv", 0))
        t = dev(x)
        ctx.ntt_forward(t, p, w, **_kw(policy))
        got = host(t, dt)
        if ref is None:
            ref = got
            np.testing.assert_array_equal(got[0].astype(np.uint64), orc.forward(x[0], l, p, w))
        np.testing.assert_array_equal(got, ref, err_msg=str(cand))
        ctx.ntt_inverse(t, p, w, **_kw(policy))
        np.testing.assert_array_equal(host(t, dt), x, err_msg=str(cand))
    ctx.set_tuning(l, wb)


def test_memory_budget_exhausted_then_usable(orc):
    """A context whose budget cannot hold a transform's tables refuses it with ENOMEM,
    releases what it had uploaded for it, and keeps working.  Table sizes (u32 pairs):
    2^10 whole 16 KiB; 2^16 split 8 KiB of per-stage tables + 64 KiB + 64 KiB of split
    twiddles; 2^12 whole 64 KiB.  With a 100 KiB budget the 2^16 tables fail on their
    last upload; the 2^12 tables fit only if that failure left nothing counted."""
    print("memory budget", flush=True)
    c = hntt.Context(0, mem_budget=100 * 1024)
    try:
        p = P30

        def run(l, seed):
            w = hntt.root_of_unity(p, l)
            x = uniform_residues(seed, (1, 1 << l), p, np.uint32)
            t = dev(x)
            c.ntt_forward(t, p, w)
            np.testing.assert_array_equal(host(t, np.uint32)[0], orc.forward(x[0], l, p, w).astype(np.uint32))

        run(10, 60)
        w16 = hntt.root_of_unity(p, 16)
        x16 = uniform_residues(61, (1, 1 << 16), p, np.uint32)
        t16 = dev(x16)
        for _ in range(2):  # a retry fails the same way: nothing was counted twice
            with pytest.raises(hntt.HnttError) as ei:
                c.ntt_forward(t16, p, w16)
            assert ei.value.status == hntt.ENOMEM and "budget" in c.last_error()
        np.testing.assert_array_equal(host(t16, np.uint32), x16)  # nothing was enqueued
        run(12, 62)
        run(10, 63)
    finally:
        c.close()
