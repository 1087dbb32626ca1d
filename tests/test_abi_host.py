"""The C-ABI library without a GPU: it loads, exports every declared symbol, and its
host logic (number theory, Shoup constants, descriptor checks) is right."""
import ctypes
import os
import random
import re

import pytest
import sympy

from paper_1205_2926_amd import hntt
from paper_1205_2926_amd.workloads import CRT_PRIMES, P30, P62

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hntt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hntt_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = hntt.load()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(hntt.SIGNATURES), "binding signatures must cover exactly the header"


def test_strerror():
    for s in (0, -1, -2, -3, -4, -5):
        assert hntt.strerror(s)
    assert hntt.strerror(-99) == "unknown status"


def test_is_prime_matches_sympy():
    r = random.Random(1)
    nums = list(range(3000)) + [2047, 1373653, 3215031751, 3825123056546413051, P30, P62, 2**64 - 59]
    nums += [r.randrange(1 << 64) for _ in range(300)]
    for n in nums:
        assert hntt.is_prime(n) == sympy.isprime(n), n


def test_primitive_roots_and_roots_of_unity():
    for p, g in list(CRT_PRIMES) + [(P62, 3), (17, 3), (7681, 17)]:
        assert hntt.primitive_root(p) == sympy.primitive_root(p) == g
    # the constants of the small and headline configurations
    assert hntt.root_of_unity(P30, 10) == 258648936
    assert hntt.root_of_unity(P30, 20) == 565042129
    assert hntt.root_of_unity(P62, 22) == 3217870244631358983
    for p, _ in CRT_PRIMES:
        for l in (1, 9, 17, 23):
            w = hntt.root_of_unity(p, l)
            assert pow(w, 1 << l, p) == 1 and pow(w, 1 << (l - 1), p) == p - 1
    with pytest.raises(hntt.HnttError):
        hntt.root_of_unity(P30, 24)


def test_find_prime():
    assert hntt.find_prime(62, 24) == P62
    assert hntt.find_prime(30, 25) == 0 or sympy.isprime(hntt.find_prime(30, 25))
    for bits, v in ((20, 8), (31, 20), (40, 30)):
        c = ((1 << bits) - 2) // (1 << v) * (1 << v) + 1
        while not sympy.isprime(c):
            c -= 1 << v
        assert hntt.find_prime(bits, v) == c


def test_shoup_constants_bracket():
    """W' = floor(W beta / p):  W' p <= W beta < (W' + 1) p  (Algorithm 2 input conditions)."""
    r = random.Random(2)
    for p, bits in ((P30, 32), (754974721, 32), (167772161, 32), (P62, 64)):
        beta = 1 << bits
        for w in [0, 1, p - 1, p // 2] + [r.randrange(p) for _ in range(200)]:
            wp = hntt.shoup_constant(w, p, bits)
            assert wp * p <= w * beta < (wp + 1) * p
    assert hntt.shoup_constant(258648936, P30, 32) == 1112842479
    with pytest.raises(hntt.HnttError):
        hntt.shoup_constant(P30, P30, 32)


@pytest.fixture(scope="module")
def ctx():
    c = hntt.Context(0)
    yield c
    c.close()


def _desc(p=P30, omega=258648936, data=4096, l=10, wb=32):
    return (hntt.Desc * 1)(hntt.Desc(p, omega, data, l, wb))


@pytest.mark.parametrize("kw,status,msg", [
    (dict(data=0), hntt.EINVAL, "NULL"),
    (dict(data=4098), hntt.EINVAL, "aligned"),
    (dict(data=4100), hntt.EINVAL, "aligned to 16"),
    (dict(data=4104, l=1, omega=P30 - 1), hntt.OK, ""),
    (dict(wb=16), hntt.EINVAL, "word_bits"),
    (dict(l=0), hntt.EINVAL, "log2_len"),
    (dict(l=31), hntt.EINVAL, "log2_len"),
    (dict(p=998244351), hntt.EINVAL, "divide"),
    (dict(p=998244352), hntt.EINVAL, "odd"),
    (dict(p=1 + 2**30), hntt.EUNSUPPORTED, "2^30"),
    (dict(omega=3), hntt.EINVAL, "primitive"),
    (dict(omega=P30), hntt.EINVAL, "omega"),
    (dict(l=24), hntt.EINVAL, "divide"),
    (dict(p=12289, omega=pow(11, 3, 12289), l=12), hntt.OK, ""),
    (dict(p=7681 * 1 + 0, omega=1, l=1), hntt.EINVAL, "primitive"),
])
def test_descriptor_checks(ctx, kw, status, msg):
    arr = _desc(**kw)
    assert ctx.validate(arr) == status, ctx.last_error()
    assert msg in ctx.last_error()


def test_plain_allows_larger_primes(ctx):
    # 2013265921 = 15 * 2^27 + 1 < 2^31: legal for Algorithm 2 (p < beta/2), not for Algorithm 3 (p < beta/4)
    p = 2013265921
    w = pow(31, (p - 1) >> 10, p)
    arr = _desc(p=p, omega=w)
    assert ctx.validate(arr) == hntt.EUNSUPPORTED
    assert ctx.validate(arr, hntt.PLAIN) == hntt.OK


def test_montgomery_flag_checks(ctx):
    """Algorithm 5 has the lazy bound p < beta/4; HNTT_PLAIN and HNTT_MONT exclude each other."""
    arr = _desc()
    assert ctx.validate(arr, hntt.MONT) == hntt.OK
    assert ctx.validate(arr, hntt.MONT | hntt.PLAIN) == hntt.EINVAL
    assert "HNTT_MONT" in ctx.last_error()
    p = 2013265921  # < beta/2 but not < beta/4
    assert ctx.validate(_desc(p=p, omega=pow(31, (p - 1) >> 10, p)), hntt.MONT) == hntt.EUNSUPPORTED
    assert ctx.validate(arr, 0x20) == hntt.EINVAL
    assert ctx.validate(arr, hntt.VALIDATE) == hntt.OK  # host checks only; the device check is per call


def test_validate_flag_value_matches_header():
    import re
    text = open(os.path.join(ROOT, "include", "hntt.h")).read()
    assert int(re.search(r"#define HNTT_VALIDATE (0x[0-9a-f]+)u", text).group(1), 16) == hntt.VALIDATE


def test_pointwise_flags_checked_on_host(ctx):
    d = (hntt.PwDesc * 1)(hntt.PwDesc(P30, 4096, 4096, 4096, 16, 32, 0))
    assert ctx.lib.hntt_pointwise_mul(ctx.handle, d, 1, hntt.PLAIN, None) == hntt.EINVAL
    assert "HNTT_VALIDATE" in ctx.last_error()


def test_composite_modulus_rejected(ctx):
    # 3 * 2^30 + 1 = 3221225473 is composite (and above beta/4 anyway), 7 * 2^20 + 1 = 7340033 is prime
    n = 5 * 7340033  # composite, odd, = 1 mod 2^? small
    arr = _desc(p=n, omega=1, l=1)
    assert ctx.validate(arr) == hntt.EINVAL


def test_transform_argument_errors_enqueue_nothing(ctx):
    """Bad descriptors fail on the host before any device call, so this runs without a GPU."""
    bad = (hntt.Desc * 2)(hntt.Desc(P30, 258648936, 4096, 10, 32), hntt.Desc(P30, 3, 8192, 10, 32))
    rc = ctx.lib.hntt_ntt_forward(ctx.handle, bad, 2, 0, None)
    assert rc == hntt.EINVAL and "primitive" in ctx.last_error()
    rc = ctx.lib.hntt_ntt_inverse(ctx.handle, bad, 2, 0x80, None)
    assert rc == hntt.EINVAL and "flag" in ctx.last_error()
    assert ctx.lib.hntt_ntt_forward(ctx.handle, None, 0, 0, None) == hntt.OK
    assert ctx.lib.hntt_ntt_forward(None, None, 0, 0, None) == hntt.EINVAL


def test_tuning_overrides_checked_on_host(ctx):
    base = ctx.get_plan(20, 32)
    assert base["g_cols"] >= 1 and base["g_rows"] >= 1 and base["batch_chunk"] == 64
    assert base["row_log2"] == 10  # the built-in split of 2^20: ten stages per pass
    assert base["g_rows_inv"] == base["g_rows"]  # the inverse row pass follows g_rows unless told otherwise
    ctx.set_tuning(20, 32, g_cols=8, g_rows=2, batch_chunk=16)
    assert ctx.get_plan(20, 32) == {"g_cols": 8, "g_rows": 2, "batch_chunk": 16, "row_log2": 10, "g_rows_inv": 2}
    ctx.set_tuning(20, 32, g_rows=16, g_rows_inv=8)
    assert (ctx.get_plan(20, 32)["g_rows"], ctx.get_plan(20, 32)["g_rows_inv"]) == (16, 8)
    # another split of Algorithm 1's stages between the passes: 9 in the row pass, 11 in the column pass
    ctx.set_tuning(20, 32, row_log2=9)
    assert ctx.get_plan(20, 32)["row_log2"] == 9
    for bad in (dict(g_cols=3), dict(g_cols=64), dict(g_rows=1024), dict(g_rows_inv=3), dict(g_rows_inv=1024),
                dict(batch_chunk=65), dict(row_log2=13), dict(row_log2=7),
                dict(row_log2=20)):  # (7 and 20 leave the column pass 13 and 0 stages)
        with pytest.raises(hntt.HnttError):
            ctx.set_tuning(20, 32, **bad)
    with pytest.raises(hntt.HnttError):
        ctx.set_tuning(12, 32, row_log2=6)  # one-pass length has no split
    with pytest.raises(hntt.HnttError):
        ctx.set_tuning(25, 32, g_cols=4)  # beyond the two-pass range
    with pytest.raises(hntt.HnttError):
        ctx.set_tuning(10, 32, g_cols=4)  # one-pass length has no column pass
    with pytest.raises(hntt.HnttError):
        ctx.set_tuning(10, 32, g_rows_inv=2)  # nor a row pass
    ctx.set_tuning(20, 32)
    assert ctx.get_plan(20, 32) == base


def _poly(a=4096, b=8192, out=16384, na=10, nb=7):
    return (hntt.PolyDesc * 1)(hntt.PolyDesc(a, b, out, na, nb))


@pytest.mark.parametrize("kw,status,msg", [
    (dict(na=0), hntt.EINVAL, "empty"),
    (dict(a=0), hntt.EINVAL, "NULL"),
    (dict(out=0), hntt.EINVAL, "NULL"),
    (dict(a=4098), hntt.EINVAL, "misaligned"),
    (dict(out=16388), hntt.EINVAL, "misaligned"),
    (dict(na=(1 << 22) + 1), hntt.EUNSUPPORTED, "2^23"),
])
def test_polymul_descriptor_checks(ctx, kw, status, msg):
    """Bad product descriptors are rejected on the host before any device call."""
    import ctypes
    h = ctypes.c_void_p()
    rc = ctx.lib.hntt_polymul_plan_create(ctx.handle, _poly(**kw), 1, 0, None, 0, None, ctypes.byref(h))
    assert rc == status and msg in ctx.last_error(), ctx.last_error()
    assert not h.value
    assert ctx.lib.hntt_polymul_crt(ctx.handle, _poly(**kw), 1, 0, None) == status
    assert ctx.lib.hntt_polymul_crt(ctx.handle, _poly(), 1, 0x80, None) == hntt.EINVAL


def test_polymul_workspace_size_host_only():
    # 6 arrays of L = 2 * nextpow2(max(na, nb)) words plus metadata, no device needed
    s = hntt.polymul_workspace_size([(1 << 20, 1 << 20)])
    assert 6 * 4 * (1 << 21) <= s < 6 * 4 * (1 << 21) + (1 << 20)
    assert hntt.polymul_workspace_size([(3, 5)]) >= 6 * 4 * 16
    with pytest.raises(hntt.HnttError):
        hntt.polymul_workspace_size([(0, 5)])
    with pytest.raises(hntt.HnttError):
        hntt.polymul_workspace_size([((1 << 22) + 1, 5)])


def test_serving_arena_allocator():
    from paper_1205_2926_amd.serve import Arena
    a = Arena(4096)
    x = a.alloc(1000)
    y = a.alloc(1000)
    z = a.alloc(2100)
    assert x == 0 and y == 1024 and z is None
    a.release(x, 1000)
    assert a.alloc(1024) == 0
    a.release(0, 1024)
    a.release(y, 1000)
    assert a.free == [(0, 4096)] and a.used == 0 and a.peak == 2048


def test_serving_workspace_bound_covers_library_size():
    """The server's additive per-request workspace bound is never below the library's exact
    workspace size of a group (host-only sizing, no GPU)."""
    import numpy as np
    from paper_1205_2926_amd.serve import Request, _GROUP_SLACK
    gen = np.random.default_rng(0)
    for _ in range(100):
        k = int(gen.integers(1, 70))
        reqs = [Request(i, 0.0, np.zeros(int(2 ** gen.uniform(0, 20)), np.uint32),
                        np.zeros(int(2 ** gen.uniform(0, 20)), np.uint32)) for i in range(k)]
        exact = hntt.polymul_workspace_size([(r.a.size, r.b.size) for r in reqs])
        assert exact <= sum(r.workspace_bound() for r in reqs) + _GROUP_SLACK


def test_serving_client_buffers_are_checked():
    """A request's own result buffer must be a writable contiguous uint64 array of at least
    na + nb - 1 words; anything else is refused when the request is made (host only)."""
    import numpy as np
    from paper_1205_2926_amd.serve import Request
    a, b = np.ones(10, np.uint32), np.ones(7, np.uint32)
    Request(0, 0.0, a, b, np.empty(16, np.uint64))
    Request(0, 0.0, a, b, np.empty(40, np.uint64))
    ro = np.empty(16, np.uint64)
    ro.flags.writeable = False
    for bad in (np.empty(15, np.uint64), np.empty(16, np.int32), np.empty((4, 4), np.uint64),
                np.empty(32, np.uint64)[::2], ro):
        with pytest.raises(ValueError):
            Request(0, 0.0, a, b, bad)


def test_bigmul_sizing_checks():
    """Large-integer plans: workspace from lengths alone, operand limits checked on the host."""
    ws = hntt.bigmul_workspace_size([(1000, 3000), (1, 1)])
    assert ws >= hntt.polymul_workspace_size([(1000, 3000), (1, 1)])
    assert hntt.bigmul_workspace_size([(1 << 22, 1 << 22)]) > 0
    with pytest.raises(hntt.HnttError):
        hntt.bigmul_workspace_size([((1 << 22) + 1, 1)])
    with pytest.raises(hntt.HnttError):
        hntt.bigmul_workspace_size([(0, 4)])


def test_missing_library_fails_loudly(tmp_path):
    """There is no CPU fallback: loading a library that is not there raises HnttNotBuilt."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1205_2926_amd import hntt\n"
            "try:\n"
            "    hntt.load(%r)\n"
            "except hntt.HnttNotBuilt:\n"
            "    print('raised')\n") % (os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                        str(tmp_path / "libhntt.so"))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert out.stdout.strip() == "raised", out.stderr


def test_oracle_is_not_imported_by_the_library():
    """The product path never imports the oracle package."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_1205_2926_amd.hntt, paper_1205_2926_amd.serve, paper_1205_2926_amd.autotune\n"
            "print('oracle' in sys.modules)\n") % root
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert out.stdout.strip() == "False", out.stderr
