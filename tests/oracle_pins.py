"""Pins that tie the CPU oracle to the paper and to mathematics outside itself.

Each ``pin_*`` takes an ``oracle.Oracle`` and raises ``AssertionError`` when
the oracle disagrees with an independent fact: the hand-worked example in
``tests/golden/``, brute-force sums of the NTT definition (Section 1, display
eq.), sympy's own NTT and number theory, closed forms of the transform,
a primality certificate, exact Python big-integer products.  None of them
re-types the oracle's own algorithm.  ``test_oracle_pins.py`` runs them on the
real oracle; ``test_oracle_mutants.py`` runs them on deliberately broken
copies of it to show that plausible mistakes are caught.
"""
from __future__ import annotations

import os
import random

import numpy as np

from paper_1205_2926_amd.workloads import CRT_PRIMES, P30, G30, P62, G62

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
PRIMES = [(P30, G30), (754974721, 11), (167772161, 3), (P62, G62)]


def _rev(j: int, l: int) -> int:
    return int(format(j, f"0{l}b")[::-1], 2) if l else 0


def naive_dft(a, p, w):
    """b_j = sum_i w^(ij) a_i mod p, straight from the definition."""
    L = len(a)
    out = []
    for j in range(L):
        wj = pow(w, j, p)
        acc, wij = 0, 1
        for i in range(L):
            acc += int(a[i]) * wij
            wij = wij * wj % p
        out.append(acc % p)
    return out


def to_bitrev(b):
    L = len(b)
    l = L.bit_length() - 1
    out = [0] * L
    for j in range(L):
        out[_rev(j, l)] = b[j]
    return out


def _root(p, g, l):
    return pow(g, (p - 1) >> l, p)


def read_golden(name):
    d = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *v = line.split()
            d[k] = [int(t) for t in v]
    return d


# ---------------------------------------------------------------------------------------------
def pin_golden_tiny(orc):
    g = read_golden("ntt_p17_L8.txt")
    p, l, w = g["p"][0], g["log2_len"][0], g["omega"][0]
    out = orc.forward(g["input"], l, p, w)
    assert out.tolist() == g["bitreversed"], out
    back = orc.inverse(g["bitreversed"], l, p, w)
    assert back.tolist() == g["input"], back


def pin_forward_naive(orc, max_l=7):
    r = random.Random(11)
    for p, g in PRIMES:
        for l in range(1, max_l + 1):
            w = _root(p, g, l)
            a = [r.randrange(p) for _ in range(1 << l)]
            got = orc.forward(a, l, p, w).tolist()
            assert got == to_bitrev(naive_dft(a, p, w)), (p, l)


def pin_forward_sympy(orc, ls=(8, 10, 11, 12)):
    from sympy.discrete.transforms import ntt
    r = random.Random(12)
    for p, g in PRIMES[:3]:
        for l in ls:
            a = [r.randrange(p) for _ in range(1 << l)]
            got = orc.forward(a, l, p, _root(p, g, l)).tolist()
            assert got == to_bitrev(ntt(a, p)), (p, l)


def pin_inverse_naive(orc, max_l=7):
    r = random.Random(13)
    for p, g in PRIMES:
        for l in range(1, max_l + 1):
            L = 1 << l
            w = _root(p, g, l)
            b = [r.randrange(p) for _ in range(L)]
            # inverse definition: a_i = L^-1 sum_j w^(-ij) b_j, input given in bit-reversed order
            a = [x * pow(L, -1, p) % p for x in naive_dft(b, p, pow(w, -1, p))]
            got = orc.inverse(to_bitrev(b), l, p, w).tolist()
            assert got == a, (p, l)


def pin_inverse_sympy(orc, ls=(9, 12)):
    from sympy.discrete.transforms import intt
    r = random.Random(14)
    for p, g in PRIMES[:3]:
        for l in ls:
            b = [r.randrange(p) for _ in range(1 << l)]
            got = orc.inverse(to_bitrev(b), l, p, _root(p, g, l)).tolist()
            assert got == intt(b, p), (p, l)


def pin_roundtrip(orc, l30=16, l62=14):
    for (p, g), l in ((PRIMES[0], l30), (PRIMES[2], l30), (PRIMES[3], l62)):
        w = _root(p, g, l)
        a = np.random.Generator(np.random.PCG64(15)).integers(0, p, size=(2, 1 << l), dtype=np.uint64)
        f = orc.forward(a, l, p, w)
        assert not np.array_equal(f, a)
        assert np.array_equal(orc.inverse(f, l, p, w), a), (p, l)


def pin_closed_forms(orc, l=14, primes=(PRIMES[0], PRIMES[3])):
    """delta_0 -> all ones; all ones -> L e_0; w^(-ci) -> L at rev(c); shift theorem; linearity."""
    for p, g in primes:
        L = 1 << l
        w = _root(p, g, l)
        delta = np.zeros(L, dtype=np.uint64)
        delta[0] = 1
        assert np.all(orc.forward(delta, l, p, w) == 1)
        ones = np.ones(L, dtype=np.uint64)
        f = orc.forward(ones, l, p, w)
        assert f[0] == L % p and not np.any(f[1:])
        assert np.array_equal(orc.inverse(f, l, p, w), ones)
        for c in (1, 3, L // 2 + 5, L - 1):
            winv_c = pow(w, -c, p)
            x = np.empty(L, dtype=np.uint64)
            acc = 1
            for i in range(L):
                x[i] = acc
                acc = acc * winv_c % p
            f = orc.forward(x, l, p, w)
            spike = _rev(c, l)
            assert f[spike] == L % p, (p, c)
            f[spike] = 0
            assert not np.any(f), (p, c)
        # shift theorem on a short random vector: x_{i-s} -> w^(s j) b_j
        ls = 6
        Ls = 1 << ls
        ws = _root(p, g, ls)
        a = [random.Random(16).randrange(p) for _ in range(Ls)]
        b = orc.forward(a, ls, p, ws).tolist()
        for s in (1, 5):
            sh = a[-s:] + a[:-s]
            bs = orc.forward(sh, ls, p, ws).tolist()
            for j in range(Ls):
                assert bs[_rev(j, ls)] == pow(ws, s * j, p) * b[_rev(j, ls)] % p
        # linearity
        r = random.Random(17)
        u = [r.randrange(p) for _ in range(Ls)]
        v = [r.randrange(p) for _ in range(Ls)]
        fu = orc.forward(u, ls, p, ws).tolist()
        fv = orc.forward(v, ls, p, ws).tolist()
        fuv = orc.forward([(x + y) % p for x, y in zip(u, v)], ls, p, ws).tolist()
        assert fuv == [(x + y) % p for x, y in zip(fu, fv)]


def pin_dft_point(orc):
    from sympy.discrete.transforms import ntt
    r = random.Random(18)
    for p, g in PRIMES[:3]:
        l = 6
        a = [r.randrange(p) for _ in range(1 << l)]
        ref = ntt(a, p)
        w = _root(p, g, l)
        for j in (0, 1, 7, 63):
            assert orc.dft_point(a, l, p, w, j) == ref[j]
    # a large closed form: x_i = w^(-ci) gives b_c = L and b_j = 0 otherwise
    p, g = PRIMES[3]
    l = 12
    L = 1 << l
    w = _root(p, g, l)
    c = 77
    x = [pow(w, -c * i, p) for i in range(L)]
    assert orc.dft_point(x, l, p, w, c) == L
    assert orc.dft_point(x, l, p, w, c + 1) == 0


def pin_bitrev(orc):
    for l in (1, 3, 10, 20):
        for j in {0, 1, 5 % (1 << l), (1 << l) - 1, (1 << l) // 3}:
            assert orc.bitrev(j, l) == _rev(j, l)


_PSEUDOPRIMES = [561, 1105, 1729, 2047, 1373653, 25326001, 3215031751, 2152302898747, 3474749660383,
                 341550071728321, 3825123056546413051]


def pin_number_theory(orc):
    import sympy
    for n in list(range(0, 3000)) + _PSEUDOPRIMES + [P30, P62, 2**61 - 1, 2**64 - 59, 2**64 - 1]:
        assert orc.is_prime(n) == sympy.isprime(n), n
    r = random.Random(19)
    for _ in range(200):
        n = r.randrange(1 << 63) | 1
        assert orc.is_prime(n) == sympy.isprime(n), n
    for p, g in PRIMES + [(17, 3), (97, 5), (7681, 17)]:
        assert orc.primitive_root(p) == sympy.primitive_root(p) == g, p
    for p, g in PRIMES:
        for l in (1, 10, 20, 23):
            w = orc.root_of_unity(p, g, l)
            assert pow(w, 1 << l, p) == 1 and pow(w, 1 << (l - 1), p) == p - 1, (p, l)
    assert orc.root_of_unity(P30, 3, 24) == 0  # 2^24 does not divide p - 1
    assert orc.inv_mod(3, P30) * 3 % P30 == 1
    assert orc.pow_mod(3, P62 - 1, P62) == 1


def pin_prime_search(orc):
    """The 62-bit prime: Pocklington/Lucas certificate, and every larger candidate composite."""
    p = orc.largest_ntt_prime(62, 24)
    assert p == P62
    # p - 1 = 2^25 * 47189 * 2912521, the odd factors prime by trial division
    f = [2, 47189, 2912521]
    assert (p - 1) == 2**25 * 47189 * 2912521
    for q in f[1:]:
        assert all(q % d for d in range(2, int(q**0.5) + 1))
    # Lucas: 3^(p-1) = 1 and 3^((p-1)/q) != 1 for each prime q | p-1  =>  p prime and 3 generates F_p^*
    assert pow(3, p - 1, p) == 1
    assert all(pow(3, (p - 1) // q, p) != 1 for q in f)
    c = p + (1 << 24)
    while c < (1 << 62):
        assert pow(2, c - 1, c) != 1 or pow(3, c - 1, c) != 1, c  # a Fermat witness proves c composite
        c += 1 << 24
    # small case against a brute-force sympy search
    import sympy
    for bits, v in ((20, 8), (31, 20), (40, 30)):
        c = ((1 << bits) - 2) // (1 << v) * (1 << v) + 1
        while not sympy.isprime(c):
            c -= 1 << v
        assert orc.largest_ntt_prime(bits, v) == c, (bits, v)


def pin_pointwise(orc):
    r = random.Random(20)
    for p, _ in PRIMES:
        a = [r.randrange(p) for _ in range(100)] + [p - 1, 0, p - 1]
        b = [r.randrange(p) for _ in range(100)] + [p - 1, p - 1, 0]
        assert orc.pointwise(a, b, p).tolist() == [x * y % p for x, y in zip(a, b)]


def _conv(a, b):
    c = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            c[i + j] += int(x) * int(y)
    return c


def pin_polymul_mod(orc):
    r = random.Random(21)
    for p, g in PRIMES:
        for na, nb in ((1, 1), (1, 7), (5, 3), (64, 64), (100, 37), (129, 128)):
            a = [r.randrange(p) for _ in range(na)]
            b = [r.randrange(p) for _ in range(nb)]
            assert orc.polymul_mod(a, b, p, g).tolist() == [x % p for x in _conv(a, b)], (p, na, nb)


def pin_crt3(orc):
    (q1, _), (q2, _), (q3, _) = CRT_PRIMES
    r = random.Random(22)
    xs = [0, 1, q1, q1 * q2 - 1, q1 * q2 + 5, (1 << 64) - 1] + [r.randrange(1 << 64) for _ in range(200)]
    out = orc.crt3([x % q1 for x in xs], [x % q2 for x in xs], [x % q3 for x in xs], q1, q2, q3)
    assert out.tolist() == xs


def pin_schoolbook(orc):
    r = random.Random(23)
    for na, nb in ((1, 1), (3, 9), (50, 41)):
        a = [r.randrange(1 << 20) for _ in range(na)]
        b = [r.randrange(1 << 20) for _ in range(nb)]
        ref = np.convolve(np.array(a, dtype=object), np.array(b, dtype=object)).tolist()
        assert orc.schoolbook(a, b).tolist() == ref
        for k in {0, na + nb - 2, (na + nb - 2) // 2}:
            assert orc.product_coeff(a, b, k) == ref[k]


def pin_polymul_exact(orc):
    r = random.Random(24)
    for n in (1, 2, 37, 256, 700):
        a = [r.randrange(1 << 20) for _ in range(n)]
        b = [r.randrange(1 << 20) for _ in range(n)]
        assert orc.polymul_exact(a, b, CRT_PRIMES).tolist() == _conv(a, b), n
    # the worst case for exactness: all coefficients 2^20 - 1
    n = 3000
    a = [(1 << 20) - 1] * n
    got = orc.polymul_exact(a, a, CRT_PRIMES).tolist()
    assert got[n - 1] == n * ((1 << 20) - 1) ** 2 and got[0] == ((1 << 20) - 1) ** 2


def pin_poly_eval(orc):
    r = random.Random(25)
    for m in ((1 << 61) - 1, 998244353, 17):
        for n in (1, 2, 50, 300):
            c = [r.randrange(1 << 63) for _ in range(n)]
            x = r.randrange(1 << 62)
            assert orc.poly_eval(c, x, m) == sum(ci * pow(x, i, m) for i, ci in enumerate(c)) % m
    # evaluation respects products: (a b)(x) = a(x) b(x)
    a = [r.randrange(1 << 20) for _ in range(40)]
    b = [r.randrange(1 << 20) for _ in range(33)]
    m, x = (1 << 61) - 1, 123456789
    assert orc.poly_eval(_conv(a, b), x, m) == orc.poly_eval(a, x, m) * orc.poly_eval(b, x, m) % m


def pin_bigmul(orc):
    """Long multiplication of limb arrays against Python's integer product (an independent
    multiplication), the square of beta^n - 1 in closed form, and products by 0, 1 and beta^k."""
    r = random.Random(26)
    for na, nb in ((1, 1), (1, 7), (7, 1), (3, 3), (17, 40), (64, 5)):
        a = np.array([r.randrange(1 << 32) for _ in range(na)], np.uint32)
        b = np.array([r.randrange(1 << 32) for _ in range(nb)], np.uint32)
        got = orc.bigmul_schoolbook(a, b)
        want = orc.limbs_to_int(a) * orc.limbs_to_int(b)
        assert orc.limbs_to_int(got) == want and got.size == na + nb
        np.testing.assert_array_equal(orc.bigmul(a, b), got)
    for n in (1, 2, 9):
        # (beta^n - 1)^2 = beta^2n - 2 beta^n + 1: limbs 1, 0.., 0xFFFFFFFE, 0xFFFFFFFF..
        ones = np.full(n, 0xFFFFFFFF, np.uint32)
        want = np.array([1] + [0] * (n - 1) + [0xFFFFFFFE] + [0xFFFFFFFF] * (n - 1), np.uint32)
        np.testing.assert_array_equal(orc.bigmul_schoolbook(ones, ones), want)
    a = np.array([r.randrange(1 << 32) for _ in range(12)], np.uint32)
    np.testing.assert_array_equal(orc.bigmul_schoolbook(a, np.zeros(3, np.uint32)), np.zeros(15, np.uint32))
    np.testing.assert_array_equal(orc.bigmul_schoolbook(a, np.array([1], np.uint32))[:12], a)
    shift = np.array([0, 0, 1], np.uint32)  # beta^2
    np.testing.assert_array_equal(orc.bigmul_schoolbook(a, shift), np.concatenate([[0, 0], a, [0]]).astype(np.uint32))
    for m in ((1 << 61) - 1, 998244353, 3):
        assert orc.limbs_mod(a, m) == orc.limbs_to_int(a) % m


ALL_PINS = [pin_golden_tiny, pin_forward_naive, pin_forward_sympy, pin_inverse_naive, pin_inverse_sympy,
            pin_roundtrip, pin_closed_forms, pin_dft_point, pin_bitrev, pin_number_theory, pin_prime_search,
            pin_pointwise, pin_polymul_mod, pin_crt3, pin_schoolbook, pin_polymul_exact, pin_poly_eval,
            pin_bigmul]
