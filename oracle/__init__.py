"""Plain CPU oracle for the lazy-butterfly NTT (arXiv:1205.2926).

TEST INFRASTRUCTURE ONLY: this package is the checker that the GPU library is
compared against.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the GPU library neither imports nor links it,
and it imports nothing from the GPU library.

The arithmetic lives in ``ntt_oracle.c`` (plain C, every operation fully
reduced to [0, p)); this module compiles it with gcc and marshals numpy
``uint64`` arrays to it.  Each wrapper names the passage of the paper that the
C function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ntt_oracle.c")
# ORACLE_LIB: another build of the oracle (e.g. one with sanitizers)
_LIB = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "libntt_oracle.so")

_u64 = ctypes.c_uint64
_p64 = ctypes.POINTER(ctypes.c_uint64)
_p32 = ctypes.POINTER(ctypes.c_uint32)
_lib = None


def build(extra_flags: tuple[str, ...] = (), out: str | None = None) -> str:
    """Compile ``ntt_oracle.c`` into a shared library with gcc -O2."""
    out = out or _LIB
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra", *extra_flags, _SRC, "-o", out]
    subprocess.run(cmd, check=True)
    return out


def _declare(lib):
    sig = {
        "oracle_pow_mod": (_u64, [_u64, _u64, _u64]),
        "oracle_inv_mod": (_u64, [_u64, _u64]),
        "oracle_is_prime": (ctypes.c_int, [_u64]),
        "oracle_primitive_root": (_u64, [_u64]),
        "oracle_root_of_unity": (_u64, [_u64, _u64, ctypes.c_uint]),
        "oracle_largest_ntt_prime": (_u64, [ctypes.c_uint, ctypes.c_uint]),
        "oracle_ntt_forward": (None, [_p64, ctypes.c_uint, _u64, _u64]),
        "oracle_ntt_inverse": (None, [_p64, ctypes.c_uint, _u64, _u64]),
        "oracle_ntt_forward_batch": (None, [_p64, ctypes.c_size_t, ctypes.c_uint, _u64, _u64]),
        "oracle_ntt_inverse_batch": (None, [_p64, ctypes.c_size_t, ctypes.c_uint, _u64, _u64]),
        "oracle_dft_point": (_u64, [_p64, ctypes.c_uint, _u64, _u64, _u64]),
        "oracle_bitrev": (_u64, [_u64, ctypes.c_uint]),
        "oracle_pointwise": (None, [_p64, _p64, _p64, ctypes.c_size_t, _u64]),
        "oracle_polymul_mod": (ctypes.c_int, [_p64, ctypes.c_size_t, _p64, ctypes.c_size_t, _p64,
                                              ctypes.c_uint, _u64, _u64]),
        "oracle_crt3": (None, [_p64, _p64, _p64, _p64, ctypes.c_size_t, _u64, _u64, _u64]),
        "oracle_schoolbook": (None, [_p64, ctypes.c_size_t, _p64, ctypes.c_size_t, _p64]),
        "oracle_product_coeff": (_u64, [_p64, ctypes.c_size_t, _p64, ctypes.c_size_t, ctypes.c_size_t]),
        "oracle_poly_eval": (_u64, [_p64, ctypes.c_size_t, _u64, _u64]),
        "oracle_bigmul_schoolbook": (None, [_p32, ctypes.c_size_t, _p32, ctypes.c_size_t, _p32]),
        "oracle_limbs_mod": (_u64, [_p32, ctypes.c_size_t, _u64]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def load(path: str | None = None, rebuild: bool = False):
    """Load the compiled oracle, building it first when it is missing."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    if _lib is None or rebuild:
        if rebuild or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_p64)


def _ptr32(a: np.ndarray):
    assert a.dtype == np.uint32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_p32)


def _u64arr(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint64))


class Oracle:
    """numpy-facing wrappers over one loaded copy of the C oracle."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    # number theory (Section 1: p prime, L = 2^l | p - 1, omega of order L)
    def pow_mod(self, a: int, e: int, p: int) -> int:
        return int(self.lib.oracle_pow_mod(a, e, p))

    def inv_mod(self, a: int, p: int) -> int:
        return int(self.lib.oracle_inv_mod(a, p))

    def is_prime(self, n: int) -> bool:
        return bool(self.lib.oracle_is_prime(n))

    def primitive_root(self, p: int) -> int:
        return int(self.lib.oracle_primitive_root(p))

    def root_of_unity(self, p: int, g: int, log2_len: int) -> int:
        return int(self.lib.oracle_root_of_unity(p, g, log2_len))

    def largest_ntt_prime(self, bits: int, v: int) -> int:
        return int(self.lib.oracle_largest_ntt_prime(bits, v))

    # transforms (Algorithm 1 and Algorithm 1 run backwards, Section 4)
    def forward(self, x, log2_len: int, p: int, omega: int) -> np.ndarray:
        """Forward NTT of each row of ``x`` (shape [..., 2^l]); bit-reversed output."""
        a = _u64arr(x).copy()
        L = 1 << log2_len
        assert a.shape[-1] == L
        self.lib.oracle_ntt_forward_batch(_ptr(a), a.size // L, log2_len, p, omega)
        return a

    def inverse(self, x, log2_len: int, p: int, omega: int) -> np.ndarray:
        """Inverse NTT (bit-reversed in, natural out, times L^-1) of each row."""
        a = _u64arr(x).copy()
        L = 1 << log2_len
        assert a.shape[-1] == L
        self.lib.oracle_ntt_inverse_batch(_ptr(a), a.size // L, log2_len, p, omega)
        return a

    def dft_point(self, a, log2_len: int, p: int, omega: int, j: int) -> int:
        """b_j of the definition (Section 1, display eq.), by the direct sum."""
        arr = _u64arr(a)
        return int(self.lib.oracle_dft_point(_ptr(arr), log2_len, p, omega, j))

    def bitrev(self, j: int, l: int) -> int:
        return int(self.lib.oracle_bitrev(j, l))

    # polynomial products
    def pointwise(self, a, b, p: int) -> np.ndarray:
        a = _u64arr(a)
        b = _u64arr(b)
        c = np.empty_like(a)
        self.lib.oracle_pointwise(_ptr(a), _ptr(b), _ptr(c), a.size, p)
        return c

    def polymul_mod(self, a, b, p: int, g: int) -> np.ndarray:
        """(a*b) mod p via the convolution theorem at L = 2*nextpow2(max(na, nb))."""
        a = _u64arr(a)
        b = _u64arr(b)
        n = max(a.size, b.size)
        l = max(1, (n - 1).bit_length() + 1)
        omega = self.root_of_unity(p, g, l)
        c = np.empty(a.size + b.size - 1, dtype=np.uint64)
        rc = self.lib.oracle_polymul_mod(_ptr(a), a.size, _ptr(b), b.size, _ptr(c), l, p, omega)
        assert rc == 0
        return c

    def crt3(self, r1, r2, r3, q1: int, q2: int, q3: int) -> np.ndarray:
        r1, r2, r3 = _u64arr(r1), _u64arr(r2), _u64arr(r3)
        out = np.empty_like(r1)
        self.lib.oracle_crt3(_ptr(r1), _ptr(r2), _ptr(r3), _ptr(out), r1.size, q1, q2, q3)
        return out

    def polymul_exact(self, a, b, primes) -> np.ndarray:
        """Exact integer product from three NTT primes and the textbook CRT."""
        (q1, g1), (q2, g2), (q3, g3) = primes
        r = [self.polymul_mod(a, b, q, g) for q, g in ((q1, g1), (q2, g2), (q3, g3))]
        return self.crt3(r[0], r[1], r[2], q1, q2, q3)

    def schoolbook(self, a, b) -> np.ndarray:
        a = _u64arr(a)
        b = _u64arr(b)
        c = np.empty(a.size + b.size - 1, dtype=np.uint64)
        self.lib.oracle_schoolbook(_ptr(a), a.size, _ptr(b), b.size, _ptr(c))
        return c

    def poly_eval(self, c, r: int, m: int) -> int:
        """c(r) mod m by Horner's rule."""
        c = _u64arr(c)
        return int(self.lib.oracle_poly_eval(_ptr(c), c.size, r, m))

    def product_coeff(self, a, b, k: int) -> int:
        a = _u64arr(a)
        b = _u64arr(b)
        return int(self.lib.oracle_product_coeff(_ptr(a), a.size, _ptr(b), b.size, k))

    # large-integer products (Section 1: the application of fast transforms)
    def bigmul_schoolbook(self, a, b) -> np.ndarray:
        """a * b for little-endian base-2^32 limb arrays by long multiplication (O(na nb))."""
        a = np.ascontiguousarray(a, dtype=np.uint32)
        b = np.ascontiguousarray(b, dtype=np.uint32)
        out = np.empty(a.size + b.size, dtype=np.uint32)
        self.lib.oracle_bigmul_schoolbook(_ptr32(a), a.size, _ptr32(b), b.size, _ptr32(out))
        return out

    @staticmethod
    def limbs_to_int(x) -> int:
        return int.from_bytes(np.ascontiguousarray(x, dtype="<u4").tobytes(), "little")

    @staticmethod
    def int_to_limbs(v: int, n: int) -> np.ndarray:
        return np.frombuffer(v.to_bytes(4 * n, "little"), dtype="<u4").astype(np.uint32)

    def bigmul(self, a, b) -> np.ndarray:
        """a * b as na + nb limbs, with Python's arbitrary-precision integer product as the
        multiplication step (fast enough for the larger test cases)."""
        a = np.ascontiguousarray(a, dtype=np.uint32)
        b = np.ascontiguousarray(b, dtype=np.uint32)
        return self.int_to_limbs(self.limbs_to_int(a) * self.limbs_to_int(b), a.size + b.size)

    def limbs_mod(self, x, m: int) -> int:
        """The integer with limbs x, reduced mod m."""
        x = np.ascontiguousarray(x, dtype=np.uint32)
        return int(self.lib.oracle_limbs_mod(_ptr32(x), x.size, m))
