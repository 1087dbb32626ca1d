"""Plant plausible mistakes in copies of the CPU oracle and check that the pins catch each one.

Every mutant is a one-token edit of ``oracle/ntt_oracle.c`` (a wrong sign, a
wrong index, a dropped term, a swapped operand, an off-by-one) compiled into a
throw-away library under pytest's tmp dir.  The real oracle is never touched.
"""
import os

import pytest

import oracle
from tests.oracle_pins import ALL_PINS

SRC = os.path.join(os.path.dirname(oracle.__file__), "ntt_oracle.c")

# (name, original text, mutated text, which occurrence (0-based))
MUTANTS = [
    ("fwd_sub_sign", "x[t + k + m] = mul_mod(w, sub_mod(X, Y, p), p);",
     "x[t + k + m] = mul_mod(w, sub_mod(Y, X, p), p);", 0),
    ("fwd_add_drops_y", "x[t + k] = add_mod(X, Y, p);", "x[t + k] = add_mod(X, X, p);", 0),
    ("fwd_zeta_index", "uint64_t zeta = oracle_pow_mod(omega, 1ull << (i - 1), p);",
     "uint64_t zeta = oracle_pow_mod(omega, 1ull << i, p);", 0),
    ("fwd_half_distance", "size_t m = (size_t)1 << (l - i);", "size_t m = (size_t)1 << (l - i) >> 1;", 0),
    ("fwd_twiddle_not_advanced", "        w = mul_mod(w, zeta, p);\n      }\n    }\n  }\n}\n\n/* Inverse",
     "      }\n    }\n  }\n}\n\n/* Inverse", 0),
    ("inv_no_scaling", "x[n] = mul_mod(x[n], Linv, p);", "x[n] = x[n];", 0),
    ("inv_sub_swapped", "x[t + k + m] = sub_mod(X, S, p);", "x[t + k + m] = sub_mod(S, X, p);", 0),
    ("inv_uses_forward_root", "uint64_t zeta = oracle_pow_mod(omega_inv, 1ull << (i - 1), p);",
     "uint64_t zeta = oracle_pow_mod(omega, 1ull << (i - 1), p);", 0),
    ("add_mod_strict", "if (s >= p) s -= p;", "if (s > p) s -= p;", 0),
    ("sub_mod_abs_diff", "return (a >= b) ? a - b : a + (p - b);", "return (a >= b) ? a - b : b - a;", 0),
    ("mul_mod_threshold", "if (p <= 0xFFFFFFFFull) return (a * b) % p;",
     "if (p <= 0xFFFFFFFFFFFFFFull) return (a * b) % p;", 0),
    ("dft_point_wrong_step", "w = mul_mod(w, wj, p);", "w = mul_mod(w, omega, p);", 0),
    ("crt_wrong_cofactor", "M2 = (u128)q1 * q3", "M2 = (u128)q1 * q2", 0),
    ("schoolbook_operand", "c[i + j] += a[i] * b[j];", "c[i + j] += a[i] * b[i];", 0),
    ("polymul_operand", "oracle_pointwise(fa, fb, fa, L, p);", "oracle_pointwise(fa, fa, fa, L, p);", 0),
    ("mr_single_base", "for (int i = 0; i < 12; ++i) {\n    uint64_t x",
     "for (int i = 0; i < 1; ++i) {\n    uint64_t x", 0),
    ("primroot_wrong_test", "== 1) ok = 0;", "== p - 1) ok = 0;", 0),
    ("bitrev_shift", "<< (l - 1 - b);", "<< (l - b);", 0),
    ("coeff_low_bound", "size_t lo = (k + 1 > nb) ? k + 1 - nb : 0;", "size_t lo = (k + 1 > nb) ? k + 1 - nb : 1;", 0),
    ("poly_eval_drops_coeff", "acc = add_mod(mul_mod(acc, r % m, m), c[i] % m, m);",
     "acc = mul_mod(acc, r % m, m);", 0),
    ("prime_search_step", "uint64_t c = k * step + 1;", "uint64_t c = k * step - 1;", 0),
    ("bigmul_drops_carry", "const uint64_t t = (uint64_t)a[i] * b[j] + out[i + j] + carry;",
     "const uint64_t t = (uint64_t)a[i] * b[j] + out[i + j];", 0),
    ("bigmul_last_carry_slot", "out[i + nb] = (uint32_t)carry;", "out[i + nb - 1] += (uint32_t)carry;", 0),
    ("limbs_mod_base", "acc = add_mod(mul_mod(acc, base, m), (uint64_t)x[i] % m, m);",
     "acc = add_mod(acc, (uint64_t)x[i] % m, m);", 0),
]


def _mutate(text, old, new, occ):
    assert text.count(old) >= occ + 1, old
    idx = -1
    for _ in range(occ + 1):
        idx = text.index(old, idx + 1)
    return text[:idx] + new + text[idx + len(old):]


@pytest.mark.parametrize("name,old,new,occ", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new, occ):
    src = open(SRC).read()
    mutated = _mutate(src, old, new, occ)
    assert mutated != src
    cpath = tmp_path / "ntt_oracle.c"
    cpath.write_text(mutated)
    so = tmp_path / f"mut_{name}.so"
    import subprocess
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", str(cpath), "-o", str(so)], check=True)
    orc = oracle.Oracle(oracle.load(str(so)))
    caught = []
    for pin in ALL_PINS:
        try:
            pin(orc)
        except (AssertionError, ValueError, ZeroDivisionError, OverflowError) as e:  # noqa: PERF203
            caught.append((pin.__name__, type(e).__name__))
    assert caught, f"mutant {name} passed every pin"
