"""The CPU oracle against its pins (no GPU).  See ``oracle_pins.py``."""
import pytest

import oracle
from tests.oracle_pins import ALL_PINS, pin_closed_forms, pin_roundtrip


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle(oracle.load(rebuild=True))


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_closed_forms_full_length(orc):
    """The closed forms at the headline length L = 2^20 (30-bit prime) and at 2^18 (62-bit prime)."""
    from paper_1205_2926_amd.workloads import P30, G30, P62, G62
    pin_closed_forms(orc, l=20, primes=((P30, G30),))
    pin_closed_forms(orc, l=18, primes=((P62, G62),))


def test_roundtrip_full_length(orc):
    pin_roundtrip(orc, l30=20, l62=20)
