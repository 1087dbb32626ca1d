"""The host-CPU re-run of Table 1: both butterflies give the oracle's transform."""
import numpy as np
import pytest

import oracle
from paper_1205_2926_amd import cpu
from paper_1205_2926_amd.workloads import G62, P62


@pytest.mark.parametrize("l", [1, 4, 11])
@pytest.mark.parametrize("alg", [2, 3])
def test_table1_transforms_match_oracle(l, alg):
    orc = oracle.Oracle()
    w = orc.root_of_unity(P62, G62, l)
    x = np.random.Generator(np.random.PCG64(70 + l)).integers(0, P62, size=1 << l, dtype=np.uint64)
    np.testing.assert_array_equal(cpu.forward(x, P62, w, alg), orc.forward(x, l, P62, w))


def test_table1_timing_fields():
    orc = oracle.Oracle()
    w = orc.root_of_unity(P62, G62, 11)
    x = np.random.Generator(np.random.PCG64(71)).integers(0, P62, size=1 << 11, dtype=np.uint64)
    r = cpu.run(x, P62, w, reps=50)
    assert r["alg2"]["ns_per_butterfly"] > 0 and r["alg3"]["tsc_ticks_per_butterfly"] > 0
