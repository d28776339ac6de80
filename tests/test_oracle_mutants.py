"""Each deliberately planted mistake in the oracle must fail at least one pin.

The mutants are compiled from oracle.c with -DORACLE_MUTANT=n into a temporary
directory (CPU only); see the ORACLE_MUTANT blocks in oracle/oracle.c.
"""
import pytest

import oracle
from oracle.build import build
from tests import pins

MUTANTS = {
    1: "encode ties go to the higher index",
    2: "a selected zero gets -1",
    3: "Delta drops the disagreeing terms",
    4: "top-k ties go to the higher id",
    5: "bit planes packed most-significant-bit first",
    6: "rerank keeps the worst candidates",
    7: "rerank ties go to the higher id",
    8: "masked addition ignores the sign",
    9: "b1.58 rounds ties away from zero",
    10: "ternary distance counts differing coordinates",
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS), ids=lambda m: MUTANTS[m].replace(" ", "_"))
def test_mutant_is_caught(mutant, tmp_path):
    lib = oracle.load(build(mutant=mutant, out_dir=str(tmp_path)))
    o = oracle.Oracle(lib)
    failed = []
    for check in pins.ALL_CHECKS:
        try:
            check(o)
        except (AssertionError, oracle.OracleError):
            failed.append(check.__name__)
    assert failed, f"mutant {mutant} ({MUTANTS[mutant]}) passed every pin"
