"""How the oracle composes Algorithm 1 (Sec. 2): steps 3(a), 4(c)-(d) and 5
pinned by ensembles whose outcome the paper's formulas fix (tests/oracle_pins.py)."""
import pytest

import oracle_pins as P


@pytest.mark.parametrize("pin", P.PINS, ids=[p.__name__ for p in P.PINS])
def test_composition(oracle, pin):
    pin(oracle)
