"""The CPU oracle against facts fixed by the paper and by mathematics."""
import pytest

import oracle_pins as P


@pytest.mark.parametrize("pin", P.FAST_PINS + P.CHAIN_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    fails = pin()
    assert not fails, "\n".join(fails)
