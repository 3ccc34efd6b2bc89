"""The CPU oracle against what the paper and the mathematics fix (no GPU)."""
import pytest

import oracle_pins as P


@pytest.mark.parametrize("pin", P.FAST, ids=lambda f: f.__name__)
def test_fast_pin(pin):
    pin()


@pytest.mark.slow
@pytest.mark.parametrize("pin", P.SLOW, ids=lambda f: f.__name__)
def test_slow_pin(pin):
    pin()
