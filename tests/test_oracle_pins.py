"""The CPU oracle against closed forms, identities and library routines."""
import pytest

import oracle_pins as pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    assert pin(), pin.__doc__
