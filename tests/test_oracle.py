"""The oracle's pins (see tests/_pins.py): closed forms, dense sampling, an
independent clamped formula, a NumPy twin and invariants."""
import pytest

from tests._pins import PINS


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__[4:] for p in PINS])
def test_oracle_pin(pin):
    pin()
