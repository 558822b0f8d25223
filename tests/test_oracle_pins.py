"""The oracle against the pins the paper and the mathematics fix (CPU only)."""
import pytest

from . import pins_oracle


@pytest.mark.parametrize("pin", pins_oracle.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin):
    pin()
