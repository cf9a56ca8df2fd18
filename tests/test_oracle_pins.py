"""The oracle against brute force, closed forms and invariants (CPU only)."""

import pytest

from pins import ALL_PINS


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(orc, pin):
    pin(orc)
