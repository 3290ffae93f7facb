"""The CPU oracle against its pins (Table 1, Figure 1, closed forms, a
third-party varint codec, brute force, numpy's wrapping cumsum)."""
import pytest

import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc.oracle.load())
