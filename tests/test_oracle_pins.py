"""The CPU oracle against closed forms, brute force and convergence orders
(see ``tests/pins.py`` for what each pin checks and why it is independent)."""
import pytest

import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=[p.__name__ for p in pins.ALL_PINS])
def test_pin(orc, pin):
    ok, detail = pin(orc)
    print(detail)
    assert ok, detail
