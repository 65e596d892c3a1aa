"""The oracle's least-squares fit (§III.B) against facts fixed outside it.
CPU only."""
import pytest

import oracle
import pins_fit


@pytest.fixture(scope="module")
def o():
    return oracle.get()


@pytest.mark.parametrize("pin", pins_fit.ALL_FIT_PINS, ids=lambda p: p.__name__)
def test_fit_pin(o, pin):
    pin(o)
