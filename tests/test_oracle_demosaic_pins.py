"""The oracle's bilinear demosaicing (§III.A) against facts fixed outside it.
CPU only."""
import pytest

import oracle
import pins_demosaic


@pytest.fixture(scope="module")
def o():
    return oracle.get()


@pytest.mark.parametrize("pin", pins_demosaic.ALL_DEMOSAIC_PINS, ids=lambda p: p.__name__)
def test_demosaic_pin(o, pin):
    pin(o)
