"""The oracle's gradient-based demosaicing (adaptive colour plane
interpolation) against facts fixed outside it. CPU only."""
import pytest

import oracle
import pins_demosaic_gradient


@pytest.fixture(scope="module")
def o():
    return oracle.get()


@pytest.mark.parametrize("pin", pins_demosaic_gradient.ALL_GRADIENT_PINS, ids=lambda p: p.__name__)
def test_gradient_pin(o, pin):
    pin(o)
