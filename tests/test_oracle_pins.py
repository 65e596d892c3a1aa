"""The CPU oracle against facts fixed outside it (closed forms, exact
arithmetic, brute force, invariants). CPU only."""
import numpy as np
import pytest

import oracle
import pins


@pytest.fixture(scope="module")
def o():
    return oracle.get()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(o, pin):
    pin(o)


def test_exact_rational_mismatch_count(o):
    # Diagnostic: how often the fixed binary64 evaluation order differs from
    # rounding the exact real value (only possible next to halfway points).
    n = pins.pin_exact_rational(o, detectors=6)
    assert n <= 2


def test_saturating_index(o):
    # DN values at or above L index the last LUT entry (not a wrap-around mask).
    L = 1024
    lut = np.arange(2 * L, dtype=np.uint16).reshape(1, 2, L) % 997
    dn = np.array([[[1023, 1024], [2047, 65535]]], dtype=np.uint16)
    out = o.correct(dn, lut)
    assert out.tolist() == [[[lut[0, 0, 1023], lut[0, 1, 1023]],
                             [lut[0, 0, 1023], lut[0, 1, 1023]]]]


def test_in_place(o):
    rng = np.random.default_rng(3)
    dn = rng.integers(0, 1024, size=(2, 9, 11)).astype(np.uint16)
    lut = rng.integers(0, 1024, size=(2, 11, 1024)).astype(np.uint16)
    want = o.correct(dn, lut)
    o.lib.oracle_correct(oracle._u16(dn), oracle._u16(lut), 9, 11, 2, 1024, oracle._u16(dn))
    assert np.array_equal(dn, want)
