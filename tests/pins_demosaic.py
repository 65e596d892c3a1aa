"""Checks that pin the oracle's bilinear demosaicing (§III.A) to facts fixed
outside it: pixels worked out by hand (tests/golden/demosaic_cases.txt), the
textbook formulation of bilinear demosaicing as two 3x3 kernels applied to the
sparse colour planes (scipy's mirror mode is the border reading), linear ramps
reproduced exactly inside the image, constants, own samples, full-scale input
and the array layout. None of them retypes the oracle's four cases."""
import os

import numpy as np
from scipy import ndimage

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "demosaic_cases.txt")
IMAGES = {
    "ramp": (8 * np.arange(4)[:, None] + 2 * np.arange(4)[None, :]).astype(np.uint16),
    "half": np.array([[1, 0, 2, 0], [0, 3, 0, 0]], dtype=np.uint16),
}
PLANE = {"R": 0, "G": 1, "B": 2}


def masks(H, W):
    r = np.arange(H)[:, None] % 2
    c = np.arange(W)[None, :] % 2
    red = (r == 0) & (c == 0)
    blue = (r == 1) & (c == 1)
    return red, ~(red | blue), blue


def convolution_reference(raw):
    """Bilinear demosaicing as correlations of the sparse colour planes with
    [[0,1,0],[1,4,1],[0,1,0]] / 4 (green) and [[1,2,1],[2,4,2],[1,2,1]] / 4
    (red, blue), mirrored borders, quotients rounded half up."""
    I, H, W = raw.shape
    kg = np.array([[0, 1, 0], [1, 4, 1], [0, 1, 0]], dtype=np.int64)
    krb = np.array([[1, 2, 1], [2, 4, 2], [1, 2, 1]], dtype=np.int64)
    out = np.empty((I, 3, H, W), dtype=np.uint16)
    for i in range(I):
        for ch, (m, k) in enumerate(zip(masks(H, W), (krb, kg, krb))):
            sparse = np.where(m, raw[i].astype(np.int64), 0)
            num = ndimage.correlate(sparse, k, mode="mirror")
            out[i, ch] = (num + 2) >> 2
    return out


def pin_demosaic_golden(o):
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if not line:
                continue
            name, plane, r, c, want = line[0], line[1], int(line[2]), int(line[3]), int(line[4])
            got = o.demosaic(IMAGES[name][None])[0, PLANE[plane], r, c]
            assert got == want, f"{name} {plane}({r},{c}) = {got}, want {want}"


def pin_demosaic_convolution(o):
    rng = np.random.default_rng(31)
    for H, W in ((2, 2), (2, 4), (4, 4), (6, 8), (10, 6), (64, 36), (2, 40)):
        raw = rng.integers(0, 65536, (2, H, W)).astype(np.uint16)
        assert np.array_equal(o.demosaic(raw), convolution_reference(raw)), (H, W)


def pin_demosaic_ramp(o):
    """Bilinear interpolation reproduces a linear function: every plane equals
    the ramp away from the border (steps even, so every average is exact)."""
    H, W = 12, 16
    raw = (6 * np.arange(H)[:, None] + 10 * np.arange(W)[None, :] + 100).astype(np.uint16)
    out = o.demosaic(raw[None])[0]
    for ch in range(3):
        assert np.array_equal(out[ch, 1:-1, 1:-1], raw[1:-1, 1:-1]), ch


def pin_demosaic_constant_and_own(o):
    rng = np.random.default_rng(32)
    for v in (0, 1, 777, 65535):
        out = o.demosaic(np.full((1, 6, 8), v, np.uint16))
        assert np.all(out == v), v
    raw = rng.integers(0, 65536, (1, 8, 10)).astype(np.uint16)
    out = o.demosaic(raw)[0]
    for ch, m in enumerate(masks(8, 10)):
        assert np.array_equal(out[ch][m], raw[0][m]), f"own samples, plane {ch}"


def pin_demosaic_layout(o):
    rng = np.random.default_rng(33)
    raw = rng.integers(0, 4096, (3, 6, 8)).astype(np.uint16)
    out = o.demosaic(raw)
    assert out.shape == (3, 3, 6, 8)
    for i in range(3):
        assert np.array_equal(out[i], o.demosaic(raw[i:i + 1])[0]), i


ALL_DEMOSAIC_PINS = [pin_demosaic_golden, pin_demosaic_convolution, pin_demosaic_ramp,
                     pin_demosaic_constant_and_own, pin_demosaic_layout]
