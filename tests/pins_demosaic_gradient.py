"""Checks that pin the oracle's gradient-based demosaicing (the gradient
interpolation named in §II and §III.A; method of Hamilton & Adams, U.S. Patent
5,629,734) to facts fixed outside it: pixels worked out by hand
(tests/golden/demosaic_gradient_cases.txt); the method written the way it is
usually presented, as 1-D filters on the mosaic ([-1 2 2 2 -1] / 4 green
estimates, [1 0 -1] and [-1 0 2 0 -1] gradient terms) followed by interpolation
of colour differences X - G', with scipy's and numpy's mirror borders; linear
ramps reproduced exactly three pixels away from the border; step edges along
rows or columns reproduced exactly everywhere, which bilinear interpolation
does not do; constants; own samples; and the array layout."""
import os

import numpy as np
from scipy import ndimage

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "demosaic_gradient_cases.txt")
IMAGES = {
    "g": [[100, 200, 120, 210], [190, 50, 220, 60], [110, 230, 130, 240], [250, 70, 260, 80]],
    "tie": [[100, 21, 103, 21], [30, 5, 30, 5], [97, 21, 100, 21], [30, 5, 30, 5]],
    "hi": [[65535, 65535, 0, 0], [65535, 0, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0]],
    "lo": [[0, 0, 65535, 0], [0, 0, 65535, 0], [65535, 0, 0, 0], [0, 0, 0, 0]],
    "dtie": [[50, 100, 50, 100], [100, 10, 100, 13], [50, 100, 50, 100], [100, 11, 100, 12]],
}
PLANE = {"R": 0, "G": 1, "B": 2}


def masks(H, W):
    r = np.arange(H)[:, None] % 2
    c = np.arange(W)[None, :] % 2
    red = (r == 0) & (c == 0)
    blue = (r == 1) & (c == 1)
    return red, ~(red | blue), blue


def filter_reference(raw):
    """The adaptive colour plane method as filters and colour differences."""
    I, H, W = raw.shape
    out = np.empty((I, 3, H, W), dtype=np.uint16)
    red, green, blue = masks(H, W)
    f1 = lambda x, k, axis: ndimage.correlate1d(x, np.array(k, np.int64), axis=axis, mode="mirror")
    for i in range(I):
        x = raw[i].astype(np.int64)
        # Green: the estimate along the direction with the smaller gradient.
        est_h, est_v = f1(x, [-1, 2, 2, 2, -1], 1), f1(x, [-1, 2, 2, 2, -1], 0)
        grad_h = np.abs(f1(x, [1, 0, -1], 1)) + np.abs(f1(x, [-1, 0, 2, 0, -1], 1))
        grad_v = np.abs(f1(x, [1, 0, -1], 0)) + np.abs(f1(x, [-1, 0, 2, 0, -1], 0))
        g = np.where(grad_h < grad_v, (est_h + 2) >> 2,
                     np.where(grad_v < grad_h, (est_v + 2) >> 2, (est_h + est_v + 4) >> 3))
        g = np.where(green, x, np.clip(g, 0, 65535))
        # Red and blue: interpolate the colour difference X - G'.
        diff = np.pad(x - g, 1, mode="reflect")
        gp = np.pad(g, 1, mode="reflect")
        xp = np.pad(x, 1, mode="reflect")
        at = lambda a, dr, dc: a[1 + dr:1 + dr + H, 1 + dc:1 + dc + W]
        row_pair = at(diff, 0, -1) + at(diff, 0, 1)
        col_pair = at(diff, -1, 0) + at(diff, 1, 0)
        nw = at(diff, -1, -1) + at(diff, 1, 1)
        ne = at(diff, -1, 1) + at(diff, 1, -1)
        grad_nw = np.abs(at(xp, -1, -1) - at(xp, 1, 1)) + np.abs(2 * g - at(gp, -1, -1) - at(gp, 1, 1))
        grad_ne = np.abs(at(xp, -1, 1) - at(xp, 1, -1)) + np.abs(2 * g - at(gp, -1, 1) - at(gp, 1, -1))
        diag = g + np.where(grad_nw < grad_ne, (nw + 1) >> 1,
                            np.where(grad_ne < grad_nw, (ne + 1) >> 1, (nw + ne + 2) >> 2))
        red_row = (np.arange(H)[:, None] % 2 == 0) & np.ones((1, W), bool)
        for ch, own, other in ((0, red, blue), (2, blue, red)):
            in_row = red_row if ch == 0 else ~red_row
            at_green = g + np.where(in_row, (row_pair + 1) >> 1, (col_pair + 1) >> 1)
            v = np.where(own, x, np.clip(np.where(other, diag, at_green), 0, 65535))
            out[i, ch] = v
        out[i, 1] = g
    return out


def pin_gradient_golden(o):
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if not line:
                continue
            name, plane, r, c, want = line[0], line[1], int(line[2]), int(line[3]), int(line[4])
            img = np.array(IMAGES[name], dtype=np.uint16)[None]
            got = o.demosaic_gradient(img)[0, PLANE[plane], r, c]
            assert got == want, f"{name} {plane}({r},{c}) = {got}, want {want}"


def pin_gradient_filters(o):
    rng = np.random.default_rng(41)
    for H, W in ((4, 4), (4, 8), (6, 4), (8, 12), (10, 6), (64, 36), (4, 40)):
        raw = rng.integers(0, 65536, (2, H, W)).astype(np.uint16)
        assert np.array_equal(o.demosaic_gradient(raw), filter_reference(raw)), (H, W)
        smooth = (ndimage.uniform_filter(raw.astype(np.float64), (1, 5, 5)) / 16).astype(np.uint16)
        assert np.array_equal(o.demosaic_gradient(smooth), filter_reference(smooth)), (H, W)


def pin_gradient_ramp(o):
    """The green estimate and the colour differences are exact on a linear
    function; border reach is two pixels for green, three for red and blue."""
    H, W = 16, 20
    for a, b in ((8, 2), (2, 8), (3, 5), (-3, 7), (5, -2)):
        raw = (a * np.arange(H)[:, None] + b * np.arange(W)[None, :] + 300).astype(np.uint16)
        out = o.demosaic_gradient(raw[None])[0]
        assert np.array_equal(out[1, 2:-2, 2:-2], raw[2:-2, 2:-2]), (a, b)
        for ch in (0, 2):
            assert np.array_equal(out[ch, 3:-3, 3:-3], raw[3:-3, 3:-3]), (a, b, ch)


def pin_gradient_edges(o):
    """A step along columns or rows is reproduced exactly in every plane: the
    gradient across the edge is large, so green is interpolated along it, and
    the colour differences vanish. Bilinear interpolation blurs the step."""
    for k in (3, 4, 5, 6):
        col = np.where(np.arange(12)[None, :] < k, 1000, 3000) * np.ones((12, 1))
        for img in (col, col.T):
            raw = img.astype(np.uint16)[None]
            out = o.demosaic_gradient(raw)[0]
            for ch in range(3):
                assert np.array_equal(out[ch], raw[0]), (k, ch)
            assert not np.array_equal(o.demosaic(raw)[0, 1], raw[0])


def pin_gradient_constant_and_own(o):
    rng = np.random.default_rng(42)
    for v in (0, 1, 777, 65535):
        out = o.demosaic_gradient(np.full((1, 6, 8), v, np.uint16))
        assert np.all(out == v), v
    raw = rng.integers(0, 65536, (1, 8, 10)).astype(np.uint16)
    out = o.demosaic_gradient(raw)[0]
    for ch, m in enumerate(masks(8, 10)):
        assert np.array_equal(out[ch][m], raw[0][m]), f"own samples, plane {ch}"


def pin_gradient_layout(o):
    rng = np.random.default_rng(43)
    raw = rng.integers(0, 4096, (3, 6, 8)).astype(np.uint16)
    out = o.demosaic_gradient(raw)
    assert out.shape == (3, 3, 6, 8)
    for i in range(3):
        assert np.array_equal(out[i], o.demosaic_gradient(raw[i:i + 1])[0]), i


ALL_GRADIENT_PINS = [pin_gradient_golden, pin_gradient_filters, pin_gradient_ramp,
                     pin_gradient_edges, pin_gradient_constant_and_own, pin_gradient_layout]
