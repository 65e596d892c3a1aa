"""Checks that pin the oracle's least-squares fit to facts fixed outside it.

The fit is case study 2 of the paper (§III.B): a polynomial of order m fitted
to n points by the normal equations, solved as A^-1 B. Each ``pin_fit_*``
takes an ``oracle.Oracle`` and raises AssertionError on disagreement. The
facts: fits worked out by hand as exact rationals (tests/golden/fit_cases.txt),
the textbook centred formula for a straight line, numpy's SVD-based
``polyfit`` (a different algorithm), exact recovery of noise-free
polynomials, exact linearity in y, the normal equations holding for the
residual, singular systems, and the array layout. None of them retypes the
oracle's sums or elimination.
"""
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fit_cases.txt")


def load_fit_cases():
    cases = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            t = line.split()
            m = int(t[0])
            pts = [tuple(float(Fraction(v)) for v in p.split(":")) for p in t[1:] if ":" in p]
            rest = [v for v in t[1:] if ":" not in v]
            want = [float("nan") if v == "nan" else float(Fraction(v)) for v in rest]
            cases.append((m, np.array([p[0] for p in pts]), np.array([p[1] for p in pts]),
                          np.array(want)))
    return cases


def fit1(o, x, y, m):
    """One detector, one band: x, y 1-D -> coefficients a0..a3."""
    n = len(x)
    return o.fit(np.asarray(x, np.float64).reshape(1, n, 1),
                 np.asarray(y, np.float64).reshape(1, n), m)[0, 0]


def close(got, want, rel):
    scale = max(1.0, float(np.max(np.abs(want))))
    return np.all(np.abs(got - want) <= rel * scale)


def kappa(x, m):
    """2-norm condition number of the normal matrix of points x, order m."""
    x = np.asarray(x, np.float64)
    A = np.array([[np.sum(x ** (j + k)) for k in range(m + 1)] for j in range(m + 1)])
    return float(np.linalg.cond(A))


def fit_tol(x, m):
    """Relative forward-error allowance for solving the normal equations in
    binary64: a small multiple of (m + 1) * eps * cond(A)."""
    return 8.0 * (m + 1) * np.finfo(np.float64).eps * kappa(x, m)


def pin_fit_golden(o):
    for m, x, y, want in load_fit_cases():
        got = fit1(o, x, y, m)
        if np.isnan(want).all():
            assert np.isnan(got).all(), f"singular case m={m} x={x}: {got}"
        else:
            assert close(got, want, fit_tol(x, m)), f"m={m} x={x} y={y}: {got} != {want}"


def pin_fit_closed_form_line(o):
    """Order 1 against slope = sum (x - xm)(y - ym) / sum (x - xm)^2."""
    rng = np.random.default_rng(21)
    for _ in range(20):
        n = int(rng.integers(2, 12))
        x = rng.uniform(0, 1000, n)
        y = 3.0 + 0.9 * x + rng.normal(0, 5, n)
        xm, ym = x.mean(), y.mean()
        slope = np.sum((x - xm) * (y - ym)) / np.sum((x - xm) ** 2)
        got = fit1(o, x, y, 1)
        assert close(got[:2], np.array([ym - slope * xm, slope]), 1e-8), (got, slope)


def pin_fit_polyfit(o):
    """Orders 0-3 on well-conditioned data against numpy.polyfit (SVD)."""
    rng = np.random.default_rng(22)
    for m in range(4):
        for _ in range(10):
            n = int(rng.integers(m + 1, 10))
            x = np.sort(rng.uniform(-3, 3, n))
            if np.min(np.diff(x)) < 0.05:
                continue
            y = rng.normal(0, 2, n)
            want = np.polyfit(x, y, m)[::-1]
            got = fit1(o, x, y, m)
            assert close(got[:m + 1], want, 1e-8), (m, got, want)
            assert np.all(got[m + 1:] == 0.0)


def pin_fit_noise_free(o):
    """Points on a polynomial of order <= m are reproduced (x = 0..5, the
    paper's six calibration lines, and a 10-bit DN range)."""
    polys = [np.array([2.0, 0, 0, 0]), np.array([-1.5, 0.75, 0, 0]),
             np.array([3.0, -0.5, 0.125, 0]), np.array([1.0, 2.0, -0.25, 0.0625])]
    for deg, p in enumerate(polys):
        for x in (np.arange(6.0), np.linspace(40.0, 1000.0, 6)):
            y = p[0] + p[1] * x + p[2] * x ** 2 + p[3] * x ** 3
            for m in range(deg, 4):
                tol = fit_tol(x, m)
                if tol > 1e-3:
                    continue  # too ill-conditioned for a meaningful pin (order 3, 10-bit range)
                got = fit1(o, x, y, m)
                assert close(got, p, tol), (deg, m, x, got)


def pin_fit_linear_in_y(o):
    """Scaling y by 2 scales every coefficient by exactly 2 (every operation
    on y is linear and exact under a power-of-two scale); a constant added to
    y moves a0 by that constant."""
    rng = np.random.default_rng(23)
    B, n, D = 2, 6, 5
    x = rng.uniform(0, 100, (B, n, D))
    y = rng.uniform(0, 100, (B, n))
    for m in range(4):
        a = o.fit(x, y, m)
        assert np.array_equal(o.fit(x, 2.0 * y, m), 2.0 * a), f"2y, m={m}"
    a = o.fit(x, y, 1)
    a7 = o.fit(x, y + 7.0, 1)
    assert np.allclose(a7[..., 0] - a[..., 0], 7.0, rtol=0, atol=1e-9)
    assert np.allclose(a7[..., 1], a[..., 1], rtol=0, atol=1e-11)


def pin_fit_normal_equations(o):
    """The residual r = y - f(x) is orthogonal to 1, x, ..., x^m."""
    rng = np.random.default_rng(24)
    for m in range(4):
        n = 9
        x = np.linspace(-2, 2, n) + rng.uniform(-0.05, 0.05, n)
        y = rng.normal(0, 1, n)
        a = fit1(o, x, y, m)
        r = y - sum(a[j] * x ** j for j in range(m + 1))
        for j in range(m + 1):
            assert abs(np.sum(r * x ** j)) <= 1e-10 * np.sum(np.abs(y * x ** j)), (m, j)


def pin_fit_singular(o):
    """Identical x on every line: singular for order >= 1 (all NaN); order 0
    is the mean and never singular."""
    x = np.full(5, 3.0)
    y = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    for m in (1, 2, 3):
        assert np.isnan(fit1(o, x, y, m)).all()
    a = fit1(o, x, y, 0)
    assert a[0] == 3.0 and np.all(a[1:] == 0.0)


def pin_fit_layout(o):
    """x is [bands][points][detectors], y is [bands][points], the result is
    [bands][detectors][4]; each (band, detector) depends on its own column
    and its band's targets only, and coefficients above the order are +0."""
    rng = np.random.default_rng(25)
    B, n, D, m = 3, 6, 7, 2
    x = rng.uniform(0, 50, (B, n, D))
    y = rng.uniform(0, 50, (B, n))
    a = o.fit(x, y, m)
    assert a.shape == (B, D, 4)
    for b in range(B):
        for d in range(D):
            assert np.array_equal(a[b, d], fit1(o, x[b, :, d], y[b], m)), (b, d)
    assert np.all(a[..., 3] == 0.0) and not np.signbit(a[..., 3]).any()
    perm = rng.permutation(D)
    assert np.array_equal(o.fit(x[:, :, perm], y, m), a[:, perm])


ALL_FIT_PINS = [pin_fit_golden, pin_fit_closed_form_line, pin_fit_polyfit, pin_fit_noise_free,
                pin_fit_linear_in_y, pin_fit_normal_equations, pin_fit_singular, pin_fit_layout]
