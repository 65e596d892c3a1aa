"""Checks that pin the CPU oracle to facts fixed outside it.

Each ``pin_*`` function takes an ``oracle.Oracle`` and raises AssertionError
when the oracle disagrees with the fact it checks. The facts are: closed-form
entries worked out by hand (tests/golden), exact integer arithmetic on dyadic
coefficients, the exact rational value of the polynomial together with the
binary64 Horner error bound, brute force per-pixel evaluation, and layout
invariants. None of them retypes the oracle's Horner formula.

The paper (§I) only names the task; the definition these checks encode is the
one documented in oracle/oracle.hpp.
"""
import math
import os
from fractions import Fraction

import numpy as np

import gen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
LEVELS_EDGE = (2, 3, 1000, 1024, 4096, 65536)


# --- exact arithmetic helpers (Python integers / Fractions, no binary64) -----------

def exact_value(a, v):
    """The polynomial a0 + a1 v + a2 v^2 + a3 v^3 as an exact Fraction."""
    return sum((Fraction(float(a[k])) * (v ** k) for k in range(4)), Fraction(0))


def round_half_away_exact(q):
    """Nearest integer to the Fraction q, halfway cases away from zero."""
    if q >= 0:
        return math.floor(q + Fraction(1, 2))
    return -math.floor(-q + Fraction(1, 2))


def clamp_entry(r, levels):
    return min(max(r, 0), levels - 1)


def horner_error_bound(a, v):
    """Forward error bound of binary64 Horner with 3 multiplies and 3 adds
    (Higham, Accuracy and Stability of Numerical Algorithms, eq. 5.3):
    |fl(p) - p| <= gamma_6 * sum |a_k| v^k, gamma_n = n u / (1 - n u), u = 2^-53."""
    u = Fraction(1, 2 ** 53)
    g6 = 6 * u / (1 - 6 * u)
    return g6 * sum((abs(Fraction(float(a[k]))) * (v ** k) for k in range(4)), Fraction(0))


def near_tie(q, bound):
    """True when some halfway point k + 1/2 lies within ``bound`` of q."""
    f = q - math.floor(q)
    return abs(f - Fraction(1, 2)) <= bound


# --- fixtures --------------------------------------------------------------------

def load_round_clamp():
    rows = []
    with open(os.path.join(GOLDEN, "round_clamp.txt")) as fh:
        for line in fh:
            body = line.split("#", 1)[0].split()
            if not body:
                continue
            a = [float.fromhex(t) if t.lower().lstrip("-").startswith("0x") else float(t)
                 for t in body[:4]]
            rows.append((a, int(body[4]), int(body[5]), int(body[6]), line.strip()))
    return rows


def dyadic_sets():
    """Coefficient sets whose every binary64 Horner operation is exact for
    v < 4096: small integers and fractions with power-of-two denominators."""
    return [
        (3.0, 1.0, 2.0 ** -12, 0.0),
        (-7.0, 0.75, 2.0 ** -10, 2.0 ** -24),
        (100.5, -0.5, 2.0 ** -9, 0.0),
        (0.5, 1.0, 0.0, 0.0),
        (-0.5, 1.25, -2.0 ** -13, 2.0 ** -26),
        (1023.0, -1.0, 0.0, 0.0),
    ]


# --- pins ------------------------------------------------------------------------

def pin_golden(o):
    """Hand-derived closed-form entries (rounding, ties, clamps, NaN/Inf, order)."""
    for a, levels, v, want, text in load_round_clamp():
        got = o.lut_entry(np.array(a), v, levels)
        assert got == want, f"golden case failed: got {got}: {text}"
        # The same entry through the table and through the per-pixel path.
        lut = o.lut_build(np.array(a, dtype=np.float64).reshape(1, 1, 4), levels)
        assert int(lut[0, 0, v]) == want, f"lut_build disagrees on: {text}"


def pin_identity(o):
    """a = (0, 1, 0, 0) returns the input unchanged (saturated at L-1)."""
    rng = np.random.default_rng(7)
    for levels in LEVELS_EDGE:
        a = np.zeros((2, 3, 4))
        a[..., 1] = 1.0
        lut = o.lut_build(a, levels)
        want = np.broadcast_to(np.arange(levels, dtype=np.uint16), (2, 3, levels))
        assert np.array_equal(lut, want), f"identity LUT wrong at L={levels}"
        dn = rng.integers(0, 65536, size=(2, 5, 3), dtype=np.uint16)
        dn[0, 0, 0] = 65535
        dn[1, 4, 2] = levels - 1
        out = o.correct(dn, lut)
        assert np.array_equal(out, np.minimum(dn, levels - 1)), f"identity apply at L={levels}"


def pin_half_offset(o):
    """a = (0.5, 1, 0, 0): every v gives v + 1/2 exactly, which rounds away from
    zero to v + 1 (clamped to L-1); half-to-even would return v for even v."""
    for levels in (2, 3, 1024, 4096):
        lut = o.lut_build(np.array([[[0.5, 1.0, 0.0, 0.0]]]), levels)[0, 0]
        want = np.minimum(np.arange(levels) + 1, levels - 1)
        assert np.array_equal(lut, want), f"half offset at L={levels}"


def pin_dyadic_exact(o):
    """Dyadic coefficients keep every operation exact, so the entry equals the
    exactly rounded integer value, computed here with Python integers."""
    for a in dyadic_sets():
        for levels in (1024, 4096):
            lut = o.lut_build(np.array(a, dtype=np.float64).reshape(1, 1, 4), levels)[0, 0]
            want = [clamp_entry(round_half_away_exact(exact_value(a, v)), levels)
                    for v in range(levels)]
            bad = np.nonzero(lut != np.array(want))[0]
            assert bad.size == 0, f"dyadic {a} L={levels}: first bad v={bad[:5]}"


def exact_mismatches(o, coeffs, levels):
    """Entries where the oracle differs from clamp(round(exact P(v))).

    Returns (count, count_not_near_tie). A difference is only legitimate when
    the exact value lies within the Horner error bound of a halfway point."""
    lut = o.lut_build(coeffs, levels)
    B, D, _ = coeffs.shape
    total = bad = 0
    for b in range(B):
        for d in range(D):
            a = coeffs[b, d]
            num = [Fraction(float(a[k])) for k in range(4)]
            for v in range(levels):
                q = num[0] + v * (num[1] + v * (num[2] + v * num[3]))
                want = clamp_entry(round_half_away_exact(q), levels)
                if int(lut[b, d, v]) != want:
                    total += 1
                    if not near_tie(q, horner_error_bound(a, v)):
                        bad += 1
    return total, bad


def pin_exact_rational(o, detectors=6):
    """Seeded workload coefficients: every entry equals the exactly rounded
    value of the real polynomial, except within the binary64 error bound of a
    halfway point (where the fixed evaluation order decides)."""
    s0 = gen.workload(0)
    s2 = gen.workload(2)
    c0 = gen.coeffs(s0.seed, s0.cfg, 0, s0.coef_kind, 1, detectors)
    c2 = gen.coeffs(s2.seed, s2.cfg, 0, s2.coef_kind, 1, detectors // 2)
    n0, bad0 = exact_mismatches(o, c0, 1024)
    n2, bad2 = exact_mismatches(o, c2, 4096)
    assert bad0 == 0 and bad2 == 0, f"{bad0 + bad2} entries off beyond the error bound"
    return n0 + n2


def brute_force_pixel(coeffs, dn, levels):
    """Per-pixel exact evaluation in Python integers/Fractions (tiny inputs only)."""
    B, N, D = dn.shape
    out = np.empty_like(dn)
    amb = np.zeros(dn.shape, dtype=bool)
    for b in range(B):
        for n in range(N):
            for d in range(D):
                v = min(int(dn[b, n, d]), levels - 1)
                a = coeffs[b, d]
                q = exact_value(a, v)
                out[b, n, d] = clamp_entry(round_half_away_exact(q), levels)
                amb[b, n, d] = near_tie(q, horner_error_bound(a, v))
    return out, amb


def tiny_case(seed, B, N, D, levels):
    rng = np.random.default_rng(seed)
    coeffs = np.zeros((B, D, 4))
    coeffs[..., 0] = rng.normal(0, levels / 128, size=(B, D))
    coeffs[..., 1] = rng.uniform(0.8, 1.2, size=(B, D))
    coeffs[..., 2] = rng.normal(0, 4.0 / levels, size=(B, D))
    coeffs[..., 3] = rng.normal(0, 1.0 / levels ** 2, size=(B, D))
    dn = rng.integers(0, levels + levels // 4 + 1, size=(B, N, D)).astype(np.uint16)
    dn.flat[0] = 65535
    return coeffs, dn


def pin_brute_force(o):
    """correct(lut_build(a)) equals direct per-pixel evaluation, both the
    oracle's own table-free path and exact integer arithmetic."""
    shapes = [(3, 7, 37, 1024), (1, 1, 1, 2), (2, 5, 17, 3), (1, 4, 9, 1000),
              (2, 3, 5, 4096), (1, 2, 3, 65536)]
    for i, (B, N, D, L) in enumerate(shapes):
        coeffs, dn = tiny_case(100 + i, B, N, D, L)
        out = o.correct(dn, o.lut_build(coeffs, L))
        assert np.array_equal(out, o.pixel(coeffs, dn, L)), f"table != per-pixel {B, N, D, L}"
        want, amb = brute_force_pixel(coeffs, dn, L)
        diff = (out != want) & ~amb
        assert not diff.any(), f"oracle != exact brute force at {np.argwhere(diff)[:3]}"


def pin_invariants(o):
    """Layout and monotonicity invariants."""
    rng = np.random.default_rng(11)
    B, N, D, L = 2, 6, 13, 1024
    coeffs = np.zeros((B, D, 4))
    coeffs[..., 0] = rng.uniform(-20, 20, size=(B, D))
    coeffs[..., 1] = rng.uniform(0.5, 1.5, size=(B, D))
    coeffs[..., 2] = rng.uniform(0, 1e-4, size=(B, D))
    coeffs[..., 3] = rng.uniform(0, 1e-8, size=(B, D))
    lut = o.lut_build(coeffs, L)
    # Non-decreasing polynomial on [0, L) -> non-decreasing LUT rows.
    assert (np.diff(lut.astype(np.int64), axis=2) >= 0).all(), "monotone rows"
    assert lut.max() <= L - 1
    # Each (band, detector) row depends only on its own coefficients.
    assert np.array_equal(lut[1, 4], o.lut_build(coeffs[1:2, 4:5], L)[0, 0])
    dn = rng.integers(0, 1100, size=(B, N, D)).astype(np.uint16)
    out = o.correct(dn, lut)
    assert out.max() <= L - 1
    # Permuting detectors with their coefficients permutes output columns.
    perm = rng.permutation(D)
    out_p = o.correct(dn[:, :, perm], o.lut_build(coeffs[:, perm], L))
    assert np.array_equal(out_p, out[:, :, perm]), "detector permutation"
    # Splitting lines into chunks concatenates the outputs.
    parts = [o.correct(dn[:, a:b].copy(), lut) for a, b in ((0, 2), (2, 5), (5, 6))]
    assert np.array_equal(np.concatenate(parts, axis=1), out), "line split"
    # Splitting bands likewise.
    parts = [o.correct(dn[b:b + 1].copy(), lut[b:b + 1].copy()) for b in range(B)]
    assert np.array_equal(np.concatenate(parts, axis=0), out), "band split"
    # Output at (b, n, d) is the LUT row of (b, d) read at min(dn, L-1).
    b, n, d = 1, 3, 7
    assert out[b, n, d] == lut[b, d, min(int(dn[b, n, d]), L - 1)]


ALL_PINS = [pin_golden, pin_identity, pin_half_offset, pin_dyadic_exact,
            pin_brute_force, pin_invariants, pin_exact_rational]
