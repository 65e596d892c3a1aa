"""The device kernels round a clamped binary64 value c in [0, L] with
trunc(c + h), h = 0.5 - 2^-54, instead of round-half-away-from-zero. This
checks that identity on the host (numpy binary64 arithmetic is IEEE) over every
half-integer and integer up to 65540, each +-64 ulps, plus special values,
against round-half-away computed exactly as floor + exact fraction compare."""
import numpy as np

H = np.float64(0.5) - np.float64(2.0) ** -54


def half_away_clamped(x, L):
    """Definition: round half away from zero, then clamp to [0, L-1]; NaN -> 0."""
    with np.errstate(invalid="ignore"):
        f = np.floor(x)
        r = np.where(x - f >= 0.5, f + 1, f)  # x - floor(x) is exact below 2^52
        r = np.where(np.isnan(x), 0, r)
        return np.clip(r, 0, L - 1).astype(np.int64)


def device_form(x, L):
    c = np.fmin(np.fmax(x, 0.0), np.float64(L))  # fmax/fmin drop a NaN operand
    r = np.trunc(c + H).astype(np.int64)
    return np.minimum(r, L - 1)


def sweep_values():
    base = np.arange(-8, 2 * 65540 + 1, dtype=np.float64) * 0.5
    cols = [base]
    up, dn = base.copy(), base.copy()
    for _ in range(64):
        up = np.nextafter(up, np.inf)
        dn = np.nextafter(dn, -np.inf)
        cols += [up, dn]
    tiny = np.ldexp(1.0, np.arange(-1074, 20))
    special = np.array([np.nan, np.inf, -np.inf, 0.0, -0.0, H, 0.5, 1.5 - 2.0 ** -52])
    return np.concatenate(cols + [tiny, np.nextafter(tiny, 0), -tiny, special])


def test_h_is_predecessor_of_half():
    assert H == np.nextafter(np.float64(0.5), 0.0)


def test_trunc_of_c_plus_h_is_half_away_rounding():
    x = sweep_values()
    for L in (2, 3, 1000, 1024, 4096, 65536):
        want = half_away_clamped(x, L)
        got = device_form(x, L)
        bad = np.flatnonzero(want != got)
        assert bad.size == 0, f"L={L}: x={x[bad[:5]]!r} want {want[bad[:5]]} got {got[bad[:5]]}"


def test_plain_half_would_fail():
    """The reason for h: with 0.5 itself, c = 0.5 - 2^-54 would round up to 1."""
    c = np.float64(0.5) - np.float64(2.0) ** -54
    assert np.trunc(c + 0.5) == 1.0 and np.trunc(c + H) == 0.0
