"""GPU path (through the C ABI) against the CPU oracle, bit-exact.

Covers the hand-derived golden entries, the three single-scene workloads at
full size with the plan the benchmark times, ragged and degenerate shapes,
every launch-shape knob on both correction paths, in-place correction,
2-byte-aligned pointers and out-of-bounds write guards."""
import itertools

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_1505_05655_amd as rc
import pins
from gpu_util import Guarded, dev, to_dev_f64, to_dev_u16, to_host_u16

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def o():
    return oracle.get()


def run_case(o, coeffs, dn, levels, plan=None, dn_offset=0, out_offset=0, in_place=False):
    """Build + correct on the GPU; return (lut, out) on the host and check the
    guard bands."""
    B, N, D = dn.shape
    lut_g = Guarded((B, D, levels))
    rc.lut_build(to_dev_f64(coeffs), levels, lut=lut_g.t)
    dn_g = Guarded((B, N, D), offset=dn_offset)
    dn_g.t.copy_(to_dev_u16(dn))
    if in_place:
        out_g = dn_g
    else:
        out_g = Guarded((B, N, D), offset=out_offset)
    rc.correct(dn_g.t, lut_g.t, out=out_g.t, plan=plan)
    torch.cuda.synchronize()
    for g in (lut_g, dn_g, out_g):
        g.check_pads()
    return lut_g.host(), out_g.host()


def expect(o, coeffs, dn, levels):
    lut = o.lut_build(coeffs, levels)
    return lut, o.correct(dn, lut)


def test_golden_entries():
    rows = pins.load_round_clamp()
    for a, levels, v, want, text in rows:
        lut = rc.lut_build(to_dev_f64(np.array(a).reshape(1, 1, 4)), levels)
        got = int(to_host_u16(lut)[0, 0, v])
        assert got == want, f"GPU golden case failed: got {got}: {text}"


@pytest.mark.parametrize("w", [0, 1, 2])
def test_lut_build_workloads(o, w):
    s = gen.workload(w)
    coeffs = s.coeffs()
    lut = to_host_u16(rc.lut_build(to_dev_f64(coeffs), s.levels))
    assert np.array_equal(lut, o.lut_build(coeffs, s.levels))


@pytest.mark.parametrize("levels", [2, 3, 7, 1000, 1023, 1024, 4097, 65536])
def test_lut_build_levels_and_specials(o, levels):
    rng = np.random.default_rng(levels)
    coeffs = np.zeros((2, 5, 4))
    coeffs[..., 0] = rng.normal(0, levels / 64, size=(2, 5))
    coeffs[..., 1] = rng.uniform(0.5, 1.5, size=(2, 5))
    coeffs[..., 2] = rng.normal(0, 2.0 / levels, size=(2, 5))
    coeffs[..., 3] = rng.normal(0, 1.0 / levels ** 2, size=(2, 5))
    coeffs[0, 0] = [np.nan, 1, 0, 0]
    coeffs[0, 1] = [np.inf, 0, 0, 0]
    coeffs[0, 2] = [-np.inf, 0, 0, 0]
    coeffs[1, 0] = [0.5, 1, 0, 0]
    coeffs[1, 1] = [0, 1, 0, 0]
    want = o.lut_build(coeffs, levels)
    # Aligned and misaligned (2-byte) LUT pointers take different store paths.
    for off in (0, 1):
        g = Guarded((2, 5, levels), offset=off)
        rc.lut_build(to_dev_f64(coeffs), levels, lut=g.t)
        torch.cuda.synchronize()
        g.check_pads()
        assert np.array_equal(g.host(), want), f"L={levels} offset={off}"


SHAPES = [
    (1, 1, 1, 2),          # single pixel, smallest L
    (3, 7, 37, 1024),      # tiny ragged
    (2, 333, 1000, 1024),  # ragged strip and line tails
    (1, 1030, 1031, 1024),  # odd detector count -> one pixel per lane
    (1, 1030, 1030, 1024),  # 2 mod 4 detector count
    (2, 517, 130, 4096),   # 12-bit LUT, narrow strips
    (1, 64, 12000, 1024),  # wide line, few lines
    (1, 3, 5, 65536),      # 16-bit LUT -> L2 path
    (2, 100, 300, 3),      # three levels
    (1, 2000, 8, 1000),    # narrower than a strip, non-power-of-two L
    (4, 50, 70, 1024),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_correct_shapes(o, shape):
    B, N, D, L = shape
    coeffs, dn = pins.tiny_case(sum(shape), B, N, D, L)
    want_lut, want = expect(o, coeffs, dn, L)
    lut, out = run_case(o, coeffs, dn, L)
    assert np.array_equal(lut, want_lut)
    assert np.array_equal(out, want)


def plans_for(N, D, L):
    plans = []
    for path, strip, vec, threads, unroll, xcd, nt in itertools.product(
            (rc.RC_PATH_LDS, rc.RC_PATH_L2, rc.RC_PATH_PACKED), (8, 16, 64, 256), (1, 2, 4),
            (256, 1024), (4, 16), (0, 1), (0, 1, 2)):
        if path == rc.RC_PATH_LDS and strip * L * 2 > 128 * 1024:
            continue
        if path == rc.RC_PATH_PACKED and (L + 31) // 32 * strip * 10 > 128 * 1024:
            continue
        if strip // vec > threads:
            continue
        if (strip + vec + threads + unroll + xcd + nt + path) % 4:  # thin the grid
            continue
        for chunk in (1, 37, N):
            plans.append(rc.Plan(path=path, strip=strip, vec=vec, threads=threads, unroll=unroll,
                                 chunk_lines=chunk, xcd_remap=xcd, nontemporal=nt))
    return plans


@pytest.mark.parametrize("shape", [(2, 301, 1000, 1024), (1, 211, 600, 4096)],
                         ids=lambda s: "x".join(map(str, s)))
def test_correct_forced_plans(o, shape):
    B, N, D, L = shape
    coeffs, dn = pins.tiny_case(7, B, N, D, L)
    want_lut, want = expect(o, coeffs, dn, L)
    lut_t = rc.lut_build(to_dev_f64(coeffs), L)
    dn_t = to_dev_u16(dn)
    plans = plans_for(N, D, L)
    assert len(plans) > 20
    for plan in plans:
        out = Guarded((B, N, D))
        rc.correct(dn_t, lut_t, out=out.t, plan=plan)
        torch.cuda.synchronize()
        out.check_pads()
        assert np.array_equal(out.host(), want), f"plan {plan}"


UNEVEN_SHAPES = [(3, 401, 6000, 4096), (2, 257, 1000, 1024), (1, 1000, 24, 1024), (2, 33, 8, 3),
                 (1, 100, 1000, 65536)]


@pytest.mark.parametrize("shape", UNEVEN_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_uneven_strips(o, shape):
    """Strips of nearly equal, non-power-of-two widths (the `strips` plan
    field), 1 to 8 pixels per lane (8: 16-byte accesses), every LUT mode,
    line chunks that leave a ragged last chunk."""
    B, N, D, L = shape
    coeffs, dn = pins.tiny_case(D + L, B, N, D, L)
    rng = np.random.default_rng(D)
    coeffs[..., 0] = rng.normal(0, L / 128, size=(B, D))
    coeffs[..., 1] = rng.uniform(0.9, 1.1, size=(B, D))
    coeffs[..., 2] = rng.normal(0, 0.05 / L, size=(B, D))
    coeffs[..., 3] = 0.0
    want_lut, want = expect(o, coeffs, dn, L)
    lut_t = rc.lut_build(to_dev_f64(coeffs), L)
    dn_t = to_dev_u16(dn)
    n = 0
    for path, vec, strips, threads, unroll, chunk, nt, lmap in itertools.product(
            (rc.RC_PATH_PACKED, rc.RC_PATH_LDS, rc.RC_PATH_L2, rc.RC_PATH_DENSE), (8, 4, 2, 1),
            (1, 3, 7, 85),
            (256, 1024), (4, 8), (N, 37), (0, 2, 4, 5), (0, 1)):
        if D % vec or strips > D // vec:
            continue
        if (vec + strips + threads + unroll + chunk + nt + 5 * lmap) % 7:  # thin the grid
            continue
        widest = vec * -(-(D // vec) // strips)
        W = 1
        while W < widest:
            W <<= 1
        lds = {rc.RC_PATH_LDS: W * L * 2, rc.RC_PATH_PACKED: (L + 31) // 32 * W * 10,
               rc.RC_PATH_DENSE: (L + 63) // 64 * W * 10, rc.RC_PATH_L2: 0}[path]
        if lds > 160 * 1024 or W > 1024 or W // vec > threads:
            continue
        if path == rc.RC_PATH_DENSE and (L > 8192 or threads > 512):
            continue
        if vec == 8 and unroll != 4:
            continue
        plan = rc.Plan(path=path, strip=W, vec=vec, threads=threads, unroll=unroll,
                       chunk_lines=chunk, xcd_remap=1, nontemporal=nt, strips=strips,
                       lane_map=lmap)
        out = Guarded((B, N, D))
        rc.correct(dn_t, lut_t, out=out.t, plan=plan)
        torch.cuda.synchronize()
        out.check_pads()
        assert np.array_equal(out.host(), want), f"plan {plan}"
        n += 1
    assert n >= 3


def test_uneven_plan_rejects():
    """strips beyond the unit count, or strips wider than W: RC_EINVAL."""
    dn = torch.zeros((1, 4, 64), dtype=torch.int16, device=dev())
    lut = torch.zeros((1, 64, 1024), dtype=torch.int16, device=dev())
    base = dict(path=rc.RC_PATH_PACKED, strip=64, vec=8, threads=256, unroll=4, chunk_lines=4,
                xcd_remap=1, nontemporal=0, strips=1)
    for upd in ({"strips": 9}, {"strips": 1, "strip": 32}, {"strips": -1}, {"unroll": 8}):
        d = dict(base)
        d.update(upd)
        with pytest.raises(rc.RcError) as e:
            rc.correct(dn, lut, plan=rc.Plan(**d))
        assert e.value.status == rc.RC_EINVAL, upd
    rc.correct(dn, lut, plan=rc.Plan(**base))
    torch.cuda.synchronize()


PACKED_SHAPES = [(2, 301, 1000, 1024), (1, 77, 333, 1000), (3, 40, 50, 3), (1, 65, 130, 4096),
                 (1, 9, 64, 33), (2, 31, 520, 2048)]


@pytest.mark.parametrize("shape", PACKED_SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("packable", [True, False])
def test_packed_path(o, shape, packable):
    """Packed LDS tiles: exact for packable rows (steps 0..3), and exact through
    the global-gather fallback for rows that are not (decreasing or steep)."""
    B, N, D, L = shape
    coeffs, dn = pins.tiny_case(L + N, B, N, D, L)
    rng = np.random.default_rng(L + D)
    # Gain near 1 and a small curvature: rows rise by 0, 1 or 2 per level.
    coeffs[..., 0] = rng.normal(0, L / 128, size=(B, D))
    coeffs[..., 1] = rng.uniform(0.9, 1.1, size=(B, D))
    coeffs[..., 2] = rng.normal(0, 0.05 / L, size=(B, D))
    coeffs[..., 3] = 0.0
    if not packable:
        coeffs[0, D // 2] = [L - 1, -1.0, 0, 0]  # one decreasing row in band 0
        coeffs[-1, 0] = [0, 5.0, 0, 0]           # one steep row (steps of 5) in the last band
    want_lut, want = expect(o, coeffs, dn, L)
    steps = np.diff(want_lut.astype(np.int64), axis=2)
    assert packable == bool(((steps >= 0) & (steps <= 3)).all())
    lut_t = rc.lut_build(to_dev_f64(coeffs), L)
    dn_t = to_dev_u16(dn)
    for strip, vec, threads, chunk in ((256, 1, 256, N), (64, 2, 512, 7), (16, 1, 1024, 3),
                                       (128, 2, 256, 1)):
        if (L + 31) // 32 * strip * 10 > 128 * 1024 or D % vec:
            continue
        plan = rc.Plan(path=rc.RC_PATH_PACKED, strip=strip, vec=vec, threads=threads, unroll=8,
                       chunk_lines=chunk, xcd_remap=1, nontemporal=0)
        out = Guarded((B, N, D))
        rc.correct(dn_t, lut_t, out=out.t, plan=plan)
        torch.cuda.synchronize()
        out.check_pads()
        assert np.array_equal(out.host(), want), f"plan {plan}"


DENSE_SHAPES = [(2, 301, 1000, 4096), (1, 77, 333, 1000), (3, 40, 64, 64), (1, 65, 130, 8192),
                (2, 31, 520, 2048), (1, 50, 40, 100), (2, 20, 24, 2)]


@pytest.mark.parametrize("shape", DENSE_SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("rows", ["calibration", "clamped", "unpackable", "steep"])
def test_dense_path(o, shape, rows):
    """Dense LDS tiles (1 bit per step, per-block slope 0 or 1, saturated
    runs extrapolated): exact for calibration-like rows, for rows that
    saturate at both ends inside a block, and through the global-gather
    fallback for rows that do not fit (decreasing, steps of 5, slopes
    growing past 2, and every row with gains of 2 to 3: steps of 2 and 3)."""
    B, N, D, L = shape
    coeffs, dn = pins.tiny_case(L + N + D, B, N, D, L)
    rng = np.random.default_rng(L + D + N)
    coeffs[..., 0] = rng.normal(0, L / 128, size=(B, D))
    coeffs[..., 1] = rng.uniform(0.9, 1.1, size=(B, D))
    coeffs[..., 2] = rng.normal(0, 0.05 / L, size=(B, D))
    coeffs[..., 3] = 0.0
    if rows == "clamped":
        # Offsets of +-L/4 and gains up to 1.6: long runs of 0 and L-1, the
        # transitions anywhere inside a 64-level block.
        coeffs[..., 0] = rng.uniform(-L / 4, L / 4, size=(B, D))
        coeffs[..., 1] = rng.uniform(0.6, 1.6, size=(B, D))
    if rows == "steep":
        coeffs[..., 1] = rng.uniform(2.0, 3.0, size=(B, D))
        coeffs[..., 2] = 0.0
    if rows == "unpackable":
        coeffs[0, D // 2] = [L - 1, -1.0, 0, 0]      # decreasing
        coeffs[-1, 0] = [0, 5.0, 0, 0]               # steps of 5
        coeffs[-1, D - 1] = [L / 3, 1.0, 3.0 / L, 0]  # slope growing from 1 to 7
    want_lut, want = expect(o, coeffs, dn, L)
    lut_t = rc.lut_build(to_dev_f64(coeffs), L)
    dn_t = to_dev_u16(dn)
    n = 0
    for strip, vec, threads, unroll, chunk, nt, strips in (
            (256, 8, 256, 4, N, 0, 0), (64, 2, 512, 8, 7, 2, 0), (16, 1, 512, 16, 3, 4, 0),
            (128, 4, 256, 4, 1, 0, 0), (256, 4, 256, 8, N, 0, 3), (128, 2, 512, 8, 11, 5, 2),
            (256, 1, 256, 8, N, 0, 0)):
        if D % vec or -(-L // 64) * strip * 10 > 160 * 1024 or strip // vec > threads:
            continue
        if strips and (strips > D // vec or vec * -(-(D // vec) // strips) > strip):
            continue
        plan = rc.Plan(path=rc.RC_PATH_DENSE, strip=strip, vec=vec, threads=threads,
                       unroll=unroll, chunk_lines=chunk, xcd_remap=1, nontemporal=nt,
                       strips=strips)
        out = Guarded((B, N, D))
        rc.correct(dn_t, lut_t, out=out.t, plan=plan)
        torch.cuda.synchronize()
        out.check_pads()
        assert np.array_equal(out.host(), want), f"plan {plan}"
        n += 1
    assert n >= 2


@pytest.mark.parametrize("path", [rc.RC_PATH_LDS, rc.RC_PATH_PACKED, rc.RC_PATH_DENSE])
def test_staging_waves_tile_count_boundary(o, path):
    """Tiles alone on their CU launch more threads than stream (extra waves
    only stage the strip); one tile more and the workgroup is the plan's.
    Both sides of that boundary, and one tile below it, match the oracle."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    B, N, D, L = 1, 37, (cus + 1) * 4, 1024
    coeffs, dn = pins.tiny_case(cus + path, B, N, D, L)
    rng = np.random.default_rng(cus + 7 * path)
    coeffs[..., 0] = rng.normal(0, L / 128, size=(B, D))
    coeffs[..., 1] = rng.uniform(0.9, 1.1, size=(B, D))
    coeffs[..., 2] = rng.normal(0, 0.05 / L, size=(B, D))
    coeffs[..., 3] = 0.0
    coeffs[0, 5] = [L - 1, -1.0, 0, 0]  # one row no compact form holds
    _, want = expect(o, coeffs, dn, L)
    lut_t = rc.lut_build(to_dev_f64(coeffs), L)
    dn_t = to_dev_u16(dn)
    for strips in (cus - 1, cus, cus + 1):
        plan = rc.Plan(path=path, strip=16, vec=4, threads=256, unroll=4, chunk_lines=N,
                       xcd_remap=1, nontemporal=0, strips=strips)
        out = Guarded((B, N, D))
        rc.correct(dn_t, lut_t, out=out.t, plan=plan)
        torch.cuda.synchronize()
        out.check_pads()
        assert np.array_equal(out.host(), want), f"strips {strips}, plan {plan}"


def test_dense_rejects_long_rows():
    dn = torch.zeros((1, 4, 64), dtype=torch.int16, device=dev())
    lut = torch.zeros((1, 64, 8200), dtype=torch.int16, device=dev())
    plan = rc.Plan(path=rc.RC_PATH_DENSE, strip=16, vec=2, threads=256, unroll=4, chunk_lines=4,
                   xcd_remap=1, nontemporal=0)
    with pytest.raises(rc.RcError) as e:
        rc.correct(dn, lut, plan=plan)
    assert e.value.status == rc.RC_EINVAL


def test_dense_rejects_1024_threads():
    """The dense kernels are built for at most 512 threads per workgroup."""
    dn = torch.zeros((1, 4, 64), dtype=torch.int16, device=dev())
    lut = torch.zeros((1, 64, 4096), dtype=torch.int16, device=dev())
    plan = rc.Plan(path=rc.RC_PATH_DENSE, strip=16, vec=2, threads=1024, unroll=4,
                   chunk_lines=4, xcd_remap=1, nontemporal=0)
    with pytest.raises(rc.RcError) as e:
        rc.correct(dn, lut, plan=plan)
    assert e.value.status == rc.RC_EINVAL


def test_tuner_roundtrip(tmp_path):
    """rc_tune picks a plan that reproduces the oracle, stores it in the cache
    under the shape class, and the cache survives a save/load round trip."""
    B, N, D, L = 2, 300, 1000, 1024
    coeffs, dn = pins.tiny_case(1, B, N, D, L)
    o = oracle.get()
    _, want = expect(o, coeffs, dn, L)
    lut_t = rc.lut_build(to_dev_f64(coeffs), L)
    dn_t = to_dev_u16(dn)
    out_t = torch.empty_like(dn_t)
    rc.rc_tune_clear()
    plan, us = rc.rc_tune(dn_t, lut_t, N, D, B, L, out_t, effort=0)
    assert us > 0
    got, tuned = rc.rc_plan_for(N, D, B, L, dn_t, out_t)
    assert tuned and got.as_dict() == plan.as_dict()
    path = str(tmp_path / "cache.json")
    assert rc.rc_tune_save(path) == 1
    rc.rc_tune_clear()
    assert not rc.rc_plan_for(N, D, B, L, dn_t, out_t)[1]
    assert rc.rc_tune_load(path) == 1
    assert rc.rc_plan_for(N, D, B, L, dn_t, out_t)[1]
    out = rc.correct(dn_t, lut_t)
    torch.cuda.synchronize()
    assert np.array_equal(to_host_u16(out), want)
    rc.rc_tune_load(None)  # back to the packaged cache


def test_plan_rejected_when_lds_too_small():
    dn = torch.zeros((1, 4, 64), dtype=torch.int16, device=dev())
    lut = torch.zeros((1, 64, 4096), dtype=torch.int16, device=dev())
    bad = rc.Plan(path=rc.RC_PATH_LDS, strip=64, vec=2, threads=256, unroll=4, chunk_lines=4,
                  xcd_remap=0, nontemporal=0)  # 64 x 4096 x 2 B = 512 KiB of LDS
    with pytest.raises(rc.RcError) as e:
        rc.correct(dn, lut, plan=bad)
    assert e.value.status == rc.RC_EINVAL


@pytest.mark.parametrize("field,value", [("nontemporal", 6), ("nontemporal", -1), ("xcd_remap", 2),
                                         ("lane_map", 2), ("lane_map", -1)])
def test_plan_rejects_bad_policy(field, value):
    dn = torch.zeros((1, 4, 64), dtype=torch.int16, device=dev())
    lut = torch.zeros((1, 64, 1024), dtype=torch.int16, device=dev())
    d = dict(path=rc.RC_PATH_PACKED, strip=64, vec=2, threads=256, unroll=4, chunk_lines=4,
             xcd_remap=1, nontemporal=0)
    d[field] = value
    with pytest.raises(rc.RcError) as e:
        rc.correct(dn, lut, plan=rc.Plan(**d))
    assert e.value.status == rc.RC_EINVAL


def test_in_place(o):
    B, N, D, L = 2, 129, 200, 1024
    coeffs, dn = pins.tiny_case(5, B, N, D, L)
    _, want = expect(o, coeffs, dn, L)
    _, out = run_case(o, coeffs, dn, L, in_place=True)
    assert np.array_equal(out, want)


@pytest.mark.parametrize("offs", [(1, 0), (0, 1), (1, 1), (2, 3)])
def test_misaligned_images(o, offs):
    B, N, D, L = 2, 77, 96, 1024
    coeffs, dn = pins.tiny_case(9, B, N, D, L)
    _, want = expect(o, coeffs, dn, L)
    _, out = run_case(o, coeffs, dn, L, dn_offset=offs[0], out_offset=offs[1])
    assert np.array_equal(out, want)


def test_saturating_dn(o):
    B, N, D, L = 1, 16, 64, 1024
    coeffs, _ = pins.tiny_case(3, B, N, D, L)
    dn = np.full((B, N, D), 65535, dtype=np.uint16)
    dn[0, ::2] = 1024
    dn[0, 1::4] = 1023
    _, want = expect(o, coeffs, dn, L)
    _, out = run_case(o, coeffs, dn, L)
    assert np.array_equal(out, want)


@pytest.mark.parametrize("w", [0, 1, 2])
def test_workload_full_size(o, w):
    """Full-size single-scene workloads with the plan rc_correct picks (the one
    the benchmark times): every output pixel compared with the oracle."""
    s = gen.workload(w)
    print(f"workload {w}: {s.name}", flush=True)
    coeffs = s.coeffs()
    dn = s.dn()
    want_lut = o.lut_build(coeffs, s.levels)
    want = o.correct(dn, want_lut)
    c_t = to_dev_f64(coeffs)
    dn_t = to_dev_u16(dn)
    lut_t = rc.lut_build(c_t, s.levels)
    out_t = torch.empty_like(dn_t)
    rc.correct(dn_t, lut_t, out=out_t)
    torch.cuda.synchronize()
    assert np.array_equal(to_host_u16(lut_t), want_lut)
    out = to_host_u16(out_t)
    bad = np.count_nonzero(out != want)
    assert bad == 0, f"{bad} pixels differ"
