"""rc_correct_ws (the LUT encoded once into a workspace, then the dense
correction) against the oracle, bit-exact: long and short LUT rows,
calibration-like, saturating and unpackable rows, forced plans, and the
workspace checks."""
import numpy as np
import pytest
import torch

import oracle
import paper_1505_05655_amd as rc
import pins
from gpu_util import Guarded, dev, to_dev_f64, to_dev_u16

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def o():
    return oracle.get()


def case(shape, rows, seed):
    B, N, D, L = shape
    coeffs, dn = pins.tiny_case(seed, B, N, D, L)
    rng = np.random.default_rng(seed)
    coeffs[..., 0] = rng.normal(0, L / 128, size=(B, D))
    coeffs[..., 1] = rng.uniform(0.9, 1.1, size=(B, D))
    coeffs[..., 2] = rng.normal(0, 0.05 / L, size=(B, D))
    coeffs[..., 3] = rng.normal(0, 0.01 / L ** 2, size=(B, D))
    if rows == "clamped":
        coeffs[..., 0] = rng.uniform(-L / 4, L / 4, size=(B, D))
        coeffs[..., 1] = rng.uniform(0.6, 1.6, size=(B, D))
    if rows == "unpackable":
        coeffs[0, D // 2] = [L - 1, -1.0, 0, 0]
        coeffs[-1, D - 1] = [L / 3, 1.0, 3.0 / L, 0]
    return coeffs, dn


# 2112 levels: 33 whole blocks, so the last group of 8 blocks a workgroup of
# the encoder stages holds one block; 3000: a partial last block.
SHAPES = [(3, 401, 1000, 4096), (1, 300, 520, 2048), (2, 77, 96, 8192), (1, 129, 333, 3000),
          (2, 64, 200, 1024), (1, 5, 7, 4096), (1, 50, 45, 2112)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("rows", ["calibration", "clamped", "unpackable"])
def test_ws_matches_oracle(o, shape, rows):
    B, N, D, L = shape
    coeffs, dn = case(shape, rows, B * 7 + N + D + L)
    lut = o.lut_build(coeffs, L)
    want = o.correct(dn, lut)
    lut_t = rc.lut_build(to_dev_f64(coeffs), L)
    dn_t = to_dev_u16(dn)
    need = rc.rc_correct_ws_bytes(D, B, L)
    assert need == (0 if L < 2048 else
                    ((B * -(-L // 64) * D * 8 + 255) // 256 * 256 +
                     (B * -(-L // 64) * D * 2 + 255) // 256 * 256))
    ws = torch.full((max(need, 256) // 2 + 128,), 0x3C3C, dtype=torch.int16, device=dev())
    plans = [None]
    if L >= 2048:
        for strip, vec, threads, unroll, chunk, strips in ((256, 4, 512, 8, N, 0),
                                                           (128, 8, 256, 4, 17, 0),
                                                           (64, 2, 512, 16, 5, 0),
                                                           (256, 4, 256, 8, 33, 3)):
            if D % vec or -(-L // 64) * strip * 10 > 160 * 1024:
                continue
            if strips and (strips > D // vec or vec * -(-(D // vec) // strips) > strip):
                continue
            plans.append(rc.Plan(path=rc.RC_PATH_DENSE, strip=strip, vec=vec, threads=threads,
                                 unroll=unroll, chunk_lines=chunk, xcd_remap=1, nontemporal=0,
                                 strips=strips))
    for plan in plans:
        out = Guarded((B, N, D))
        rc.rc_correct_ws(dn_t, lut_t, N, D, B, L, out.t, ws, need, plan)
        torch.cuda.synchronize()
        out.check_pads()
        assert np.array_equal(out.host(), want), f"plan {plan}"


WS_SHAPES = [s for s in SHAPES if 2048 <= s[3] <= 8192]


@pytest.mark.parametrize("shape", WS_SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("rows", ["calibration", "clamped", "unpackable"])
def test_build_ws_then_pre(o, shape, rows):
    """rc_lut_build_ws writes the oracle's LUT and the encoding rc_correct_ws
    makes of it (headers equal everywhere, planes wherever the header marks
    an encoded block); rc_correct_pre then gives the oracle's image, with the
    library's plan and with forced dense plans."""
    B, N, D, L = shape
    coeffs, dn = case(shape, rows, B * 7 + N + D + L)
    want_lut = o.lut_build(coeffs, L)
    want = o.correct(dn, want_lut)
    need = rc.rc_correct_ws_bytes(D, B, L)
    n = B * -(-L // 64) * D
    hoff = (n * 8 + 255) // 256 * 256
    dn_t = to_dev_u16(dn)
    lut_g = Guarded((B, D, L))
    ws = torch.full((need // 2 + 128,), 0x3C3C, dtype=torch.int16, device=dev())
    rc.rc_lut_build_ws(to_dev_f64(coeffs), B, D, L, lut_g.t, ws, need)
    torch.cuda.synchronize()
    lut_g.check_pads()
    assert np.array_equal(lut_g.host(), want_lut)
    ws_ref = torch.full_like(ws, 0x3C3C)
    tmp = torch.empty_like(dn_t)
    rc.rc_correct_ws(dn_t, lut_g.t, N, D, B, L, tmp, ws_ref, need)
    torch.cuda.synchronize()
    got_b = ws.cpu().numpy().view(np.uint8)
    ref_b = ws_ref.cpu().numpy().view(np.uint8)
    heads = got_b[hoff:hoff + 2 * n].view(np.int16)
    assert np.array_equal(heads, ref_b[hoff:hoff + 2 * n].view(np.int16))
    enc = heads != -32768
    assert np.array_equal(got_b[:8 * n].view(np.uint64)[enc], ref_b[:8 * n].view(np.uint64)[enc])
    if rows == "unpackable":
        assert not enc.all()
    plans = [None]
    for strip, vec, threads, unroll, chunk, strips in ((256, 4, 512, 8, N, 0),
                                                       (128, 8, 256, 4, 17, 0),
                                                       (256, 4, 256, 8, 33, 3)):
        if D % vec or -(-L // 64) * strip * 10 > 160 * 1024:
            continue
        if strips and (strips > D // vec or vec * -(-(D // vec) // strips) > strip):
            continue
        plans.append(rc.Plan(path=rc.RC_PATH_DENSE, strip=strip, vec=vec, threads=threads,
                             unroll=unroll, chunk_lines=chunk, xcd_remap=1, nontemporal=0,
                             strips=strips))
    for plan in plans:
        out = Guarded((B, N, D))
        rc.rc_correct_pre(dn_t, lut_g.t, N, D, B, L, out.t, ws, need, plan)
        torch.cuda.synchronize()
        out.check_pads()
        assert np.array_equal(out.host(), want), f"plan {plan}"


def test_ws_rejects():
    B, N, D, L = 1, 8, 64, 4096
    dn = torch.zeros((B, N, D), dtype=torch.int16, device=dev())
    lut = torch.zeros((B, D, L), dtype=torch.int16, device=dev())
    out = torch.empty_like(dn)
    need = rc.rc_correct_ws_bytes(D, B, L)
    ws = torch.empty(need // 2 + 1024, dtype=torch.int16, device=dev())
    for args in ((ws, need - 256), (None, need), (ws[1:], need)):
        with pytest.raises(rc.RcError) as e:
            rc.rc_correct_ws(dn, lut, N, D, B, L, out, args[0], args[1])
        assert e.value.status == rc.RC_EINVAL
    # Overlapping the image, and a plan that is not dense.
    big = torch.zeros(need // 2 + B * N * D + 1024, dtype=torch.int16, device=dev())
    with pytest.raises(rc.RcError):
        rc.rc_correct_ws(big[:B * N * D], lut, N, D, B, L, out, big, need)
    bad = rc.Plan(path=rc.RC_PATH_PACKED, strip=64, vec=2, threads=256, unroll=4, chunk_lines=4,
                  xcd_remap=1, nontemporal=0)
    with pytest.raises(rc.RcError):
        rc.rc_correct_ws(dn, lut, N, D, B, L, out, ws, need, bad)
