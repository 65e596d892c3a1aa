"""rc_correct_noalloc (the library's scratch instead of a workspace; for
callers that cannot allocate) against rc_correct_ws and the oracle, through
the C ABI: two calls in a row, the second on a smaller scene (the scratch
keeps the first call's contents), a shape that needs no scratch, and a shape
that needs more than the scratch holds."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1505_05655_amd as rc
import pins
from gpu_util import dev, to_dev_f64, to_dev_u16

pytestmark = pytest.mark.gpu


def scene(seed, B, N, D, L):
    coeffs, dn = pins.tiny_case(seed, B, N, D, L)
    rng = np.random.default_rng(seed)
    coeffs[..., 0] = rng.uniform(-L / 8, L / 8, size=(B, D))
    coeffs[..., 1] = rng.uniform(0.8, 1.3, size=(B, D))
    coeffs[..., 2] = rng.normal(0, 0.05 / L, size=(B, D))
    coeffs[..., 3] = 0.0
    return coeffs, dn


def call_noalloc(dn_t, lut_t, shape, out_t, stream):
    B, N, D, L = shape
    return rc.lib().rc_correct_noalloc(ctypes.c_void_p(dn_t.data_ptr()),
                                       ctypes.c_void_p(lut_t.data_ptr()), N, D, B, L,
                                       ctypes.c_void_p(out_t.data_ptr()),
                                       ctypes.c_void_p(stream.cuda_stream))


def test_noalloc_matches_ws_twice():
    o = oracle.get()
    stream = torch.cuda.Stream(device=dev())
    for shape in ((3, 700, 1800, 4096), (1, 90, 300, 2048)):  # the second call is smaller
        B, N, D, L = shape
        print("noalloc case", shape, flush=True)
        coeffs, dn = scene(sum(shape), B, N, D, L)
        lut_t = rc.lut_build(to_dev_f64(coeffs), L)
        dn_t = to_dev_u16(dn)
        need = rc.rc_correct_ws_bytes(D, B, L)
        assert 0 < need <= rc.NOALLOC_SCRATCH_BYTES
        ws = torch.empty(need // 2 + 128, dtype=torch.int16, device=dev())
        out_ws = torch.empty_like(dn_t)
        out_na = torch.full_like(dn_t, 0x1234)
        torch.cuda.synchronize()
        rc.rc_correct_ws(dn_t, lut_t, N, D, B, L, out_ws, ws, need, None, stream)
        st = call_noalloc(dn_t, lut_t, shape, out_na, stream)
        assert st == rc.RC_OK, rc.lib().rc_status_str(st)
        stream.synchronize()
        assert torch.equal(out_na, out_ws)
        want = o.correct(dn, o.lut_build(coeffs, L))
        assert np.array_equal(out_na.cpu().numpy().view(np.uint16), want)


def test_noalloc_without_scratch_and_too_large():
    stream = torch.cuda.Stream(device=dev())
    B, N, D, L = 2, 50, 100, 1024  # no workspace for this shape: the plain call
    coeffs, dn = scene(5, B, N, D, L)
    lut_t = rc.lut_build(to_dev_f64(coeffs), L)
    dn_t = to_dev_u16(dn)
    out_na = torch.empty_like(dn_t)
    out_pl = torch.empty_like(dn_t)
    rc.rc_correct(dn_t, lut_t, N, D, B, L, out_pl, stream)
    assert call_noalloc(dn_t, lut_t, (B, N, D, L), out_na, stream) == rc.RC_OK
    stream.synchronize()
    assert torch.equal(out_na, out_pl)
    # 4 x 128 blocks x 7000 detectors x 10 B > 32 MiB: refused before any work.
    shape = (4, 1, 7000, 8192)
    assert rc.rc_correct_ws_bytes(7000, 4, 8192) > rc.NOALLOC_SCRATCH_BYTES
    dn_big = torch.zeros((4, 1, 7000), dtype=torch.int16, device=dev())
    lut_big = torch.zeros((4, 7000, 8192), dtype=torch.int16, device=dev())
    out_big = torch.empty_like(dn_big)
    assert call_noalloc(dn_big, lut_big, shape, out_big, stream) == rc.RC_EINVAL
