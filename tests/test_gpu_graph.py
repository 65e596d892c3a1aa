"""The plain entry points allocate nothing and never synchronise, so they can
be captured into a HIP graph. Capture fit -> LUT build -> correction and both
demosaicing calls once, then replay the graph several times with new inputs
written eagerly between replays; every replay must equal the oracle."""
import numpy as np
import pytest
import torch

import gen
import oracle
import paper_1505_05655_amd as rc

pytestmark = pytest.mark.gpu


def test_graph_replays_match_oracle():
    dev = torch.device("cuda:0")
    o = oracle.get()
    B, n, D, N, L, m = 2, 6, 520, 301, 1024, 2
    H, W = 66, 260
    x_s = torch.empty((B, n, D), dtype=torch.float64, device=dev)
    y_s = torch.empty((B, n), dtype=torch.float64, device=dev)
    dn_s = torch.empty((B, N, D), dtype=torch.int16, device=dev)
    raw_s = torch.empty((1, H, W), dtype=torch.int16, device=dev)
    coeffs = torch.empty((B, D, 4), dtype=torch.float64, device=dev)
    lut = torch.empty((B, D, L), dtype=torch.int16, device=dev)
    out = torch.empty_like(dn_s)
    rgb = torch.empty((1, 3, H, W), dtype=torch.int16, device=dev)
    rgb_g = torch.empty((1, 3, H, W), dtype=torch.int16, device=dev)

    def inputs(k):
        x, y = gen.calib(gen.BASE_SEED, 50, k, B, n, D, L)
        dn = gen.dn(gen.BASE_SEED, 50, k, gen.DN_GAUSS_SAT10, B, N, D)
        raw = gen.bayer(gen.BASE_SEED, 50, k, 1, H, W)
        return x, y, dn, raw

    def load(k):
        x, y, dn, raw = inputs(k)
        x_s.copy_(torch.from_numpy(x))
        y_s.copy_(torch.from_numpy(y))
        dn_s.copy_(torch.from_numpy(dn.view(np.int16)))
        raw_s.copy_(torch.from_numpy(raw.view(np.int16)))
        out.fill_(-1)
        rgb.fill_(-1)
        rgb_g.fill_(-1)
        torch.cuda.synchronize()
        return x, y, dn, raw

    s = torch.cuda.Stream(device=dev)

    def work():
        rc.rc_fit(x_s, y_s, B, n, D, m, coeffs, s)
        rc.rc_lut_build(coeffs, B, D, L, lut, s)
        rc.rc_correct(dn_s, lut, N, D, B, L, out, s)
        rc.rc_demosaic(raw_s, 1, H, W, rgb, s)
        rc.rc_demosaic_gradient(raw_s, 1, H, W, rgb_g, s)

    load(0)
    work()  # first calls set the device up outside the capture
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        work()
    for k in range(1, 4):
        x, y, dn, raw = load(k)
        g.replay()
        torch.cuda.synchronize()
        want_c = o.fit(x, y, m)
        want = o.correct(dn, o.lut_build(want_c, L))
        assert np.array_equal(coeffs.cpu().numpy().view(np.uint64), want_c.view(np.uint64)), k
        assert np.array_equal(out.cpu().numpy().view(np.uint16), want), k
        assert np.array_equal(rgb.cpu().numpy().view(np.uint16), o.demosaic(raw)), k
        assert np.array_equal(rgb_g.cpu().numpy().view(np.uint16), o.demosaic_gradient(raw)), k


def test_graph_build_ws_pair_replays_match_oracle():
    """rc_lut_build_ws + rc_correct_pre (long LUT rows, the encoding passed
    through the workspace) captured once and replayed with new coefficients
    and images written eagerly between replays."""
    dev = torch.device("cuda:0")
    o = oracle.get()
    B, N, D, L = 2, 97, 300, 4096
    need = rc.rc_correct_ws_bytes(D, B, L)
    assert need > 0
    c_s = torch.empty((B, D, 4), dtype=torch.float64, device=dev)
    dn_s = torch.empty((B, N, D), dtype=torch.int16, device=dev)
    lut = torch.empty((B, D, L), dtype=torch.int16, device=dev)
    out = torch.empty_like(dn_s)
    ws = torch.empty((need // 2 + 128,), dtype=torch.int16, device=dev)

    def load(k):
        c = gen.coeffs(gen.BASE_SEED, 51, k, gen.COEF_CUBIC, B, D)
        dn = gen.dn(gen.BASE_SEED, 51, k, gen.DN_SCENE12, B, N, D)
        c_s.copy_(torch.from_numpy(c))
        dn_s.copy_(torch.from_numpy(dn.view(np.int16)))
        out.fill_(-1)
        torch.cuda.synchronize()
        return c, dn

    s = torch.cuda.Stream(device=dev)

    def work():
        rc.rc_lut_build_ws(c_s, B, D, L, lut, ws, need, s)
        rc.rc_correct_pre(dn_s, lut, N, D, B, L, out, ws, need, None, s)

    load(0)
    work()
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        work()
    for k in range(1, 4):
        c, dn = load(k)
        g.replay()
        torch.cuda.synchronize()
        want_lut = o.lut_build(c, L)
        assert np.array_equal(lut.cpu().numpy().view(np.uint16), want_lut), k
        assert np.array_equal(out.cpu().numpy().view(np.uint16), o.correct(dn, want_lut)), k
