"""Seeded input generators: published SplitMix64 vector, counter-based
reproducibility and the workload recipes' ranges. CPU only."""
import numpy as np

import gen


def test_splitmix64_reference_vector():
    # First outputs of SplitMix64 seeded with 1234567 (Vigna's reference
    # implementation, splitmix64.c).
    assert gen.splitmix64_sequence(1234567, 3) == [
        6457827717110365317, 3203168211198807973, 9817491932198370423]


def test_subrange_and_threads_reproducible():
    s = gen.workload(1)
    full = gen.dn(s.seed, s.cfg, 0, s.dn_kind, 2, 40, 33, threads=1)
    part = gen.dn(s.seed, s.cfg, 0, s.dn_kind, 2, 40, 33, n0=17, nlines=9, threads=3)
    assert np.array_equal(full[:, 17:26], part)
    again = gen.dn(s.seed, s.cfg, 0, s.dn_kind, 2, 40, 33, threads=4)
    assert np.array_equal(full, again)


def test_workload_ranges():
    s0, s1, s2 = gen.workload(0), gen.workload(1), gen.workload(2)
    d0 = s0.dn()
    assert d0.shape == (1, 1024, 1024) and d0.max() <= 1023
    assert abs(d0.mean() - 511.5) < 2
    d1 = s1.dn(nlines=64)
    assert d1.max() == 1023 and d1.min() == 0
    sat = (d1 == 1023).mean()
    assert 0.009 < sat < 0.012
    body = d1[(d1 > 0) & (d1 < 1023)].astype(np.float64)
    assert abs(body.mean() - 400) < 3 and abs(body.std() - 150) < 4
    d2 = s2.dn(nlines=64)
    assert d2.max() <= 4095 and d2.max() >= 4090
    c0 = s0.coeffs()
    assert c0.shape == (1, 1024, 4) and (c0[..., 3] == 0).all()
    assert ((c0[..., 1] >= 0.9) & (c0[..., 1] < 1.1)).all()
    assert abs(c0[..., 0].std() - 8) < 1
    c2 = s2.coeffs()
    assert abs(c2[..., 0].std() - 32) < 2 and (c2[..., 3] != 0).all()


def test_batch_and_serve_shapes():
    reqs = gen.batch_requests(256)
    assert len(reqs) == 256
    for r in reqs:
        assert 512 <= r.lines <= 8192 and 512 <= r.detectors <= 8192
        assert 1 <= r.bands <= 4 and r.levels in (1024, 4096)
    assert {r.levels for r in reqs} == {1024, 4096}
    trace = gen.serve_trace(200, qps=150.0)
    t = np.array([a for a, _ in trace])
    assert (np.diff(t) > 0).all()
    assert abs(len(t) / t[-1] - 150) < 40
    for _, j in trace:
        assert 1024 <= j.detectors <= 12000 and 1 <= j.bands <= 4


def test_calib_is_deterministic_and_shaped():
    x1, y1 = gen.calib(gen.BASE_SEED, 5, 0, 2, 6, 100, 1024)
    x2, y2 = gen.calib(gen.BASE_SEED, 5, 0, 2, 6, 100, 1024)
    assert x1.shape == (2, 6, 100) and y1.shape == (2, 6)
    assert np.array_equal(x1, x2) and np.array_equal(y1, y2)
    # Reference levels evenly inside (0, L-1); responses rise with the level.
    assert np.allclose(y1[0], np.arange(1, 7) / 7 * 1023)
    assert (np.diff(x1, axis=1) > 0).mean() > 0.99
    # A detector's data do not depend on how many detectors are drawn.
    x3, _ = gen.calib(gen.BASE_SEED, 5, 0, 2, 6, 40, 1024)
    assert np.array_equal(x3, x1[:, :, :40])


def test_bayer_is_deterministic():
    a = gen.bayer(gen.BASE_SEED, 7, 0, 2, 64, 96)
    b = gen.bayer(gen.BASE_SEED, 7, 0, 2, 64, 96, threads=1)
    assert a.shape == (2, 64, 96) and a.dtype == np.uint16
    assert np.array_equal(a, b)
    assert not np.array_equal(a[0], a[1])  # phases drawn per image
