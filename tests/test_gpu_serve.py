"""Serving runtime: every job's result is the same alone and in a concurrent
mix (tolerance 0, the work is per-pixel with no reduction), equal to the
oracle; admission under a small arena, refusals, polling and shutdown."""
import threading
import time

import numpy as np
import pytest

import gen
import oracle
import paper_1505_05655_amd as rc
import pins

pytestmark = pytest.mark.gpu

# (bands, lines, detectors, levels, coefficient style)
SPECS = [
    (2, 700, 1000, 1024, "quad"),
    (1, 1300, 513, 1024, "quad"),    # odd detector count
    (3, 400, 600, 4096, "cubic"),
    (1, 20, 77, 65536, "tiny"),      # L2 path: LUT built by the build kernel
    (2, 0, 50, 1024, "quad"),        # LUT only
    (2, 90, 300, 3, "tiny"),         # raw LDS tiles
    (1, 2500, 256, 1024, "tiny"),    # rows that cannot be packed
    (4, 64, 1030, 1024, "quad"),
]


def make(i, spec):
    B, N, D, L, style = spec
    if style == "tiny":
        coeffs, dn = pins.tiny_case(900 + i, B, max(N, 1), D, L)
        dn = np.ascontiguousarray(dn[:, :N])
    else:
        kind = gen.COEF_QUADRATIC if style == "quad" else gen.COEF_CUBIC
        dkind = gen.DN_GAUSS_SAT10 if style == "quad" else gen.DN_SCENE12
        coeffs = gen.coeffs(gen.BASE_SEED, 11, i, kind, B, D)
        dn = gen.dn(gen.BASE_SEED, 11, i, dkind, B, N, D) if N else np.zeros((B, 0, D), np.uint16)
    o = oracle.get()
    want_lut = o.lut_build(coeffs, L)
    want = o.correct(dn, want_lut)
    c_p = rc.pinned_empty(coeffs.shape, np.float64)
    c_p[...] = coeffs
    dn_p = rc.pinned_empty(dn.shape, np.uint16)
    dn_p[...] = dn
    return c_p, dn_p, want_lut, want


@pytest.fixture(scope="module")
def jobs():
    return [make(i, s) for i, s in enumerate(SPECS)]


def job_bytes(spec):
    B, N, D, L, _ = spec
    r = lambda x: (x + 255) // 256 * 256
    return r(32 * B * D) + r(2 * B * D * L) + 2 * r(2 * B * N * D)


def run(srv, jobs, idx, pageable=()):
    """Pinned outputs are written by the kernel directly; outputs in `pageable`
    (ordinary numpy memory) go through the device-to-host copy path."""
    outs = {}
    for i in idx:
        c, d, wl, w = jobs[i]
        img = np.empty(w.shape, np.uint16) if i in pageable else rc.pinned_empty(w.shape, np.uint16)
        outs[i] = (img, rc.pinned_empty(wl.shape, np.uint16))
    ids = {i: srv.submit(jobs[i][0], jobs[i][1], outs[i][0], SPECS[i][3], lut=outs[i][1])
           for i in idx}
    return outs, ids


def test_alone_equals_mix_equals_oracle(jobs):
    # Alone: one job at a time through a server with small pieces.
    srv = rc.Server(piece_pixels=1 << 16)
    alone = {}
    for i in range(len(SPECS)):
        outs, ids = run(srv, jobs, [i])
        st = srv.wait(ids[i])
        assert st["status"] == rc.RC_OK, SPECS[i]
        assert np.array_equal(outs[i][1], jobs[i][2]), f"alone LUT {SPECS[i]}"
        assert np.array_equal(outs[i][0], jobs[i][3]), f"alone image {SPECS[i]}"
        alone[i] = outs[i]
    srv.close()
    # Mix: everything at once into an arena that holds only a few jobs, with
    # small pieces and quanta so that tiles of different jobs share launches.
    arena = 3 * max(job_bytes(s) for s in SPECS)
    srv = rc.Server(arena_bytes=arena, max_jobs=4, piece_pixels=1 << 16, max_quantum_tiles=64)
    outs, ids = run(srv, jobs, range(len(SPECS)), pageable={i for i in range(len(SPECS)) if i % 2})
    for i in range(len(SPECS)):
        st = srv.wait(ids[i])
        assert st["status"] == rc.RC_OK, SPECS[i]
        assert st["done_s"] >= st["admit_s"] >= st["submit_s"]
        assert np.array_equal(outs[i][0], alone[i][0]), f"mix != alone {SPECS[i]}"
        assert np.array_equal(outs[i][1], alone[i][1]), f"mix LUT != alone {SPECS[i]}"
    info = srv.info()
    assert info["completed"] == len(SPECS) and info["quanta"] > 1 and info["arena_used"] == 0
    # Pinned outputs of jobs with pixels are written directly; pageable ones are copied.
    assert info["direct_out"] == sum(1 for i, sp in enumerate(SPECS) if i % 2 == 0 and sp[1] > 0)
    srv.close()


def test_refusals(jobs):
    srv = rc.Server(arena_bytes=1 << 20)
    c, d, wl, w = jobs[0]
    out = np.empty_like(w)
    with pytest.raises(rc.RcError) as e:
        srv.submit(c, d, out, 1024)  # needs far more than 1 MiB
    assert e.value.status == rc.RC_ENOMEM
    with pytest.raises(rc.RcError) as e:
        srv.submit(c, d, out, 1)     # levels < 2
    assert e.value.status == rc.RC_EINVAL
    srv.close()


def test_poll(jobs):
    srv = rc.Server()
    c, d, wl, w = jobs[2]
    out = rc.pinned_empty(w.shape, np.uint16)
    jid = srv.submit(c, d, out, SPECS[2][3])
    t0 = time.time()
    st = None
    while st is None and time.time() - t0 < 60:
        st = srv.poll(jid)
        time.sleep(0.001)
    assert st is not None and st["status"] == rc.RC_OK
    assert np.array_equal(out, w)
    srv.close()


def test_shutdown_refuses_pending():
    """Destroy with jobs queued: admitted jobs finish correctly, jobs still
    waiting for admission complete with RC_ECLOSED."""
    B, N, D, L = 1, 4000, 4000, 1024
    coeffs = gen.coeffs(gen.BASE_SEED, 12, 0, gen.COEF_QUADRATIC, B, D)
    dn = gen.dn(gen.BASE_SEED, 12, 0, gen.DN_GAUSS_SAT10, B, N, D)
    o = oracle.get()
    want = o.correct(dn, o.lut_build(coeffs, L))
    c_p = rc.pinned_empty(coeffs.shape, np.float64)
    c_p[...] = coeffs
    d_p = rc.pinned_empty(dn.shape, np.uint16)
    d_p[...] = dn
    nj = 8
    srv = rc.Server(arena_bytes=job_bytes((B, N, D, L, "")) + 4096, max_jobs=1,
                    piece_pixels=1 << 20)
    outs = [rc.pinned_empty(dn.shape, np.uint16) for _ in range(nj)]
    ids = [srv.submit(c_p, d_p, o_, L) for o_ in outs]
    results = {}

    def waiter(k):
        results[k] = srv.wait(ids[k])

    threads = [threading.Thread(target=waiter, args=(k,)) for k in range(nj)]
    for t in threads:
        t.start()
    t0 = time.time()
    # Close only once every waiter is blocked inside rc_server_wait (or done).
    while srv.info()["waiters"] + len(results) < nj and time.time() - t0 < 30:
        time.sleep(0.0002)
    srv.close()
    for t in threads:
        t.join(timeout=60)
    statuses = [results[k]["status"] for k in range(nj)]
    assert statuses[0] == rc.RC_OK
    assert rc.RC_ECLOSED in statuses
    for k in range(nj):
        assert statuses[k] in (rc.RC_OK, rc.RC_ECLOSED)
        if statuses[k] == rc.RC_OK:
            assert np.array_equal(outs[k], want)
