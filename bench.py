"""Benchmark: LUT build + image correction on one MI355X.

One step = rc_lut_build + rc_correct over the 3-band x 50000-line x 6000-detector
scene (L = 4096, cubic coefficients; the largest single-scene workload), inputs
resident in HBM. Prints one JSON line with whole-step Gpix/s, the correction
kernel's roofline position (algorithmic bytes / HIP-event duration vs 8 TB/s),
the CPU oracle's rate on this host, and whether the GPU output is
bit-identical to the oracle's; beside it the 4 x 12000 x 12000 scene with its
own roofline, end-to-end (pinned host to pinned host) throughput, and the
batch, serving, fit and demosaicing legs.
"""
import argparse
import hashlib
import json
import os
import platform
import re
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", type=int, default=2, choices=(0, 1, 2))
    ap.add_argument("--no-scenes", action="store_true",
                    help="skip the other single-scene workload (1 or 2)")
    ap.add_argument("--no-e2e", action="store_true",
                    help="skip the end-to-end (pinned host to host) leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum CPU time spent timing the oracle")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-request batch leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-fit", action="store_true", help="skip the calibration-fit leg")
    ap.add_argument("--no-demosaic", action="store_true", help="skip the demosaicing legs")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the graph-replayed 1 x 1024 x 1024 scene")
    ap.add_argument("--serve-jobs", type=int, default=2000)
    ap.add_argument("--serve-qps", type=float, default=150.0)
    ap.add_argument("--batch-requests", type=int, default=256)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 4 device-to-device copies of MIB MiB (hardware counter "
                         "calibration: a plain copy kernel of known size) and exit")
    return ap.parse_args()


def calibrate_copy(mib):
    import torch
    n = mib * (1 << 20) // 2
    src = torch.ones(n, dtype=torch.int16, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(4):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes_each_way": n * 2, "launches": 4}))


def bench_batch(args, torch, rc, dev):
    """Workload 3: uneven requests resident in HBM. Plain path (rc_lut_build +
    rc_correct per request on one stream) against one batched graph replay."""
    import gen
    import oracle

    reqs = gen.batch_requests(args.batch_requests)
    t0 = time.time()
    jobs = []
    for r in reqs:
        c_t = torch.from_numpy(r.coeffs()).to(dev)
        d_t = torch.from_numpy(r.dn().view(np.int16)).to(dev)
        jobs.append((r, c_t, d_t,
                     torch.empty((r.bands, r.detectors, r.levels), dtype=torch.int16, device=dev),
                     torch.empty_like(d_t),
                     torch.empty((r.bands, r.detectors, r.levels), dtype=torch.int16, device=dev),
                     torch.empty_like(d_t)))
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    px = sum(r.pixels for r in reqs)
    lut_entries = sum(r.bands * r.detectors * r.levels for r in reqs)
    algo = 4 * px + 2 * lut_entries + 2 * lut_entries  # image r+w, LUT written + read
    stream = torch.cuda.Stream(device=dev)

    def plain(sync_each=False):
        for r, c_t, d_t, lut_p, out_p, _, _ in jobs:
            rc.rc_lut_build(c_t, r.bands, r.detectors, r.levels, lut_p, stream)
            rc.rc_correct(d_t, lut_p, r.lines, r.detectors, r.bands, r.levels, out_p, stream)
            if sync_each:
                stream.synchronize()

    batch_jobs = [(c_t, d_t, lut_b, out_b) for _, c_t, d_t, _, _, lut_b, out_b in jobs]
    # Tile shapes from the batch autotuner: every request class is timed on
    # the batch kernel (untimed setup; the runs write lut_b/out_b, which the
    # timed replays overwrite).
    t1 = time.time()
    classes = rc.batch_tune(batch_jobs, stream=stream)
    torch.cuda.synchronize()
    tune_s = time.time() - t1
    batch = rc.Batch(batch_jobs)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - w0) * 1e3 / reps, e0.elapsed_time(e1) / reps

    reps = 3
    plain_ms, plain_gpu_ms = timed(plain, reps)
    plain_sync_ms, _ = timed(lambda: plain(True), reps)
    batch_ms, batch_gpu_ms = timed(lambda: batch.run(stream), reps)
    same = all(torch.equal(lp, lb) and torch.equal(op, ob)
               for _, _, _, lp, op, lb, ob in jobs)
    # Oracle check on a sample: the 6 smallest requests and 2 seeded others.
    o = oracle.get()
    order = sorted(range(len(reqs)), key=lambda i: reqs[i].pixels)
    rng = np.random.default_rng(7)
    sample = order[:6] + list(rng.choice(order[6:], size=min(2, len(order) - 6), replace=False))
    oracle_ok = True
    for i in sample:
        r, c_t, d_t, _, _, lut_b, out_b = jobs[i]
        wl = o.lut_build(r.coeffs(), r.levels)
        w = o.correct(d_t.cpu().numpy().view(np.uint16), wl)
        oracle_ok &= bool(np.array_equal(lut_b.cpu().numpy().view(np.uint16), wl) and
                          np.array_equal(out_b.cpu().numpy().view(np.uint16), w))
    info = batch.info()
    batch.close()
    del jobs, batch_jobs
    torch.cuda.empty_cache()
    # Bytes the batch actually moves: the image read and written, every LUT
    # written once, and read back only for requests corrected from the global
    # LUT (fused tiles evaluate their strip in LDS).
    moved = 4 * px + 2 * lut_entries + 2 * info["lut_gather_entries"]
    with_px = sum(1 for r in reqs if r.pixels > 0)
    return {
        "workload": f"{len(reqs)} uneven requests (lines, detectors in [512, 8192], 1-4 bands, "
                    "10/12-bit)",
        "pixels": px, "lut_entries": lut_entries, "algorithmic_bytes": algo,
        "tiles": info["tiles"], "persistent_workgroups": info["slots"], "graph": bool(info["graph"]),
        "plain_ms": round(plain_ms, 3), "plain_gpu_ms": round(plain_gpu_ms, 3),
        "plain_sync_each_ms": round(plain_sync_ms, 3),
        "batched_ms": round(batch_ms, 3), "batched_gpu_ms": round(batch_gpu_ms, 3),
        "plain_gpix_s": round(px / (plain_ms * 1e-3) / 1e9, 2),
        "batched_gpix_s": round(px / (batch_ms * 1e-3) / 1e9, 2),
        "bytes_moved": moved,
        "batched_gb_s": round(moved / (batch_ms * 1e-3) / 1e9, 1),
        "batched_frac_hbm": round(moved / (batch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "batched_frac_hbm_algorithmic": round(algo / (batch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "note_frac": "batched_frac_hbm counts the bytes moved (image in and out, LUT written, "
                     "LUT read back only where not fused); the _algorithmic figure counts every "
                     "LUT written and read once",
        "tuned_requests": info["tuned"], "default_requests": with_px - info["tuned"],
        "tuned_classes": classes, "tune_s": round(tune_s, 1),
        "fused_requests": info["fused"], "lut_gather_entries": info["lut_gather_entries"],
        "speedup_vs_plain": round(plain_ms / batch_ms, 3),
        "speedup_vs_plain_sync_each": round(plain_sync_ms / batch_ms, 3),
        "bit_exact_batched_vs_plain": same,
        "bit_exact_oracle_sample": oracle_ok, "oracle_sample_requests": [int(i) for i in sample],
        "setup_s": round(gen_s, 1),
    }


def bench_fit(args, torch, rc, dev):
    """Least-squares calibration fit (the paper's case study 2, the step that
    produces the coefficients): the paper's data shape and the calibration of
    the benchmark scene, each timed on the launch stream and checked bit for
    bit against the oracle, which is timed beside it."""
    import gen
    import oracle
    o = oracle.get()
    stream = torch.cuda.Stream(device=dev)
    res = []
    for w in (0, 1):
        c = gen.fit_workload(w)
        x, y = c.data()
        xt, yt = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
        out = torch.empty((c.bands, c.detectors, 4), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        for _ in range(5):
            rc.rc_fit(xt, yt, c.bands, c.points, c.detectors, c.order, out, stream)
        reps = 200
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            rc.rc_fit(xt, yt, c.bands, c.points, c.detectors, c.order, out, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        c0, k = time.perf_counter(), 0
        while True:
            want = o.fit(x, y, c.order)
            k += 1
            if time.perf_counter() - c0 > 0.5:
                break
        cpu_us = (time.perf_counter() - c0) * 1e6 / k
        got = out.cpu().numpy()
        exact = bool(np.array_equal(got.view(np.uint64), want.view(np.uint64)))
        nbytes = x.nbytes + y.nbytes + got.nbytes
        res.append({"workload": c.name, "bands": c.bands, "points": c.points,
                    "detectors": c.detectors, "order": c.order,
                    "fit_us": round(us, 2), "detectors_per_s": round(c.bands * c.detectors / (us * 1e-6), 1),
                    "bytes": nbytes, "gb_s": round(nbytes / (us * 1e-6) / 1e9, 1),
                    "frac_hbm": round(nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 5),
                    "oracle_us": round(cpu_us, 1), "oracle_cores": 1, "bit_exact": exact})
    return res


def bench_small(args, torch, rc, dev):
    """The 1 x 1024 x 1024 scene, whose 6 MiB per step take about a microsecond
    at HBM speed, below a launch's own latency: 96 steps (rc_lut_build +
    rc_correct), each on its own buffer set (579 MB in all, more than twice
    the 256 MB MALL, so no set is still cached when its turn comes), captured
    once in a HIP graph and replayed; the eager loop of the same 96 steps is
    timed beside it. Every set is checked bit for bit against the oracle after
    a replay that follows an eager clearing of all outputs."""
    import gen
    import oracle
    s = gen.workload(0)
    sets = 96
    coeffs, dn = s.coeffs(), s.dn()
    c_t = torch.from_numpy(coeffs).to(dev)
    d_t = torch.from_numpy(dn.view(np.int16)).to(dev)
    cs = [c_t.clone() for _ in range(sets)]
    ds = [d_t.clone() for _ in range(sets)]
    luts = [torch.empty((s.bands, s.detectors, s.levels), dtype=torch.int16, device=dev)
            for _ in range(sets)]
    outs = [torch.empty_like(d_t) for _ in range(sets)]
    stream = torch.cuda.Stream(device=dev)  # default priority

    def steps():
        for i in range(sets):
            rc.rc_lut_build(cs[i], s.bands, s.detectors, s.levels, luts[i], stream)
            rc.rc_correct(ds[i], luts[i], s.lines, s.detectors, s.bands, s.levels, outs[i],
                          stream)

    torch.cuda.synchronize()
    steps()  # the first calls set the device up outside the capture
    stream.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        steps()
    for t in outs + luts:
        t.fill_(-1)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        g.replay()
    stream.synchronize()
    o = oracle.get()
    want_lut = o.lut_build(coeffs, s.levels)
    want = o.correct(dn, want_lut)
    exact = all(np.array_equal(outs[i].cpu().numpy().view(np.uint16), want) and
                np.array_equal(luts[i].cpu().numpy().view(np.uint16), want_lut)
                for i in range(sets))

    def timed(fn, reps):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        stream.synchronize()
        return [a.elapsed_time(b) for a, b in ev]

    def replay():
        with torch.cuda.stream(stream):
            g.replay()

    timed(replay, 3)
    graph_ms = timed(replay, 20)
    timed(steps, 3)
    eager_ms = timed(steps, 20)
    del g
    step_us = statistics.median(graph_ms) * 1e3 / sets
    eager_us = statistics.median(eager_ms) * 1e3 / sets
    lut_bytes = s.bands * s.detectors * s.levels * 2
    step_bytes = 4 * s.pixels + lut_bytes + lut_bytes + s.bands * s.detectors * 32
    return {"workload": s.name, "steps_per_graph": sets,
            "buffer_bytes": sets * (4 * s.pixels + lut_bytes + s.bands * s.detectors * 32),
            "graph_step_us": round(step_us, 2), "eager_step_us": round(eager_us, 2),
            "graph_gpix_s": round(s.pixels / (step_us * 1e-6) / 1e9, 1),
            "step_bytes": step_bytes,
            "graph_gb_s": round(step_bytes / (step_us * 1e-6) / 1e9, 1),
            "graph_frac_hbm": round(step_bytes / (step_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "bit_exact_all_sets": bool(exact)}


def bench_demosaic(args, torch, rc, dev, method="bilinear"):
    """Bayer demosaicing (the paper's case study 1), bilinear (rc_demosaic) or
    gradient-based (rc_demosaic_gradient): the paper's one 2048 x 2048 16-bit
    image and a batch of 16, timed on the launch stream, checked bit for bit
    against the oracle, which is timed beside it."""
    import gen
    import oracle
    o = oracle.get()
    call = rc.rc_demosaic if method == "bilinear" else rc.rc_demosaic_gradient
    ref = o.demosaic if method == "bilinear" else o.demosaic_gradient
    stream = torch.cuda.Stream(device=dev)
    res = []
    for w in (0, 1):
        name, seed, cfg, images, H, W = gen.demosaic_workload(w)
        raw = gen.bayer(seed, cfg, 0, images, H, W)
        r_t = torch.from_numpy(raw.view(np.int16)).to(dev)
        out = torch.empty((images, 3, H, W), dtype=torch.int16, device=dev)
        torch.cuda.synchronize()
        for _ in range(3):
            call(r_t, images, H, W, out, stream)
        reps = 200
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            call(r_t, images, H, W, out, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        c0 = time.perf_counter()
        want = ref(raw[:1])
        cpu_s = time.perf_counter() - c0
        got = out.cpu().numpy().view(np.uint16)
        exact = bool(np.array_equal(got[:1], want) and
                     (images == 1 or np.array_equal(got[-1:], ref(raw[-1:]))))
        px = images * H * W
        nbytes = 8 * px  # 2 B read + 6 B written per pixel
        res.append({"workload": name, "method": method, "images": images, "height": H, "width": W,
                    "demosaic_us": round(us, 2), "gpix_s": round(px / (us * 1e-6) / 1e9, 1),
                    "bytes": nbytes, "gb_s": round(nbytes / (us * 1e-6) / 1e9, 1),
                    "frac_hbm": round(nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                    "oracle_gpix_s": round(H * W / cpu_s / 1e9, 4), "oracle_cores": 1,
                    "bit_exact_checked_images": "first and last", "bit_exact": exact})
        del r_t, out
    torch.cuda.empty_cache()
    return res


def bench_e2e(args, torch, rc, dev, s):
    """End to end: the scene starts in pinned host memory and its correction
    must end there. (a) Plain path, pipelined in line chunks: H2D of a chunk
    on one copy stream, rc_correct of that chunk on the compute stream (after
    rc_lut_build from the copied coefficients), D2H on a second copy stream,
    each step waiting on the previous one's event; timed on the host from the
    first copy to the last copy's completion. (b) The same scene as one job
    of rc_server. Compared with the pinned-copy ceiling: the image copied
    H2D and D2H at once on two streams (no kernels)."""
    import oracle
    coeffs = s.coeffs()
    dn = s.dn()
    px = s.pixels
    B, N, D, L = s.bands, s.lines, s.detectors, s.levels
    h_dn = rc.pinned_empty((B, N, D), np.uint16)
    h_dn[...] = dn
    h_out = rc.pinned_empty((B, N, D), np.uint16)
    h_c = rc.pinned_empty((B, D, 4), np.float64)
    h_c[...] = coeffs
    d_dn = torch.empty((B, N, D), dtype=torch.int16, device=dev)
    d_out = torch.empty_like(d_dn)
    d_lut = torch.empty((B, D, L), dtype=torch.int16, device=dev)
    d_c = torch.empty((B, D, 4), dtype=torch.float64, device=dev)
    s_in, s_comp, s_out = (torch.cuda.Stream(device=dev) for _ in range(3))
    t_dn = torch.from_numpy(h_dn.view(np.int16))
    t_out = torch.from_numpy(h_out.view(np.int16))
    t_c = torch.from_numpy(h_c)
    chunk = max(1, (32 << 20) // D)  # lines per chunk: about 32 Mi pixels

    def pipeline():
        pieces = []
        with torch.cuda.stream(s_in):
            d_c.copy_(t_c, non_blocking=True)
            ev_c = torch.cuda.Event()
            ev_c.record(s_in)
        s_comp.wait_event(ev_c)
        rc.rc_lut_build(d_c, B, D, L, d_lut, s_comp)
        for b in range(B):
            for n0 in range(0, N, chunk):
                n1 = min(N, n0 + chunk)
                e_in, e_k = torch.cuda.Event(), torch.cuda.Event()
                with torch.cuda.stream(s_in):
                    d_dn[b, n0:n1].copy_(t_dn[b, n0:n1], non_blocking=True)
                    e_in.record(s_in)
                s_comp.wait_event(e_in)
                rc.rc_correct(d_dn[b, n0:n1], d_lut[b], n1 - n0, D, 1, L, d_out[b, n0:n1],
                              s_comp)
                e_k.record(s_comp)
                s_out.wait_event(e_k)
                with torch.cuda.stream(s_out):
                    t_out[b, n0:n1].copy_(d_out[b, n0:n1], non_blocking=True)
                pieces.append(n1 - n0)
        return len(pieces)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts)

    chunks = pipeline()
    torch.cuda.synchronize()
    plain_s = timed(pipeline)
    o = oracle.get()
    want = o.correct(dn, o.lut_build(coeffs, L))
    plain_exact = bool(np.array_equal(h_out, want))

    def copies_only():
        with torch.cuda.stream(s_in):
            d_dn.copy_(t_dn, non_blocking=True)
        with torch.cuda.stream(s_out):
            t_out.copy_(d_out, non_blocking=True)

    copy_s = timed(copies_only)
    del d_dn, d_out, d_lut, d_c
    torch.cuda.empty_cache()

    # The same scene as one rc_server job (its own pieces, arena, streams).
    h_out[...] = 0
    srv = rc.Server()
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        jid = srv.submit(h_c, h_dn, h_out, L)
        st = srv.wait(jid)
        times.append(time.perf_counter() - t0)
        if st["status"] != rc.RC_OK:
            break
    srv.close()
    server_s = statistics.median(times)
    server_exact = bool(np.array_equal(h_out, want))
    host_bytes = 4 * px + B * D * 32

    def rates(sec):
        return {"s": round(sec, 4), "gpix_s": round(px / sec / 1e9, 2),
                "gb_s": round(host_bytes / sec / 1e9, 1),
                "frac_copy_ceiling": round(copy_s / sec, 3),
                "frac_hbm": round((4 * px + 2 * B * D * L * 2) / sec / 1e9 / HBM_PEAK_GBS, 5)}

    return {"workload": s.name, "host_bytes": host_bytes,
            "pinned_copy_ceiling": {"s": round(copy_s, 4),
                                    "gb_s": round(4 * px / copy_s / 1e9, 1),
                                    "gpix_s": round(px / copy_s / 1e9, 2),
                                    "note": "image H2D and D2H at once on two streams"},
            "plain_pipelined": dict(rates(plain_s), chunks=chunks, lines_per_chunk=chunk,
                                    bit_exact=plain_exact),
            "server_one_job": dict(rates(server_s), bit_exact=server_exact),
            "note": "pinned host DN + coefficients in, pinned host out; frac_copy_ceiling = "
                    "copy-only time / end-to-end time; frac_hbm counts image I/O and the LUT "
                    "written and read once on the device"}


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    f = int(k)
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def bench_serve(args, torch, rc, dev):
    """Workload 4: Poisson arrivals of 1-600 Mpix jobs from pinned host memory,
    through rc_server (continuous batching), and through a plain server that
    runs one job at a time (copy in, rc_lut_build, rc_correct, copy out, sync)."""
    import threading

    import gen
    import oracle

    trace = gen.serve_trace(args.serve_jobs, qps=args.serve_qps)
    max_px = max(j.pixels for _, j in trace)
    t0 = time.time()
    # Host data: per bit depth one pinned pool of seeded DN, several times the
    # largest job; job i's image is the pool slice at an offset drawn from a
    # generator seeded with i (distinct data per job without holding every
    # job's image: 2000 jobs average 94 Mpix). Outputs of unverified jobs
    # share one pinned sink per depth.
    pool_px = max(4 * max_px, 1 << 30)
    pools, sinks = {}, {}
    for depth, kind in ((10, gen.DN_GAUSS_SAT10), (12, gen.DN_SCENE12)):
        pool = rc.pinned_empty((pool_px,), np.uint16)
        rows = pool_px // 4096 + 1
        tmp = gen.dn(gen.BASE_SEED + 4, 4, 1000 + depth, kind, 1, rows, 4096)
        pool[:] = tmp.reshape(-1)[:pool_px]
        del tmp
        pools[depth] = pool
        sinks[depth] = rc.pinned_empty((max_px,), np.uint16)
    offsets = [int(np.random.default_rng(gen.BASE_SEED + 4 + i).integers(0, pool_px - j.pixels + 1))
               for i, (_, j) in enumerate(trace)]
    depth_of = lambda j: 10 if j.levels == 1024 else 12
    coeffs = []
    for _, j in trace:
        c = rc.pinned_empty((j.bands, j.detectors, 4), np.float64)
        c[...] = j.coeffs()
        coeffs.append(c)
    # Jobs checked against the oracle get outputs of their own.
    small = sorted(range(len(trace)), key=lambda i: trace[i][1].pixels)[:6]
    verify = set(small) | set(range(0, len(trace), max(1, len(trace) // 4)))
    outs = {i: rc.pinned_empty(trace[i][1].pixels, np.uint16) for i in verify}
    setup_s = time.time() - t0

    def dn_of(i):
        j = trace[i][1]
        o = offsets[i]
        return pools[depth_of(j)][o:o + j.pixels].reshape(j.bands, j.lines, j.detectors)

    def out_of(i):
        j = trace[i][1]
        buf = outs[i] if i in outs else sinks[depth_of(j)][:j.pixels]
        return buf.reshape(j.bands, j.lines, j.detectors)

    # Pinned copy bandwidth, for the PCIe ceiling.
    probe = pools[10][:256 << 20] if max_px >= (256 << 20) else pools[10]
    d_t = torch.empty(probe.shape, dtype=torch.int16, device=dev)
    src = torch.from_numpy(probe.view(np.int16))
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    for _ in range(3):
        d_t.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    h2d_gbs = 3 * probe.nbytes / (time.perf_counter() - c0) / 1e9
    dst = torch.from_numpy(sinks[10][:probe.size].view(np.int16))
    c0 = time.perf_counter()
    for _ in range(3):
        dst.copy_(d_t, non_blocking=True)
    torch.cuda.synchronize()
    d2h_gbs = 3 * probe.nbytes / (time.perf_counter() - c0) / 1e9
    del d_t

    def run_server():
        srv = rc.Server()
        ids = [None] * len(trace)
        start = time.perf_counter()

        def client():
            for i, (t_arr, j) in enumerate(trace):
                delay = start + t_arr - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                ids[i] = srv.submit(coeffs[i], dn_of(i), out_of(i), j.levels)

        th = threading.Thread(target=client)
        th.start()
        th.join()
        stats = [srv.wait(ids[i]) for i in range(len(trace))]
        info = srv.info()
        srv.close()
        return stats, info

    stats, info = run_server()
    ok = all(st["status"] == rc.RC_OK for st in stats)
    lat = [st["latency_s"] for st in stats]
    waits = [st["admit_s"] - st["submit_s"] for st in stats]
    first = min(st["submit_s"] for st in stats)
    last = max(st["done_s"] for st in stats)
    px = sum(j.pixels for _, j in trace)
    o = oracle.get()
    exact = True
    for i in sorted(verify):
        j = trace[i][1]
        w = o.correct(dn_of(i), o.lut_build(coeffs[i], j.levels))
        exact &= bool(np.array_equal(out_of(i), w))

    # Plain server: the same arrivals, one job at a time on one stream.
    stream = torch.cuda.Stream(device=dev)
    plain_lat, plain_done = [], []
    start = time.perf_counter()
    for i, (t_arr, j) in enumerate(trace):
        delay = start + t_arr - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        with torch.cuda.stream(stream):
            c_t = torch.from_numpy(coeffs[i]).to(dev, non_blocking=True)
            d_in = torch.from_numpy(dn_of(i).view(np.int16)).to(dev, non_blocking=True)
            lut = torch.empty((j.bands, j.detectors, j.levels), dtype=torch.int16, device=dev)
            d_out = torch.empty_like(d_in)
            rc.rc_lut_build(c_t, j.bands, j.detectors, j.levels, lut, stream)
            rc.rc_correct(d_in, lut, j.lines, j.detectors, j.bands, j.levels, d_out, stream)
            torch.from_numpy(out_of(i).view(np.int16)).copy_(d_out, non_blocking=True)
        stream.synchronize()
        now = time.perf_counter()
        plain_lat.append(now - (start + t_arr))
        plain_done.append(now - start)
        del c_t, d_in, lut, d_out
    torch.cuda.empty_cache()
    plain_span = plain_done[-1] - trace[0][0]
    return {
        "workload": f"{len(trace)} jobs, Poisson arrivals at {args.serve_qps:g} jobs/s, "
                    "log-uniform 1-600 Mpix, 1-4 bands, 10/12-bit, pinned host buffers, "
                    "each job's image at its own seeded offset of a "
                    f"{pool_px / 2**30:.1f} Gi-pixel pool per bit depth",
        "jobs": len(trace),
        "pixels": px, "offered_gpix_s": round(px / trace[-1][0] / 1e9, 2),
        "served_gpix_s": round(px / (last - first) / 1e9, 2),
        "p50_latency_ms": round(percentile(lat, 50) * 1e3, 2),
        "p99_latency_ms": round(percentile(lat, 99) * 1e3, 2),
        "p50_admission_wait_ms": round(percentile(waits, 50) * 1e3, 3),
        "p99_admission_wait_ms": round(percentile(waits, 99) * 1e3, 3),
        "max_admission_wait_ms": round(max(waits) * 1e3, 3),
        "plain_gpix_s": round(px / plain_span / 1e9, 2),
        "plain_p50_latency_ms": round(percentile(plain_lat, 50) * 1e3, 2),
        "plain_p99_latency_ms": round(percentile(plain_lat, 99) * 1e3, 2),
        "pinned_h2d_gb_s": round(h2d_gbs, 1), "pinned_d2h_gb_s": round(d2h_gbs, 1),
        "pcie_bound_gpix_s": round(min(h2d_gbs, d2h_gbs) / 2, 2),
        "quanta": info["quanta"], "tiles": info["tiles"], "direct_out_jobs": info["direct_out"],
        "all_ok": ok, "bit_exact_oracle_sample": exact,
        "oracle_sample_jobs": sorted(int(i) for i in verify), "setup_s": round(setup_s, 1),
    }


def kernel_source_hash():
    """Hash of the correction's sources with comments and whitespace removed,
    so that counters stay attached to the code they were taken on."""
    h = hashlib.sha256()
    for f in ("device_ops.h", "lut_apply.hip", "api.cpp"):
        with open(os.path.join(ROOT, "paper_1505_05655_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(workload_name):
    """HBM bytes per correction launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source.

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are each scaled by what the
    same counter reads for a plain device copy of known size on the same GPU.
    """
    path = os.path.join(PROFILES, f"lut_apply_{workload_name}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_sha") != kernel_source_hash():
        return None
    cal = d["copy_calibration"]
    fetch_scale = cal["bytes_each_way"] / (cal["fetch_kib"] * 1024.0)
    write_scale = cal["bytes_each_way"] / (cal["write_kib"] * 1024.0)
    return round(d["fetch_kib"] * 1024.0 * fetch_scale + d["write_kib"] * 1024.0 * write_scale)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def copy_plan_default(rc):
    """Launch shape of the linear-copy ceiling: one 256-thread workgroup per
    CU, 4 x 16 bytes in flight per lane, non-temporal loads and stores (the
    fastest shape of a sweep over 256-1024 threads, 2-8 loads, 1-8
    workgroups per CU and three cache policies on 1.15 and 1.8 GB copies)."""
    return rc.CopyPlan(threads=256, unroll=4, policy=1, wgs_per_cu=1)


def measure_scene(args, torch, rc, dev, s, steps, warmup, cpu_seconds, verify, cpu_baseline):
    """One single-scene workload: K timed steps of rc_lut_build + rc_correct
    (HIP events around each kernel on the launch stream, plus the wall clock
    of the whole loop), cold-cache steps, the copy ceilings of the same image,
    the CPU oracle timed on this host, and a bit-exact check."""
    import oracle
    t0 = time.time()
    coeffs = s.coeffs()
    dn = s.dn()
    print(f"[bench] workload {s.name}: {s.pixels / 1e6:.1f} Mpix generated in "
          f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    c_t = torch.from_numpy(coeffs).to(dev)
    dn_t = torch.from_numpy(dn.view(np.int16)).to(dev)
    lut_t = torch.empty((s.bands, s.detectors, s.levels), dtype=torch.int16, device=dev)
    out_t = torch.empty_like(dn_t)
    stream = torch.cuda.Stream(device=dev)  # default priority
    plan, tuned = rc.rc_plan_for(s.lines, s.detectors, s.bands, s.levels, dn_t, out_t)
    # Long LUT rows: the correction with a workspace (the LUT encoded once for
    # the whole scene, then the dense tiles), else the plain call.
    ws_bytes = rc.rc_correct_ws_bytes(s.detectors, s.bands, s.levels)
    ws_t = torch.empty(max(ws_bytes, 256) // 2, dtype=torch.int16, device=dev)

    def correct_plain():
        rc.rc_correct(dn_t, lut_t, s.lines, s.detectors, s.bands, s.levels, out_t, stream)

    def correct_ws():
        rc.rc_correct_ws(dn_t, lut_t, s.lines, s.detectors, s.bands, s.levels, out_t, ws_t,
                         ws_bytes, None, stream)

    def correct_pre():
        rc.rc_correct_pre(dn_t, lut_t, s.lines, s.detectors, s.bands, s.levels, out_t, ws_t,
                          ws_bytes, None, stream)

    def build_plain():
        rc.rc_lut_build(c_t, s.bands, s.detectors, s.levels, lut_t, stream)

    def build_ws():
        rc.rc_lut_build_ws(c_t, s.bands, s.detectors, s.levels, lut_t, ws_t, ws_bytes, stream)

    # Long LUT rows: the build also writes the LUT's dense encoding to the
    # workspace, and the correction's tiles stage that (no encoding pass).
    build = build_ws if ws_bytes else build_plain
    correct = correct_pre if ws_bytes else correct_plain
    entry = "rc_lut_build_ws + rc_correct_pre" if ws_bytes else "rc_lut_build + rc_correct"

    def step():
        build()
        correct()

    torch.cuda.synchronize()
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()

    # Timed region: K whole steps, events around each kernel on the launch stream.
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        build()
        ev[k][1].record(stream)
        correct()
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    build_ms = [ev[k][0].elapsed_time(ev[k][1]) for k in range(steps)]
    apply_ms = [ev[k][1].elapsed_time(ev[k][2]) for k in range(steps)]
    ms_per_step = wall * 1e3 / steps

    px = s.pixels
    lut_bytes = s.bands * s.detectors * s.levels * 2
    # 2 B read + 2 B written per pixel + the LUT read once; with the
    # workspace the LUT reaches the correction as its dense encoding (8-byte
    # plane + 2-byte header per 64-level block), which the build writes.
    enc_bytes = s.bands * s.detectors * -(-s.levels // 64) * 10 if ws_bytes else 0
    apply_bytes = 4 * px + (enc_bytes if ws_bytes else lut_bytes)
    build_bytes = lut_bytes + enc_bytes + s.bands * s.detectors * 32  # written + coefficients
    apply_avg = statistics.mean(apply_ms)
    achieved = apply_bytes / (apply_avg * 1e-3) / 1e9

    # Cold caches: before each of 10 extra steps a 512 MiB scratch write
    # evicts the LUT from L2 and the 256 MB MALL; events around each kernel.
    scratch = torch.empty(256 << 20, dtype=torch.int16, device=dev)
    cold_b, cold_a = [], []
    for _ in range(10):
        with torch.cuda.stream(stream):
            scratch.fill_(1)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        build()
        e[1].record(stream)
        correct()
        e[2].record(stream)
        stream.synchronize()
        cold_b.append(e[0].elapsed_time(e[1]))
        cold_a.append(e[1].elapsed_time(e[2]))
    del scratch
    cold_avg = statistics.mean(cold_a)

    # Practical ceilings beside the roofline: plain copies of the same image
    # (2 B read + 2 B written per pixel, no LUT) on the same stream, timed the
    # same way: the library's hand-written linear copy and torch's.
    cp_t = torch.empty_like(dn_t)
    cplan = copy_plan_default(rc)

    def time_copy(fn, n=20):
        res = []
        for i in range(n + 3):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e[0].record(stream)
            fn()
            e[1].record(stream)
            if i >= 3:
                res.append(e)
        stream.synchronize()
        return [a.elapsed_time(b) for a, b in res]

    # The plain call on the same scene (when the headline uses the workspace);
    # the headline path's output is kept for the bit-exact check first.
    head_out = out_t.cpu().numpy().view(np.uint16) if ws_bytes else None
    pair = None
    if ws_bytes:
        # The same step as two plain calls, for reference: rc_lut_build, then
        # rc_correct_ws (which encodes the LUT itself); 3 + 10 steps.
        pev = []
        for i in range(13):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(stream)
            build_plain()
            e[1].record(stream)
            correct_ws()
            e[2].record(stream)
            if i >= 3:
                pev.append(e)
        stream.synchronize()
        pair = {"lut_build_ms": round(statistics.mean(e[0].elapsed_time(e[1]) for e in pev), 4),
                "rc_correct_ws_ms": round(statistics.mean(e[1].elapsed_time(e[2]) for e in pev), 4),
                "step_ms": round(statistics.mean(e[0].elapsed_time(e[2]) for e in pev), 4),
                "note": "rc_lut_build + rc_correct_ws back to back, 10 steps"}
    plain_ms = time_copy(correct_plain, 10) if ws_bytes else None
    rc_cp_ms = time_copy(lambda: rc.rc_stream_copy(dn_t, cp_t, 2 * px, cplan, stream))
    copy_ok = bool(torch.equal(cp_t, dn_t))

    def torch_copy():
        with torch.cuda.stream(stream):
            cp_t.copy_(dn_t)

    th_cp_ms = time_copy(torch_copy)
    del cp_t
    rc_copy_gbs = 4 * px / (statistics.mean(rc_cp_ms) * 1e-3) / 1e9
    th_copy_gbs = 4 * px / (statistics.mean(th_cp_ms) * 1e-3) / 1e9

    bit_exact = None
    cpu = None
    if cpu_baseline or verify:
        o = oracle.get()
        # The oracle is single-threaded; time whole passes of the same step
        # (LUT build + correction) until at least cpu_seconds have elapsed.
        # The calling thread is pinned to one core while it runs the oracle.
        want = np.empty_like(dn)
        affinity = os.sched_getaffinity(0)
        core = max(affinity)
        try:
            os.sched_setaffinity(0, {core})
            pinned = f"pinned to core {core}"
        except OSError:
            pinned = "not pinned (affinity refused)"
        try:
            passes, c0, build_s = 0, time.perf_counter(), 0.0
            while True:
                b0 = time.perf_counter()
                want_lut = o.lut_build(coeffs, s.levels)
                build_s += time.perf_counter() - b0
                o.correct(dn, want_lut, out=want)
                passes += 1
                el = time.perf_counter() - c0
                if not cpu_baseline or el >= cpu_seconds:
                    break
        finally:
            try:
                os.sched_setaffinity(0, affinity)
            except OSError:
                pass
        if cpu_baseline:
            cpu = {"value": round(px * passes / el / 1e9, 4), "unit": "Gpix/s", "cores": 1,
                   "kind": "oracle",
                   "lut_build_s": round(build_s / passes, 4),
                   "correct_s": round((el - build_s) / passes, 4),
                   "sample": f"{passes} full pass(es) of the same step (LUT build + correction "
                             f"of all {px} pixels), {el:.1f}s, single-threaded, {pinned}, host "
                             f"{cpu_model()} with {os.cpu_count()} logical CPUs"}
        if verify:
            got = out_t.cpu().numpy().view(np.uint16)
            got_lut = lut_t.cpu().numpy().view(np.uint16)
            bit_exact = bool(np.array_equal(got, want) and np.array_equal(got_lut, want_lut))
            if head_out is not None:  # both the workspace path and the plain call
                bit_exact = bit_exact and bool(np.array_equal(head_out, want))
    del dn_t, out_t, lut_t, c_t, ws_t
    torch.cuda.empty_cache()

    return {
        "workload": s.name, "config": {"workload": s.name, "bands": s.bands, "lines": s.lines,
                                       "detectors": s.detectors, "levels": s.levels,
                                       "seed": s.seed, "entry_point": entry,
                                       "workspace_bytes": ws_bytes,
                                       "plan": None if ws_bytes else plan.as_dict(),
                                       "plan_tuned": None if ws_bytes else tuned},
        "value": round(px / (ms_per_step * 1e-3) / 1e9, 3),
        "ms_per_step": round(ms_per_step, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic(s.name),
                     "kernel": ("correction: k_apply on the build's dense encoding (rc_correct_pre)"
                                if ws_bytes else "lut_apply (k_apply)"),
                     "algorithmic_bytes": apply_bytes,
                     "launch_ms_mean": round(apply_avg, 4),
                     "frac_cold": round(apply_bytes / (cold_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "cpu_baseline": cpu,
        "bit_exact": bit_exact,
        "kernels": {
            "lut_apply_ms": {"mean": round(apply_avg, 4), "min": round(min(apply_ms), 4),
                             "median": round(statistics.median(apply_ms), 4),
                             "p10": round(percentile(apply_ms, 10), 4),
                             "p90": round(percentile(apply_ms, 90), 4)},
            "lut_apply_gpix_s": round(px / (apply_avg * 1e-3) / 1e9, 2),
            "workspace_pair": pair,
            "plain_rc_correct": None if not ws_bytes else {
                "ms_mean": round(statistics.mean(plain_ms), 4),
                "frac_hbm": round(apply_bytes / (statistics.mean(plain_ms) * 1e-3) / 1e9 /
                                  HBM_PEAK_GBS, 4),
                "plan": plan.as_dict(), "plan_tuned": tuned},
            "lut_build_ms": {"mean": round(statistics.mean(build_ms), 4),
                             "min": round(min(build_ms), 4),
                             "median": round(statistics.median(build_ms), 4),
                             "p10": round(percentile(build_ms, 10), 4),
                             "p90": round(percentile(build_ms, 90), 4)},
            "lut_build_gb_s": round(build_bytes / (statistics.mean(build_ms) * 1e-3) / 1e9, 1),
            "cold_caches": {"lut_apply_ms_mean": round(cold_avg, 4),
                            "lut_apply_ms_median": round(statistics.median(cold_a), 4),
                            "lut_build_ms_median": round(statistics.median(cold_b), 4),
                            "frac_hbm": round(apply_bytes / (cold_avg * 1e-3) / 1e9 /
                                              HBM_PEAK_GBS, 4),
                            "steps": len(cold_a),
                            "note": "512 MiB scratch write before each step"},
            "copy_ceiling": {
                "rc_stream_copy_ms_mean": round(statistics.mean(rc_cp_ms), 4),
                "rc_stream_copy_gb_s": round(rc_copy_gbs, 1),
                "rc_stream_copy_frac": round(rc_copy_gbs / HBM_PEAK_GBS, 4),
                "rc_stream_copy_plan": cplan.as_dict(), "rc_stream_copy_exact": copy_ok,
                "torch_copy_ms_mean": round(statistics.mean(th_cp_ms), 4),
                "torch_copy_gb_s": round(th_copy_gbs, 1),
                "lut_apply_vs_rc_copy": round(achieved / rc_copy_gbs, 3),
                "note": "device-to-device copies of the input image (4 B per pixel moved), "
                        "20 launches each on the launch stream"},
        },
    }


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); the work shards "
              "by band and detector strip with no exchange between GPUs, so it is not run here.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import gen
    import paper_1505_05655_amd as rc

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    head = measure_scene(args, torch, rc, dev, gen.workload(args.workload), args.steps,
                         args.warmup, args.cpu_seconds, not args.no_verify,
                         not args.no_cpu_baseline)
    # The other single-scene workloads, each with its own roofline (20 warm-up
    # and 20 timed steps, bit-exact check, no CPU timing).
    scenes = []
    if not args.no_scenes:
        for w in (1, 2):
            if w == args.workload:
                continue
            r = measure_scene(args, torch, rc, dev, gen.workload(w), 20, 20, 0.0,
                              not args.no_verify, False)
            r.pop("cpu_baseline")
            scenes.append(r)

    # End to end (pinned host in, pinned host out) for the headline scene and,
    # with the scenes leg, the other large one.
    e2e_ws = [args.workload] + ([] if args.no_scenes else
                                [w for w in (1, 2) if w != args.workload])
    e2e_res = None if args.no_e2e else [bench_e2e(args, torch, rc, dev, gen.workload(w))
                                        for w in e2e_ws]
    fit_res = None if args.no_fit else bench_fit(args, torch, rc, dev)
    demosaic_res = None if args.no_demosaic else bench_demosaic(args, torch, rc, dev)
    gradient_res = (None if args.no_demosaic else
                    bench_demosaic(args, torch, rc, dev, method="gradient"))
    small_res = None if args.no_small else bench_small(args, torch, rc, dev)

    batch_res = None
    torch.cuda.empty_cache()
    if not args.no_batch:
        print("[bench] batch leg", file=sys.stderr, flush=True)
        batch_res = bench_batch(args, torch, rc, dev)

    serve_res = None
    if not args.no_serve:
        print("[bench] serve leg", file=sys.stderr, flush=True)
        serve_res = bench_serve(args, torch, rc, dev)

    props = torch.cuda.get_device_properties(dev)
    line = {
        "metric": "corrected Gpix/s (LUT build + correction per step), bit-exact vs CPU oracle",
        "value": head["value"],
        "unit": "Gpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16 gather (LUT build in f64)",
        "data": "synthetic, seeded",
        "config": head["config"],
        "roofline": head["roofline"],
        "cpu_baseline": head["cpu_baseline"],
        "bit_exact": head["bit_exact"],
        "kernels": head["kernels"],
        "scenes": scenes,
        "e2e": e2e_res,
        "fit": fit_res,
        "demosaic": demosaic_res,
        "demosaic_gradient": gradient_res,
        "small_scene_graph": small_res,
        "batch": batch_res,
        "serve": serve_res,
        "device": {"name": props.name, "cus": props.multi_processor_count,
                   "hbm_gib": round(props.total_memory / 2 ** 30, 1),
                   "arch": getattr(props, "gcnArchName", "")},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
