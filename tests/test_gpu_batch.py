"""Batched execution (persistent kernel + hipGraph) against the oracle and
against the same requests run alone, bit-exact, over repeated graph replays
with eager work in between."""
import json

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_1505_05655_amd as rc
import pins
from gpu_util import dev, to_dev_f64, to_dev_u16, to_host_u16

pytestmark = pytest.mark.gpu

# (bands, lines, detectors, levels, coefficient style, dn offset, in place)
SPECS = [
    (1, 1, 1, 2, "tiny", 0, False),
    (2, 333, 1000, 1024, "quad", 0, False),
    (3, 517, 130, 4096, "cubic", 0, False),
    (1, 700, 513, 1024, "quad", 0, False),      # odd detector count
    (4, 64, 1030, 1024, "quad", 0, False),      # detectors = 2 mod 4
    (1, 20, 77, 65536, "tiny", 0, False),       # 16-bit LUT: L2 path
    (2, 100, 300, 3, "tiny", 0, False),         # raw LDS path
    (1, 1300, 64, 1000, "quad", 0, False),
    (2, 200, 256, 1024, "tiny", 0, False),      # rows that cannot be packed
    (2, 150, 200, 1024, "quad", 0, True),       # in place
    (2, 0, 50, 1024, "quad", 0, False),         # LUT only, no lines
    (1, 90, 100, 1024, "quad", 1, False),       # 2-byte aligned image
    (1, 9000, 64, 1024, "quad", 0, False),      # lines split into chunks
    (2, 120, 90, 700, "quad", 0, False),        # packed: 22 blocks, L % 8 != 0
    (1, 50, 40, 513, "quad", 0, False),         # packed: last block holds one level
]


def make_inputs(i, spec):
    B, N, D, L, style, _, _ = spec
    if style == "tiny":
        coeffs, dn = pins.tiny_case(500 + i, B, max(N, 1), D, L)
        dn = dn[:, :N]
    else:
        kind = gen.COEF_QUADRATIC if style == "quad" else gen.COEF_CUBIC
        coeffs = gen.coeffs(gen.BASE_SEED, 9, i, kind, B, D)
        dkind = gen.DN_GAUSS_SAT10 if style == "quad" else gen.DN_SCENE12
        dn = gen.dn(gen.BASE_SEED, 9, i, dkind, B, N, D) if N else np.zeros((B, 0, D), np.uint16)
        if L not in (1024, 4096):
            dn = np.minimum(dn, L + 7).astype(np.uint16)
    return coeffs, np.ascontiguousarray(dn)


class Job:
    def __init__(self, i, spec):
        B, N, D, L, _, off, in_place = spec
        self.spec = spec
        self.coeffs, self.dn = make_inputs(i, spec)
        self.c_t = to_dev_f64(self.coeffs)
        n = B * N * D
        self.dn_base = torch.zeros(n + off + 8, dtype=torch.int16, device=dev())
        self.dn_t = self.dn_base[off:off + n].view(B, N, D)
        self.dn_t.copy_(to_dev_u16(self.dn))
        self.lut_t = torch.zeros((B, D, L), dtype=torch.int16, device=dev())
        self.out_t = self.dn_t if in_place else torch.zeros((B, N, D), dtype=torch.int16,
                                                            device=dev())
        o = oracle.get()
        self.want_lut = o.lut_build(self.coeffs, L)
        self.want = o.correct(self.dn, self.want_lut)

    def reset(self):
        self.lut_t.zero_()
        if self.out_t is self.dn_t:
            self.dn_t.copy_(to_dev_u16(self.dn))
        else:
            self.out_t.zero_()

    def check(self, what):
        assert np.array_equal(to_host_u16(self.lut_t), self.want_lut), f"{what}: LUT {self.spec}"
        assert np.array_equal(to_host_u16(self.out_t), self.want), f"{what}: image {self.spec}"


@pytest.fixture(scope="module")
def jobs():
    return [Job(i, s) for i, s in enumerate(SPECS)]


@pytest.mark.parametrize("graph", [True, False])
def test_batch_matches_oracle(jobs, graph):
    for j in jobs:
        j.reset()
    batch = rc.Batch([(j.c_t, j.dn_t, j.lut_t, j.out_t) for j in jobs], graph=graph)
    info = batch.info()
    assert info["requests"] == len(jobs) and info["graph"] == int(graph) and info["tiles"] > 0
    for replay in range(3):
        batch.run()
        torch.cuda.synchronize()
        for j in jobs:
            j.check(f"replay {replay}")
        # Eager work between replays: wipe every output, then replay again.
        for j in jobs:
            j.reset()
        torch.cuda.synchronize()
    batch.close()


def test_batch_equals_alone(jobs):
    for j in jobs:
        j.reset()
    alone = []
    for j in jobs:
        B, N, D, L = j.spec[:4]
        lut = rc.lut_build(j.c_t, L)
        src = to_dev_u16(j.dn)
        out = rc.correct(src, lut)
        alone.append((lut, out))
    batch = rc.Batch([(j.c_t, j.dn_t, j.lut_t, j.out_t) for j in jobs])
    batch.run()
    torch.cuda.synchronize()
    for j, (lut, out) in zip(jobs, alone):
        assert torch.equal(j.lut_t, lut) and torch.equal(j.out_t, out), f"{j.spec}"
    batch.close()


def test_batch_workload3_sample():
    """A slice of the 256-request workload (first 12 requests, lines capped at
    512) through the batch: every pixel against the oracle."""
    reqs = gen.batch_requests(12)
    o = oracle.get()
    tensors, wants = [], []
    for r in reqs:
        n = min(r.lines, 512)
        c = r.coeffs()
        d = r.dn(nlines=n)
        lut_w = o.lut_build(c, r.levels)
        wants.append((lut_w, o.correct(d, lut_w)))
        tensors.append((to_dev_f64(c), to_dev_u16(d),
                        torch.empty((r.bands, r.detectors, r.levels), dtype=torch.int16,
                                    device=dev()),
                        torch.empty((r.bands, n, r.detectors), dtype=torch.int16, device=dev())))
    batch = rc.Batch(tensors)
    batch.run()
    torch.cuda.synchronize()
    for (c, d, lut, out), (lw, w) in zip(tensors, wants):
        assert np.array_equal(to_host_u16(lut), lw)
        assert np.array_equal(to_host_u16(out), w)
    batch.close()


def test_batch_tuned(jobs):
    """rc_batch_tune times candidate tile shapes per request class on the
    batch kernel; the batch then takes every request's shape from those
    entries, and stays bit-exact."""
    tensors = [(j.c_t, j.dn_t, j.lut_t, j.out_t) for j in jobs]
    try:
        classes = rc.batch_tune(tensors)
        torch.cuda.synchronize()
        with_px = [j for j in jobs if j.spec[0] * j.spec[1] * j.spec[2] > 0]
        assert 1 <= classes <= len(with_px)
        for j in jobs:
            j.reset()  # the tuning runs corrected the in-place request repeatedly
        torch.cuda.synchronize()
        batch = rc.Batch(tensors)
        info = batch.info()
        assert info["tuned"] == len(with_px)
        assert info["fused"] + (info["lut_gather_entries"] > 0) >= 1
        for replay in range(2):
            batch.run()
            torch.cuda.synchronize()
            for j in jobs:
                j.check(f"tuned, replay {replay}")
            for j in jobs:
                j.reset()
            torch.cuda.synchronize()
        batch.close()
    finally:
        rc.rc_tune_load()  # drop the in-memory batch entries


def _vmax(j):
    """The batch's pixels per lane bound for a job (4, 2 or 1), as librc
    derives it from the detector count and the image alignment."""
    D = j.spec[2]
    al = j.dn_t.data_ptr() | j.out_t.data_ptr()
    if D % 4 == 0 and al % 8 == 0:
        return 4
    if D % 2 == 0 and al % 4 == 0:
        return 2
    return 1


@pytest.mark.parametrize("path,strip", [(rc.RC_PATH_DENSE, 128), (rc.RC_PATH_DENSE, 512),
                                        (rc.RC_PATH_PACKED, 64), (rc.RC_PATH_LDS, 16),
                                        (rc.RC_PATH_L2, 64)])
def test_batch_forced_shapes(jobs, tmp_path, path, strip):
    """Batch entries of the plan cache decide each request's tile shape: each
    mode (dense, packed and raw LDS tiles built from the coefficients, and
    the L2 path), forced for every request through a cache file, stays
    bit-exact over two replays."""
    props = torch.cuda.get_device_properties(dev())
    arch = props.gcnArchName.split(":")[0]
    lines, seen = [], set()
    for j in jobs:
        B, N, D, L = j.spec[:4]
        if B * N * D == 0:
            continue
        key = (L, max(0, (D - 1).bit_length()), _vmax(j))
        if key in seen:
            continue
        seen.add(key)
        lines.append(json.dumps({
            "arch": arch, "cus": props.multi_processor_count, "levels": key[0],
            "dclass": key[1], "nclass": 0, "bands": 0, "vmax": key[2], "path": path,
            "strip": strip, "vec": key[2], "threads": 1024, "unroll": 4, "chunks": 1,
            "xcd_remap": 1, "nontemporal": 0, "strips": 0, "lane_map": 0, "kind": 1,
            "us": 1.0}))
    cache = tmp_path / "batch_cache.json"
    cache.write_text("\n".join(lines) + "\n")
    try:
        assert rc.rc_tune_load(str(cache)) == len(lines)
        for j in jobs:
            j.reset()
        torch.cuda.synchronize()
        batch = rc.Batch([(j.c_t, j.dn_t, j.lut_t, j.out_t) for j in jobs])
        info = batch.info()
        assert info["tuned"] == sum(1 for j in jobs if j.spec[0] * j.spec[1] * j.spec[2] > 0)
        for replay in range(2):
            batch.run()
            torch.cuda.synchronize()
            for j in jobs:
                j.check(f"path {path} strip {strip}, replay {replay}")
            for j in jobs:
                j.reset()
            torch.cuda.synchronize()
        batch.close()
    finally:
        rc.rc_tune_load()
