"""Seeded synthetic inputs for the LUT-correction workloads (no method arithmetic).

Both the GPU path's tests and the CPU oracle take their inputs from here. The
native part (gen.cpp) is a counter-based SplitMix64 generator, so any band or
line range can be regenerated independently of the others.

Workloads (seed = BASE_SEED + workload index):
  0  1 band x 1024 lines x 1024 detectors, L = 1024, DN uniform 10-bit,
     quadratic coefficients a0~N(0,8), a1~U(0.9,1.1), a2~N(0,1e-5)
  1  4 bands x 12000 lines x 12000 detectors, L = 1024, DN clipped N(400,150)
     plus 1 % saturated pixels, quadratic coefficients as workload 0
  2  3 bands x 50000 lines x 6000 detectors, L = 4096, 12-bit DN (half uniform,
     half a smooth scene field), cubic coefficients a0~N(0,32), a1~U(0.9,1.1),
     a2~N(0,1e-6), a3~N(0,1e-10)
  3  256 uneven requests (lines, detectors in [512, 8192], 1-4 bands, 10/12 bit)
  4  serving trace: Poisson arrivals, 1-600 Mpix jobs, 1-4 bands, 10/12 bit
"""
import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libgen.so")
BASE_SEED = 1505056550

COEF_QUADRATIC = 0
COEF_CUBIC = 1
DN_UNIFORM10 = 0
DN_GAUSS_SAT10 = 1
DN_SCENE12 = 2
DN_UNIFORM12 = 3


def build(quiet=True):
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall",
           os.path.join(HERE, "gen.cpp"), "-o", LIB + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("gen build failed:\n" + res.stderr)
    os.replace(LIB + ".tmp", LIB)
    if not quiet:
        print("built", LIB)


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    lib = ctypes.CDLL(LIB)
    u64, i32, i64 = ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64
    P = ctypes.POINTER
    lib.gen_splitmix64_next.argtypes = [P(u64)]
    lib.gen_splitmix64_next.restype = u64
    lib.gen_stream_key.argtypes = [u64] * 5
    lib.gen_stream_key.restype = u64
    lib.gen_draw.argtypes = [u64, u64]
    lib.gen_draw.restype = u64
    lib.gen_coeffs.argtypes = [u64, i32, i64, i32, i32, i32, P(ctypes.c_double)]
    lib.gen_coeffs.restype = None
    lib.gen_dn.argtypes = [u64, i32, i64, i32, i32, i64, i32, i64, i64,
                           P(ctypes.c_uint16), i32]
    lib.gen_dn.restype = None
    lib.gen_batch_dims.argtypes = [u64, i32, i32, P(i64), P(i32), P(i32), P(i32)]
    lib.gen_batch_dims.restype = None
    lib.gen_serve_jobs.argtypes = [u64, i32, i32, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, P(ctypes.c_double), P(i64), P(i32),
                                   P(i32), P(i32)]
    lib.gen_serve_jobs.restype = None
    lib.gen_calib.argtypes = [u64, i32, i64, i32, i32, i32, i32, P(ctypes.c_double),
                              P(ctypes.c_double)]
    lib.gen_calib.restype = None
    lib.gen_bayer.argtypes = [u64, i32, i64, i32, i32, i32, P(ctypes.c_uint16), i32]
    lib.gen_bayer.restype = None
    _lib = lib
    return lib


def _ptr(a, ct):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ct))


def splitmix64_sequence(state, n):
    lib = _load()
    s = ctypes.c_uint64(state)
    return [lib.gen_splitmix64_next(ctypes.byref(s)) for _ in range(n)]


def coeffs(seed, cfg, req, kind, bands, detectors):
    out = np.empty((bands, detectors, 4), dtype=np.float64)
    _load().gen_coeffs(seed, cfg, req, kind, bands, detectors, _ptr(out, ctypes.c_double))
    return out


def dn(seed, cfg, req, kind, bands, lines, detectors, n0=0, nlines=None, out=None,
       threads=0):
    """DN rows [n0, n0+nlines) of every band, shaped [bands, nlines, detectors]."""
    if nlines is None:
        nlines = lines - n0
    if out is None:
        out = np.empty((bands, nlines, detectors), dtype=np.uint16)
    assert out.shape == (bands, nlines, detectors) and out.dtype == np.uint16
    _load().gen_dn(seed, cfg, req, kind, bands, lines, detectors, n0, nlines,
                   _ptr(out, ctypes.c_uint16), threads)
    return out


def calib(seed, cfg, req, bands, points, detectors, levels):
    """Calibration acquisitions: x [bands, points, detectors] (detector
    responses on `points` flat-field lines) and y [bands, points] (the lines'
    reference levels), float64."""
    x = np.empty((bands, points, detectors), dtype=np.float64)
    y = np.empty((bands, points), dtype=np.float64)
    _load().gen_calib(seed, cfg, req, bands, points, detectors, levels,
                      _ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double))
    return x, y


def bayer(seed, cfg, req, images, height, width, threads=0):
    """Raw RGGB Bayer images, uint16 [images, height, width]."""
    out = np.empty((images, height, width), dtype=np.uint16)
    _load().gen_bayer(seed, cfg, req, images, height, width, _ptr(out, ctypes.c_uint16), threads)
    return out


def demosaic_workload(i, seed=None):
    """Demosaicing workloads as (name, seed, cfg, images, height, width):
    0 = the paper's single 2048 x 2048 16-bit image; 1 = a batch of 16 such
    images (enough workgroups to fill the GPU)."""
    s = BASE_SEED + 7 if seed is None else seed
    if i == 0:
        return ("1x2048x2048", s, 7, 1, 2048, 2048)
    if i == 1:
        return ("16x2048x2048", s, 8, 16, 2048, 2048)
    raise ValueError(f"no demosaic workload {i}")


@dataclass
class Calib:
    """A least-squares calibration fit: `points` calibration lines of
    `detectors` detectors per band, polynomial order `order`."""
    name: str
    seed: int
    cfg: int
    bands: int
    points: int
    detectors: int
    levels: int
    order: int

    def data(self):
        return calib(self.seed, self.cfg, 0, self.bands, self.points, self.detectors, self.levels)


def fit_workload(i, seed=None):
    """Fit workloads: 0 = the paper's data shape (one band, 6 calibration
    lines of 6000 pixels), order 2; 1 = the calibration of the 4-band,
    12000-detector scene, 6 lines, order 2."""
    s = BASE_SEED + 5 if seed is None else seed
    if i == 0:
        return Calib("1x6x6000_order2", s, 5, 1, 6, 6000, 1024, 2)
    if i == 1:
        return Calib("4x6x12000_order2", s, 6, 4, 6, 12000, 1024, 2)
    raise ValueError(f"no fit workload {i}")


@dataclass
class Scene:
    """One correction job: [bands, lines, detectors] uint16 DN + [bands, detectors, 4]
    float64 coefficients + level count."""
    name: str
    seed: int
    cfg: int
    req: int
    bands: int
    lines: int
    detectors: int
    levels: int
    coef_kind: int
    dn_kind: int

    @property
    def pixels(self):
        return self.bands * self.lines * self.detectors

    def coeffs(self):
        return coeffs(self.seed, self.cfg, self.req, self.coef_kind, self.bands,
                      self.detectors)

    def dn(self, n0=0, nlines=None, out=None, threads=0):
        return dn(self.seed, self.cfg, self.req, self.dn_kind, self.bands, self.lines,
                  self.detectors, n0, nlines, out, threads)


def workload(i, seed=None):
    """The single-scene workloads 0, 1 and 2."""
    s = BASE_SEED + i if seed is None else seed
    if i == 0:
        return Scene("1x1024x1024_L1024_quadratic", s, 0, 0, 1, 1024, 1024, 1024,
                     COEF_QUADRATIC, DN_UNIFORM10)
    if i == 1:
        return Scene("4x12000x12000_L1024_quadratic", s, 1, 0, 4, 12000, 12000, 1024,
                     COEF_QUADRATIC, DN_GAUSS_SAT10)
    if i == 2:
        return Scene("3x50000x6000_L4096_cubic", s, 2, 0, 3, 50000, 6000, 4096,
                     COEF_CUBIC, DN_SCENE12)
    raise ValueError("single-scene workloads are 0, 1 and 2")


def scene_for_depth(seed, cfg, req, bands, lines, detectors, depth, name=""):
    """A request of bit depth 10 (L = 1024, quadratic, clipped-Gaussian DN) or 12
    (L = 4096, cubic, scene DN)."""
    if depth == 10:
        return Scene(name, seed, cfg, req, bands, lines, detectors, 1024,
                     COEF_QUADRATIC, DN_GAUSS_SAT10)
    if depth == 12:
        return Scene(name, seed, cfg, req, bands, lines, detectors, 4096,
                     COEF_CUBIC, DN_SCENE12)
    raise ValueError("depth must be 10 or 12")


def batch_requests(n=256, seed=None, cfg=3):
    """Workload 3: n uneven requests."""
    s = BASE_SEED + 3 if seed is None else seed
    lines = np.empty(n, np.int64)
    dets = np.empty(n, np.int32)
    bands = np.empty(n, np.int32)
    depth = np.empty(n, np.int32)
    _load().gen_batch_dims(s, cfg, n, _ptr(lines, ctypes.c_int64), _ptr(dets, ctypes.c_int32),
                           _ptr(bands, ctypes.c_int32), _ptr(depth, ctypes.c_int32))
    return [scene_for_depth(s, cfg, r, int(bands[r]), int(lines[r]), int(dets[r]),
                            int(depth[r]), name=f"req{r}") for r in range(n)]


def serve_trace(n=2000, qps=150.0, mpix_lo=1.0, mpix_hi=600.0, seed=None, cfg=4):
    """Workload 4: (arrival seconds, Scene) for n jobs."""
    s = BASE_SEED + 4 if seed is None else seed
    t = np.empty(n, np.float64)
    lines = np.empty(n, np.int64)
    dets = np.empty(n, np.int32)
    bands = np.empty(n, np.int32)
    depth = np.empty(n, np.int32)
    _load().gen_serve_jobs(s, cfg, n, qps, mpix_lo, mpix_hi, _ptr(t, ctypes.c_double),
                           _ptr(lines, ctypes.c_int64), _ptr(dets, ctypes.c_int32),
                           _ptr(bands, ctypes.c_int32), _ptr(depth, ctypes.c_int32))
    return [(float(t[r]), scene_for_depth(s, cfg, r, int(bands[r]), int(lines[r]),
                                          int(dets[r]), int(depth[r]), name=f"job{r}"))
            for r in range(n)]
