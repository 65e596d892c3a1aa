"""ctypes binding of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package. The GPU library never does; the product path fails loudly when
its own HIP library is missing instead of falling back to this code.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load(path=None):
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or _build.LIB
    if not os.path.exists(p):
        _build.build(out=p)
    lib = ctypes.CDLL(p)
    u16p = ctypes.POINTER(ctypes.c_uint16)
    f64p = ctypes.POINTER(ctypes.c_double)
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.oracle_lut_entry.argtypes = [f64p, i32, i32]
    lib.oracle_lut_entry.restype = ctypes.c_uint16
    lib.oracle_lut_build.argtypes = [f64p, i32, i32, i32, u16p]
    lib.oracle_lut_build.restype = None
    lib.oracle_correct.argtypes = [u16p, u16p, i64, i32, i32, i32, u16p]
    lib.oracle_correct.restype = None
    lib.oracle_pixel.argtypes = [f64p, u16p, i64, i32, i32, i32, u16p]
    lib.oracle_pixel.restype = None
    lib.oracle_fit.argtypes = [f64p, f64p, i32, i32, i32, i32, f64p]
    lib.oracle_fit.restype = None
    lib.oracle_demosaic.argtypes = [u16p, i32, i32, i32, u16p]
    lib.oracle_demosaic.restype = None
    lib.oracle_demosaic_gradient.argtypes = [u16p, i32, i32, i32, u16p]
    lib.oracle_demosaic_gradient.restype = None
    if path is None:
        _lib = lib
    return lib


def _f64(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u16(a):
    assert a.dtype == np.uint16 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16))


class Oracle:
    """Typed numpy front end over one oracle shared library (the real one or
    a test build)."""

    def __init__(self, path=None):
        self.lib = _load(path)

    def lut_entry(self, a, v, levels):
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(4)
        return int(self.lib.oracle_lut_entry(_f64(a), int(v), int(levels)))

    def lut_build(self, coeffs, levels, out=None):
        """coeffs: float64 [B, D, 4] -> uint16 [B, D, L]."""
        coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
        B, D, k = coeffs.shape
        assert k == 4
        if out is None:
            out = np.empty((B, D, levels), dtype=np.uint16)
        self.lib.oracle_lut_build(_f64(coeffs), B, D, int(levels), _u16(out))
        return out

    def correct(self, dn, lut, out=None):
        """dn: uint16 [B, N, D], lut: uint16 [B, D, L] -> uint16 [B, N, D]."""
        dn = np.ascontiguousarray(dn, dtype=np.uint16)
        lut = np.ascontiguousarray(lut, dtype=np.uint16)
        B, N, D = dn.shape
        assert lut.shape[:2] == (B, D)
        L = lut.shape[2]
        if out is None:
            out = np.empty_like(dn)
        self.lib.oracle_correct(_u16(dn), _u16(lut), N, D, B, L, _u16(out))
        return out

    def pixel(self, coeffs, dn, levels, out=None):
        """Brute force per-pixel evaluation, no table."""
        coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
        dn = np.ascontiguousarray(dn, dtype=np.uint16)
        B, N, D = dn.shape
        assert coeffs.shape == (B, D, 4)
        if out is None:
            out = np.empty_like(dn)
        self.lib.oracle_pixel(_f64(coeffs), _u16(dn), N, D, B, int(levels), _u16(out))
        return out


    def fit(self, x, y, order, out=None):
        """Least-squares fit. x: float64 [B, n, D] (detector values on n
        calibration lines), y: float64 [B, n] (targets) -> float64 [B, D, 4]."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        B, n, D = x.shape
        assert y.shape == (B, n)
        if out is None:
            out = np.empty((B, D, 4), dtype=np.float64)
        self.lib.oracle_fit(_f64(x), _f64(y), B, n, D, int(order), _f64(out))
        return out


    def demosaic(self, raw, out=None):
        """raw: uint16 [I, H, W] (RGGB Bayer) -> uint16 [I, 3, H, W] (R, G, B planes)."""
        raw = np.ascontiguousarray(raw, dtype=np.uint16)
        I, H, W = raw.shape
        if out is None:
            out = np.empty((I, 3, H, W), dtype=np.uint16)
        self.lib.oracle_demosaic(_u16(raw), I, H, W, _u16(out))
        return out


    def demosaic_gradient(self, raw, out=None):
        """raw: uint16 [I, H, W] (RGGB) -> uint16 [I, 3, H, W], adaptive colour plane."""
        raw = np.ascontiguousarray(raw, dtype=np.uint16)
        I, H, W = raw.shape
        if out is None:
            out = np.empty((I, 3, H, W), dtype=np.uint16)
        self.lib.oracle_demosaic_gradient(_u16(raw), I, H, W, _u16(out))
        return out


_default = None


def get():
    """The oracle built from oracle/oracle.cpp."""
    global _default
    if _default is None:
        _default = Oracle()
    return _default
