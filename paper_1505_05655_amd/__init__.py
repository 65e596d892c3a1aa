"""Python binding of librc.so: radiometric LUT build and image correction on MI355X.

Argument marshalling only. Every step runs in the HIP kernels of librc.so;
PyTorch provides device memory (tensors) and streams. There is no CPU
fallback: importing this package fails if the library has not been built.

Functions named like the C ABI (``rc_fit``, ``rc_lut_build``, ``rc_correct``,
``rc_correct_plan``, ``rc_plan_for``, ``rc_demosaic``, ``rc_demosaic_gradient``) take
device tensors or raw device pointers (ints) plus the same sizes as the C functions. ``fit``,
``lut_build``, ``correct`` and ``demosaic`` are shape-checked conveniences on
top of them.

uint16 data is carried in torch.int16 (or torch.uint16) tensors: only the
bits matter and no arithmetic is done on them in Python.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it first (python __graft_entry__.py build, or "
        "python paper_1505_05655_amd/build.py). There is no CPU fallback.")

_lib = ctypes.CDLL(LIB_PATH)

RC_OK, RC_EINVAL, RC_ENOMEM, RC_EHIP, RC_EBUSY, RC_ECLOSED = range(6)
RC_PATH_LDS, RC_PATH_L2, RC_PATH_PACKED, RC_PATH_DENSE = 0, 1, 2, 3
RC_NCOEF = 4
RC_LEVELS_MIN, RC_LEVELS_MAX = 2, 65536


class RcError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.rc_status_str(status).decode()
        if status == RC_EHIP:
            msg += f" (hipError {_lib.rc_last_hip_error()})"
        super().__init__(f"{where}: {msg}")


class Plan(ctypes.Structure):
    """Launch shape of the correction kernel (mirrors rc_plan)."""
    _fields_ = [("path", ctypes.c_int32), ("strip", ctypes.c_int32), ("vec", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("chunk_lines", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("nontemporal", ctypes.c_int32), ("strips", ctypes.c_int32),
                ("lane_map", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}

    @classmethod
    def from_dict(cls, d):
        # `strips` and `lane_map` may be absent (plans written before they
        # existed: 0, strips of W with W / vec lanes per line)
        opt = ("strips", "lane_map")
        return cls(**{k: int(d.get(k, 0) if k in opt else d[k]) for k, _ in cls._fields_})

    def __repr__(self):
        return f"Plan({self.as_dict()})"


class CopyPlan(ctypes.Structure):
    """Launch shape of rc_stream_copy (mirrors rc_copy_plan)."""
    _fields_ = [("threads", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("policy", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Request(ctypes.Structure):
    """One job of a batch (mirrors rc_request); pointers are device addresses."""
    _fields_ = [("coeffs", ctypes.c_void_p), ("dn", ctypes.c_void_p), ("lut", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("lines", ctypes.c_int64), ("detectors", ctypes.c_int32),
                ("bands", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class BatchStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_int32), ("tiles", ctypes.c_int32),
                ("slots", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("pixels", ctypes.c_int64), ("lut_entries", ctypes.c_int64),
                ("tuned", ctypes.c_int32), ("fused", ctypes.c_int32),
                ("lut_gather_entries", ctypes.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


RC_BATCH_NO_GRAPH = 1


class ServerOpts(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_uint64), ("max_jobs", ctypes.c_int32),
                ("max_quantum_tiles", ctypes.c_int32), ("piece_pixels", ctypes.c_int64),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class HostJob(ctypes.Structure):
    _fields_ = [("coeffs", ctypes.c_void_p), ("dn", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("lut", ctypes.c_void_p), ("lines", ctypes.c_int64), ("detectors", ctypes.c_int32),
                ("bands", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class JobStats(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("latency_s", ctypes.c_double), ("pixels", ctypes.c_int64),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("quanta", ctypes.c_uint64), ("tiles", ctypes.c_uint64),
                ("pixels", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64),
                ("arena_used", ctypes.c_uint64), ("pending", ctypes.c_int32),
                ("active", ctypes.c_int32), ("waiters", ctypes.c_int32),
                ("direct_out", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}

_vp, _i32, _i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
_lib.rc_status_str.argtypes = [ctypes.c_int]
_lib.rc_status_str.restype = ctypes.c_char_p
_lib.rc_last_hip_error.argtypes = []
_lib.rc_last_hip_error.restype = _i32
_lib.rc_lut_build.argtypes = [_vp, _i32, _i32, _i32, _vp, _vp]
_lib.rc_lut_build.restype = ctypes.c_int
_lib.rc_fit.argtypes = [_vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp]
_lib.rc_fit.restype = ctypes.c_int
_lib.rc_demosaic.argtypes = [_vp, _i32, _i32, _i32, _vp, _vp]
_lib.rc_demosaic.restype = ctypes.c_int
_lib.rc_demosaic_gradient.argtypes = [_vp, _i32, _i32, _i32, _vp, _vp]
_lib.rc_demosaic_gradient.restype = ctypes.c_int
_lib.rc_correct.argtypes = [_vp, _vp, _i64, _i32, _i32, _i32, _vp, _vp]
_lib.rc_correct.restype = ctypes.c_int
_lib.rc_correct_plan.argtypes = [_vp, _vp, _i64, _i32, _i32, _i32, _vp, ctypes.POINTER(Plan), _vp]
_lib.rc_correct_plan.restype = ctypes.c_int
_lib.rc_plan_for.argtypes = [_i64, _i32, _i32, _i32, _vp, _vp, ctypes.POINTER(Plan),
                             ctypes.POINTER(_i32)]
_lib.rc_plan_for.restype = ctypes.c_int
_lib.rc_tune.argtypes = [_vp, _vp, _i64, _i32, _i32, _i32, _vp, _i32, ctypes.POINTER(Plan),
                         ctypes.POINTER(ctypes.c_float), _vp]
_lib.rc_tune.restype = ctypes.c_int
_lib.rc_tune_save.argtypes = [ctypes.c_char_p]
_lib.rc_tune_save.restype = _i32
_lib.rc_tune_load.argtypes = [ctypes.c_char_p]
_lib.rc_tune_load.restype = _i32
_lib.rc_tune_clear.argtypes = []
_lib.rc_tune_clear.restype = None
_lib.rc_tune_count.argtypes = []
_lib.rc_tune_count.restype = _i32
_lib.rc_batch_create.argtypes = [ctypes.POINTER(Request), _i32, _i32, ctypes.POINTER(_vp)]
_lib.rc_batch_create.restype = ctypes.c_int
_lib.rc_batch_tune.argtypes = [ctypes.POINTER(Request), _i32, _i32, ctypes.POINTER(_i32), _vp]
_lib.rc_batch_tune.restype = ctypes.c_int
_lib.rc_batch_run.argtypes = [_vp, _vp]
_lib.rc_batch_run.restype = ctypes.c_int
_lib.rc_batch_info.argtypes = [_vp, ctypes.POINTER(BatchStats)]
_lib.rc_batch_info.restype = ctypes.c_int
_lib.rc_batch_destroy.argtypes = [_vp]
_lib.rc_batch_destroy.restype = None
_lib.rc_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(_vp)]
_lib.rc_server_create.restype = ctypes.c_int
_lib.rc_server_submit.argtypes = [_vp, ctypes.POINTER(HostJob), ctypes.POINTER(ctypes.c_uint64)]
_lib.rc_server_submit.restype = ctypes.c_int
_lib.rc_server_wait.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(JobStats)]
_lib.rc_server_wait.restype = ctypes.c_int
_lib.rc_server_poll.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(JobStats)]
_lib.rc_server_poll.restype = ctypes.c_int
_lib.rc_server_info.argtypes = [_vp, ctypes.POINTER(ServerStats)]
_lib.rc_server_info.restype = ctypes.c_int
_lib.rc_server_destroy.argtypes = [_vp]
_lib.rc_server_destroy.restype = None
_lib.rc_correct_ws_bytes.argtypes = [_i32, _i32, _i32]
_lib.rc_correct_ws_bytes.restype = ctypes.c_size_t
_lib.rc_correct_ws.argtypes = [_vp, _vp, _i64, _i32, _i32, _i32, _vp, _vp, ctypes.c_size_t,
                               ctypes.POINTER(Plan), _vp]
_lib.rc_correct_ws.restype = ctypes.c_int
_lib.rc_lut_build_ws.argtypes = [_vp, _i32, _i32, _i32, _vp, _vp, ctypes.c_size_t, _vp]
_lib.rc_lut_build_ws.restype = ctypes.c_int
_lib.rc_correct_pre.argtypes = [_vp, _vp, _i64, _i32, _i32, _i32, _vp, _vp, ctypes.c_size_t,
                                ctypes.POINTER(Plan), _vp]
_lib.rc_correct_pre.restype = ctypes.c_int
_lib.rc_correct_noalloc.argtypes = [_vp, _vp, _i64, _i32, _i32, _i32, _vp, _vp]
_lib.rc_correct_noalloc.restype = ctypes.c_int
NOALLOC_SCRATCH_BYTES = 32 << 20
_lib.rc_stream_copy.argtypes = [_vp, _vp, ctypes.c_size_t, ctypes.POINTER(CopyPlan), _vp]
_lib.rc_stream_copy.restype = ctypes.c_int
_lib.rc_host_alloc.argtypes = [ctypes.c_size_t]
_lib.rc_host_alloc.restype = _vp
_lib.rc_host_free.argtypes = [_vp]
_lib.rc_host_free.restype = None


def lib():
    """The loaded ctypes library (for tests that call the C ABI directly)."""
    return _lib


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, torch.Tensor):
        if x.numel() and not x.is_cuda:
            raise ValueError("expected a device tensor")
        if not x.is_contiguous():
            raise ValueError("expected a contiguous tensor")
        return x.data_ptr() if x.numel() else None
    raise TypeError(f"expected a tensor or an int pointer, got {type(x)}")


def _stream(s):
    if s is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _check(st, where):
    if st != RC_OK:
        raise RcError(st, where)


# --- same-name wrappers of the C ABI ------------------------------------------------------

def rc_lut_build(coeffs, bands, detectors, levels, lut, stream=None):
    _check(_lib.rc_lut_build(_ptr(coeffs), bands, detectors, levels, _ptr(lut), _stream(stream)),
           "rc_lut_build")


def rc_fit(x, y, bands, points, detectors, order, coeffs, stream=None):
    _check(_lib.rc_fit(_ptr(x), _ptr(y), bands, points, detectors, order, _ptr(coeffs),
                       _stream(stream)), "rc_fit")


def rc_demosaic(raw, images, height, width, rgb, stream=None):
    _check(_lib.rc_demosaic(_ptr(raw), images, height, width, _ptr(rgb), _stream(stream)),
           "rc_demosaic")


def rc_demosaic_gradient(raw, images, height, width, rgb, stream=None):
    _check(_lib.rc_demosaic_gradient(_ptr(raw), images, height, width, _ptr(rgb),
                                     _stream(stream)), "rc_demosaic_gradient")


def rc_correct(dn, lut, lines, detectors, bands, levels, out, stream=None):
    _check(_lib.rc_correct(_ptr(dn), _ptr(lut), lines, detectors, bands, levels, _ptr(out),
                           _stream(stream)), "rc_correct")


def rc_correct_ws_bytes(detectors, bands, levels):
    """Workspace bytes rc_correct_ws needs (0: it uses none for this shape)."""
    return int(_lib.rc_correct_ws_bytes(detectors, bands, levels))


def rc_correct_ws(dn, lut, lines, detectors, bands, levels, out, ws, ws_bytes, plan=None,
                  stream=None):
    _check(_lib.rc_correct_ws(_ptr(dn), _ptr(lut), lines, detectors, bands, levels, _ptr(out),
                              _ptr(ws), ws_bytes, ctypes.byref(plan) if plan is not None else None,
                              _stream(stream)), "rc_correct_ws")


def rc_lut_build_ws(coeffs, bands, detectors, levels, lut, ws, ws_bytes, stream=None):
    """rc_lut_build that also leaves the LUT's dense encoding in ws (see rc.h)."""
    _check(_lib.rc_lut_build_ws(_ptr(coeffs), bands, detectors, levels, _ptr(lut), _ptr(ws),
                                ws_bytes, _stream(stream)), "rc_lut_build_ws")


def rc_correct_pre(dn, lut, lines, detectors, bands, levels, out, ws, ws_bytes, plan=None,
                   stream=None):
    """rc_correct_ws with ws already holding the LUT's encoding (see rc.h)."""
    _check(_lib.rc_correct_pre(_ptr(dn), _ptr(lut), lines, detectors, bands, levels, _ptr(out),
                               _ptr(ws), ws_bytes, ctypes.byref(plan) if plan is not None else None,
                               _stream(stream)), "rc_correct_pre")


def rc_correct_noalloc(dn, lut, lines, detectors, bands, levels, out, stream=None):
    """rc_correct_ws with the library's scratch (allocates nothing; see rc.h)."""
    _check(_lib.rc_correct_noalloc(_ptr(dn), _ptr(lut), lines, detectors, bands, levels,
                                   _ptr(out), _stream(stream)), "rc_correct_noalloc")


def rc_stream_copy(src, dst, nbytes, plan=None, stream=None):
    """Plain device copy of nbytes (the streaming ceiling; see rc.h)."""
    _check(_lib.rc_stream_copy(_ptr(src), _ptr(dst), nbytes,
                               ctypes.byref(plan) if plan is not None else None, _stream(stream)),
           "rc_stream_copy")


def rc_correct_plan(dn, lut, lines, detectors, bands, levels, out, plan, stream=None):
    _check(_lib.rc_correct_plan(_ptr(dn), _ptr(lut), lines, detectors, bands, levels, _ptr(out),
                                ctypes.byref(plan), _stream(stream)), "rc_correct_plan")


def rc_plan_for(lines, detectors, bands, levels, dn=None, out=None):
    """(Plan, tuned?) that rc_correct would use for this shape and these pointers."""
    p = Plan()
    src = _i32(0)
    _check(_lib.rc_plan_for(lines, detectors, bands, levels, _ptr(dn), _ptr(out), ctypes.byref(p),
                            ctypes.byref(src)), "rc_plan_for")
    return p, bool(src.value)


def rc_tune(dn, lut, lines, detectors, bands, levels, out, effort=0, stream=None):
    """Autotune the correction plan for this shape; returns (Plan, microseconds)."""
    p = Plan()
    us = ctypes.c_float(0)
    _check(_lib.rc_tune(_ptr(dn), _ptr(lut), lines, detectors, bands, levels, _ptr(out), effort,
                        ctypes.byref(p), ctypes.byref(us), _stream(stream)), "rc_tune")
    return p, float(us.value)


def rc_tune_save(path=None):
    n = _lib.rc_tune_save(path.encode() if path else None)
    if n < 0:
        raise OSError(f"rc_tune_save failed for {path!r}")
    return n


def rc_tune_load(path=None):
    return _lib.rc_tune_load(path.encode() if path else None)


def rc_tune_clear():
    _lib.rc_tune_clear()


def rc_tune_count():
    return _lib.rc_tune_count()


def rc_batch_create(reqs, flags=0):
    """reqs: sequence of Request. Returns an opaque handle (int)."""
    arr = (Request * len(reqs))(*reqs)
    h = _vp()
    _check(_lib.rc_batch_create(arr, len(reqs), flags, ctypes.byref(h)), "rc_batch_create")
    return h.value


def rc_batch_tune(reqs, effort=0, stream=None):
    """Tunes the batch tile shape of every class among reqs (sequence of
    Request) into the plan cache; returns the number of classes tuned."""
    arr = (Request * len(reqs))(*reqs)
    n = _i32(0)
    _check(_lib.rc_batch_tune(arr, len(reqs), effort, ctypes.byref(n), _stream(stream)),
           "rc_batch_tune")
    return n.value


def rc_batch_run(handle, stream=None):
    _check(_lib.rc_batch_run(handle, _stream(stream)), "rc_batch_run")


def rc_batch_info(handle):
    st = BatchStats()
    _check(_lib.rc_batch_info(handle, ctypes.byref(st)), "rc_batch_info")
    return st.as_dict()


def rc_batch_destroy(handle):
    _lib.rc_batch_destroy(handle)


def batch_requests(jobs):
    """Request structs for jobs = [(coeffs, dn, lut, out)] of device tensors
    (coeffs [B, D, 4] float64, dn/out [B, N, D] 16-bit, lut [B, D, L] 16-bit)."""
    reqs = []
    for c, dn, lut, out in jobs:
        B, N, D = dn.shape
        assert tuple(c.shape) == (B, D, 4) and tuple(lut.shape[:2]) == (B, D)
        assert tuple(out.shape) == (B, N, D)
        reqs.append(Request(_ptr(c), _ptr(dn), _ptr(lut), _ptr(out), N, D, B, lut.shape[2], 0))
    return reqs


def batch_tune(jobs, effort=0, stream=None):
    """rc_batch_tune over jobs as Batch takes them; returns the classes tuned."""
    return rc_batch_tune(batch_requests(jobs), effort, stream)


class Batch:
    """Owns an rc_batch over device tensors: jobs = [(coeffs, dn, lut, out)], each
    coeffs [B, D, 4] float64, dn/out [B, N, D] 16-bit, lut [B, D, L] 16-bit."""

    def __init__(self, jobs, graph=True):
        self.jobs = list(jobs)  # keeps the tensors alive
        self.handle = rc_batch_create(batch_requests(self.jobs),
                                      0 if graph else RC_BATCH_NO_GRAPH)

    def run(self, stream=None):
        rc_batch_run(self.handle, stream)

    def info(self):
        return rc_batch_info(self.handle)

    def close(self):
        if self.handle:
            rc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host_ptr(x):
    """Address of a host buffer: numpy array, CPU tensor or int."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, torch.Tensor):
        if x.is_cuda or not x.is_contiguous():
            raise ValueError("expected a contiguous host tensor")
        return x.data_ptr() if x.numel() else None
    if not x.flags.c_contiguous:
        raise ValueError("expected a C-contiguous array")
    return x.ctypes.data if x.size else None


def pinned_empty(shape, dtype):
    """A numpy array in pinned host memory (backed by a pinned torch tensor)."""
    import numpy as np
    tdtype = {np.dtype(np.uint16): torch.int16, np.dtype(np.int16): torch.int16,
              np.dtype(np.float64): torch.float64}[np.dtype(dtype)]
    t = torch.empty(shape, dtype=tdtype, pin_memory=True)
    return t.numpy().view(dtype)


class Server:
    """In-process serving runtime (rc_server): submit host jobs, wait for them."""

    def __init__(self, arena_bytes=0, max_jobs=0, max_quantum_tiles=0, piece_pixels=0):
        opts = ServerOpts(arena_bytes, max_jobs, max_quantum_tiles, piece_pixels, 0, 0)
        h = _vp()
        _check(_lib.rc_server_create(ctypes.byref(opts), ctypes.byref(h)), "rc_server_create")
        self.handle = h.value
        self._keep = {}

    def submit(self, coeffs, dn, out, levels, lut=None):
        """coeffs [B, D, 4] float64, dn/out [B, N, D] uint16 host arrays (pinned
        preferred), optional lut [B, D, L] uint16. Returns the job id."""
        B, N, D = dn.shape
        job = HostJob(_host_ptr(coeffs), _host_ptr(dn), _host_ptr(out), _host_ptr(lut), N, D, B,
                      levels, 0)
        jid = ctypes.c_uint64(0)
        _check(_lib.rc_server_submit(self.handle, ctypes.byref(job), ctypes.byref(jid)),
               "rc_server_submit")
        self._keep[jid.value] = (coeffs, dn, out, lut)
        return jid.value

    def wait(self, job_id):
        st = JobStats()
        status = _lib.rc_server_wait(self.handle, job_id, ctypes.byref(st))
        self._keep.pop(job_id, None)
        d = st.as_dict()
        d["status"] = status
        return d

    def poll(self, job_id):
        st = JobStats()
        status = _lib.rc_server_poll(self.handle, job_id, ctypes.byref(st))
        if status == RC_EBUSY:
            return None
        self._keep.pop(job_id, None)
        d = st.as_dict()
        d["status"] = status
        return d

    def info(self):
        st = ServerStats()
        _check(_lib.rc_server_info(self.handle, ctypes.byref(st)), "rc_server_info")
        return st.as_dict()

    def close(self):
        if self.handle:
            _lib.rc_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --- shape-checked conveniences -------------------------------------------------------------

def _u16(t):
    return t.dtype in (torch.int16, getattr(torch, "uint16", torch.int16))


def lut_build(coeffs, levels, lut=None, stream=None):
    """coeffs: float64 device tensor [B, D, 4] -> LUT int16/uint16 device tensor [B, D, L]."""
    if coeffs.dtype != torch.float64 or coeffs.dim() != 3 or coeffs.shape[2] != RC_NCOEF:
        raise ValueError("coeffs must be float64 [bands, detectors, 4]")
    B, D, _ = coeffs.shape
    if lut is None:
        lut = torch.empty((B, D, levels), dtype=torch.int16, device=coeffs.device)
    if not _u16(lut) or tuple(lut.shape) != (B, D, levels):
        raise ValueError("lut must be 16-bit [bands, detectors, levels]")
    rc_lut_build(coeffs, B, D, levels, lut, stream)
    return lut


def fit(x, y, order, out=None, stream=None):
    """x: float64 device tensor [B, n, D] (detector responses on n calibration
    lines), y: [B, n] (the lines' reference levels) -> coefficients [B, D, 4],
    the layout lut_build takes."""
    if x.dtype != torch.float64 or y.dtype != torch.float64 or x.dim() != 3 or y.dim() != 2:
        raise ValueError("x [B, n, D] and y [B, n] must be float64 tensors")
    B, n, D = x.shape
    if tuple(y.shape) != (B, n):
        raise ValueError("y shape does not match x")
    if out is None:
        out = torch.empty((B, D, 4), dtype=torch.float64, device=x.device)
    rc_fit(x.contiguous(), y.contiguous(), B, n, D, order, out, stream)
    return out


def demosaic(raw, out=None, stream=None, method="bilinear"):
    """raw: 16-bit device tensor [I, H, W] (RGGB) -> [I, 3, H, W] R, G, B planes.
    method: "bilinear" (rc_demosaic) or "gradient" (rc_demosaic_gradient)."""
    if method not in ("bilinear", "gradient"):
        raise ValueError("method must be 'bilinear' or 'gradient'")
    if not _u16(raw) or raw.dim() != 3:
        raise ValueError("raw must be a 16-bit tensor [images, height, width]")
    I, H, W = raw.shape
    if out is None:
        out = torch.empty((I, 3, H, W), dtype=raw.dtype, device=raw.device)
    if not _u16(out) or tuple(out.shape) != (I, 3, H, W):
        raise ValueError("out must be a 16-bit tensor [images, 3, height, width]")
    call = rc_demosaic if method == "bilinear" else rc_demosaic_gradient
    call(raw, I, H, W, out, stream)
    return out


def correct(dn, lut, out=None, plan=None, stream=None):
    """dn: 16-bit device tensor [B, N, D]; lut: [B, D, L] -> out [B, N, D]."""
    if not _u16(dn) or not _u16(lut) or dn.dim() != 3 or lut.dim() != 3:
        raise ValueError("dn [B, N, D] and lut [B, D, L] must be 16-bit tensors")
    B, N, D = dn.shape
    if tuple(lut.shape[:2]) != (B, D):
        raise ValueError("lut shape does not match dn")
    L = lut.shape[2]
    if out is None:
        out = torch.empty_like(dn)
    if tuple(out.shape) != tuple(dn.shape) or not _u16(out):
        raise ValueError("out must match dn")
    if plan is None:
        rc_correct(dn, lut, N, D, B, L, out, stream)
    else:
        rc_correct_plan(dn, lut, N, D, B, L, out, plan, stream)
    return out
