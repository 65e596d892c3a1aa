"""Client side of the paper's client-server framework (§II, header template of
Fig. 3), and a handle on the library's TCP server.

A request is a 260-byte header followed by the input data:

    [0, 29)    task flag ("LUT_CORRECTION", "BILINEAR_DEMOSAIC", "GRADIENT_DEMOSAIC", "LSQ_FIT",
               "GPU_INFO")
    [29]       b"+" when data follows, b"\\0" when none does
    [30, 230)  comma-separated parameters, key=value
    [230, 260) output file name

The answer has the same layout; its parameters read "status=<name>,bytes=<n>"
and n bytes of result follow. Data layouts are those of the C calls (see
include/rc.h). Command line:

    python -m paper_1505_05655_amd.wire serve --port 5050
    python -m paper_1505_05655_amd.wire send --server 127.0.0.1:5050 --task GPU_INFO --out gpus.xml
    python -m paper_1505_05655_amd.wire send --server 127.0.0.1:5050 --task BILINEAR_DEMOSAIC \\
        --params images=1,height=2048,width=2048 --in raw.u16 --out rgb.u16
"""
import argparse
import ctypes
import socket
import sys
import time

HEADER_BYTES = 260
TASK_LEN, FLAG_OFF, PARAM_OFF, PARAM_LEN, OUT_OFF, OUT_LEN = 29, 29, 30, 200, 230, 30
TASKS = ("LUT_CORRECTION", "BILINEAR_DEMOSAIC", "LSQ_FIT", "GPU_INFO", "GRADIENT_DEMOSAIC")


def _pad(text, n, what):
    b = text.encode("ascii")
    if len(b) > n or b"\0" in b:
        raise ValueError(f"{what} must be at most {n} ASCII characters: {text!r}")
    return b + b"\0" * (n - len(b))


def encode_header(task, params=None, out_name="", has_data=False):
    """The 260-byte header; params is a dict of integers (kept in order) or a string."""
    if isinstance(params, dict):
        params = ",".join(f"{k}={int(v)}" for k, v in params.items())
    return (_pad(task, TASK_LEN, "task flag") + (b"+" if has_data else b"\0") +
            _pad(params or "", PARAM_LEN, "parameter string") +
            _pad(out_name, OUT_LEN, "output file name"))


def decode_header(h):
    """The fields of a header: task, has_data, params (dict of int), out_name."""
    if len(h) != HEADER_BYTES:
        raise ValueError("a header is 260 bytes")
    field = lambda a, n: h[a:a + n].split(b"\0", 1)[0].decode("ascii")
    params = {}
    text = field(PARAM_OFF, PARAM_LEN)
    for kv in filter(None, text.split(",")):
        k, v = kv.split("=", 1)
        params[k] = int(v) if v.isdigit() else v
    return {"task": field(0, TASK_LEN), "has_data": h[FLAG_OFF:FLAG_OFF + 1] == b"+",
            "params": params, "out_name": field(OUT_OFF, OUT_LEN)}


def _recv_exact(sock, n):
    buf = bytearray(n)
    view = memoryview(buf)
    got = 0
    while got < n:
        k = sock.recv_into(view[got:], n - got)
        if k == 0:
            raise ConnectionError("connection closed by the server")
        got += k
    return bytes(buf)


def exchange(sock, task, params=None, data=b"", out_name=""):
    """One request on an open connection: returns (answer header fields, result bytes)."""
    sock.sendall(encode_header(task, params, out_name, has_data=len(data) > 0))
    if len(data):
        sock.sendall(data)
    h = decode_header(_recv_exact(sock, HEADER_BYTES))
    n = int(h["params"].get("bytes", 0)) if h["has_data"] else 0
    return h, _recv_exact(sock, n) if n else b""


def request(host, port, task, params=None, data=b"", out_name="", timeout=120.0):
    """Connect, send one request, return (answer header fields, result bytes)."""
    with socket.create_connection((host, port), timeout=timeout) as s:
        return exchange(s, task, params, data, out_name)


class WireServer:
    """The library's TCP server (rc_wire_start / rc_wire_stop) on the current device."""

    def __init__(self, port=0, any_address=False, max_data_bytes=0, arena_bytes=0):
        from . import RcError, lib
        self._lib = lib()
        self._lib.rc_wire_start.argtypes = [ctypes.POINTER(WireOpts), ctypes.POINTER(ctypes.c_void_p)]
        self._lib.rc_wire_start.restype = ctypes.c_int
        self._lib.rc_wire_port.argtypes = [ctypes.c_void_p]
        self._lib.rc_wire_port.restype = ctypes.c_int32
        self._lib.rc_wire_stop.argtypes = [ctypes.c_void_p]
        self._lib.rc_wire_stop.restype = None
        opts = WireOpts(port, 1 if any_address else 0, max_data_bytes, arena_bytes)
        h = ctypes.c_void_p()
        st = self._lib.rc_wire_start(ctypes.byref(opts), ctypes.byref(h))
        if st != 0:
            raise RcError(st, "rc_wire_start")
        self.handle = h

    @property
    def port(self):
        return self._lib.rc_wire_port(self.handle)

    def close(self):
        if self.handle:
            self._lib.rc_wire_stop(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class WireOpts(ctypes.Structure):
    """Mirrors rc_wire_opts."""
    _fields_ = [("port", ctypes.c_int32), ("any_address", ctypes.c_int32),
                ("max_data_bytes", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64)]


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1505_05655_amd.wire")
    sub = ap.add_subparsers(dest="cmd", required=True)
    sv = sub.add_parser("serve", help="run the GPU server until interrupted")
    sv.add_argument("--port", type=int, default=5050)
    sv.add_argument("--any-address", action="store_true", help="listen on every interface")
    sd = sub.add_parser("send", help="send one task; the result is written to --out")
    sd.add_argument("--server", default="127.0.0.1:5050", help="host:port")
    sd.add_argument("--task", required=True, choices=TASKS)
    sd.add_argument("--params", default="", help="comma-separated key=value list")
    sd.add_argument("--in", dest="inp", default=None, help="input data file (raw bytes)")
    sd.add_argument("--out", required=True, help="output file name")
    a = ap.parse_args(argv)
    if a.cmd == "serve":
        with WireServer(port=a.port, any_address=a.any_address) as srv:
            print(f"listening on port {srv.port}", flush=True)
            try:
                while True:
                    time.sleep(1)
            except KeyboardInterrupt:
                pass
        return 0
    host, port = a.server.rsplit(":", 1)
    data = open(a.inp, "rb").read() if a.inp else b""
    h, res = request(host, int(port), a.task, a.params, data, out_name=a.out[-OUT_LEN:])
    status = h["params"].get("status")
    if status != "RC_OK":
        print(f"{a.task}: {status}", file=sys.stderr)
        return 1
    with open(a.out, "wb") as fh:
        fh.write(res)
    print(f"{a.task}: {len(res)} bytes -> {a.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
