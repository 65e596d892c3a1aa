"""The wire front end end to end over loopback TCP: every task's answer equals
the oracle (bit for bit), several requests share one connection, concurrent
clients' correction jobs go through the batching server together, and a
malformed header is answered with RC_EINVAL."""
import socket
import threading
import xml.etree.ElementTree as ET

import numpy as np
import pytest
import torch

import gen
import oracle
from paper_1505_05655_amd import wire

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def server():
    torch.cuda.set_device(0)
    with wire.WireServer(port=0, arena_bytes=1 << 30) as srv:
        yield srv


@pytest.fixture(scope="module")
def o():
    return oracle.get()


def correction_case(seed, B=2, N=300, D=520, L=1024):
    coeffs = gen.coeffs(gen.BASE_SEED, 60, seed, gen.COEF_QUADRATIC, B, D)
    dn = gen.dn(gen.BASE_SEED, 60, seed, gen.DN_GAUSS_SAT10, B, N, D)
    params = {"bands": B, "lines": N, "detectors": D, "levels": L, "lut": 1}
    return params, coeffs.tobytes() + dn.tobytes(), coeffs, dn


def check_correction(o, params, coeffs, dn, h, res):
    assert h["params"]["status"] == "RC_OK", h
    B, N, D, L = params["bands"], params["lines"], params["detectors"], params["levels"]
    out = np.frombuffer(res[:B * N * D * 2], np.uint16).reshape(B, N, D)
    lut = np.frombuffer(res[B * N * D * 2:], np.uint16).reshape(B, D, L)
    want_lut = o.lut_build(coeffs, L)
    assert np.array_equal(lut, want_lut)
    assert np.array_equal(out, o.correct(dn, want_lut))


def test_gpu_info(server):
    h, res = wire.request("127.0.0.1", server.port, "GPU_INFO", out_name="gpus.xml")
    assert h["params"]["status"] == "RC_OK" and h["out_name"] == "gpus.xml"
    root = ET.fromstring(res.decode())
    gpu = root.find("gpu")
    assert int(gpu.find("multiprocessor_count").text) > 0
    assert int(gpu.find("wavefront_size").text) == 64
    assert int(gpu.find("total_global_memory").text) > 0


def test_correction(server, o):
    params, data, coeffs, dn = correction_case(0)
    h, res = wire.request("127.0.0.1", server.port, "LUT_CORRECTION", params, data, "out.u16")
    check_correction(o, params, coeffs, dn, h, res)


def test_demosaic_and_fit_on_one_connection(server, o):
    raw = gen.bayer(gen.BASE_SEED, 61, 0, 1, 66, 260)
    x, y = gen.calib(gen.BASE_SEED, 61, 0, 2, 6, 300, 1024)
    with socket.create_connection(("127.0.0.1", server.port), timeout=120) as s:
        for _ in range(2):
            h, res = wire.exchange(s, "BILINEAR_DEMOSAIC", {"images": 1, "height": 66, "width": 260},
                                   raw.tobytes(), "rgb.u16")
            assert h["params"]["status"] == "RC_OK"
            rgb = np.frombuffer(res, np.uint16).reshape(1, 3, 66, 260)
            assert np.array_equal(rgb, o.demosaic(raw))
            h, res = wire.exchange(s, "GRADIENT_DEMOSAIC", {"images": 1, "height": 66, "width": 260},
                                   raw.tobytes(), "rgb.u16")
            assert h["params"]["status"] == "RC_OK"
            rgb = np.frombuffer(res, np.uint16).reshape(1, 3, 66, 260)
            assert np.array_equal(rgb, o.demosaic_gradient(raw))
            h, res = wire.exchange(s, "LSQ_FIT", {"bands": 2, "points": 6, "detectors": 300,
                                                  "order": 2}, x.tobytes() + y.tobytes(), "c.f64")
            assert h["params"]["status"] == "RC_OK"
            got = np.frombuffer(res, np.float64).reshape(2, 300, 4)
            assert np.array_equal(got.view(np.uint64), o.fit(x, y, 2).view(np.uint64))


def test_concurrent_clients(server, o):
    cases = [correction_case(10 + k, N=200 + 37 * k) for k in range(4)]
    answers = [None] * len(cases)

    def client(k):
        params, data, _, _ = cases[k]
        answers[k] = wire.request("127.0.0.1", server.port, "LUT_CORRECTION", params, data, "o")

    threads = [threading.Thread(target=client, args=(k,)) for k in range(len(cases))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    for (params, _, coeffs, dn), (h, res) in zip(cases, answers):
        check_correction(o, params, coeffs, dn, h, res)


def test_many_short_connections(server):
    """Connections come and go; the server keeps answering (finished
    connection threads are joined while it runs)."""
    for _ in range(40):
        h, res = wire.request("127.0.0.1", server.port, "GPU_INFO")
        assert h["params"]["status"] == "RC_OK" and res.startswith(b"<")


def test_malformed_header_is_refused(server):
    with socket.create_connection(("127.0.0.1", server.port), timeout=60) as s:
        s.sendall(wire.encode_header("LUT_GENERATION", "bands=1", "x", has_data=True))
        h = wire.decode_header(wire._recv_exact(s, wire.HEADER_BYTES))
        assert h["params"]["status"] == "RC_EINVAL" and not h["has_data"]
        assert s.recv(1) == b""  # the server closed the connection


def test_size_limit_covers_answers(o):
    """max_data_bytes bounds both the data a request carries and the answer it
    asks for (a LUT answer can be far larger than its coefficients); a refused
    request closes its connection and the server goes on answering."""
    with wire.WireServer(port=0, max_data_bytes=64 << 10, arena_bytes=1 << 28) as srv:
        big_answer = {"bands": 1, "lines": 1, "detectors": 64, "levels": 4096, "lut": 1}
        big_input = {"images": 1, "height": 256, "width": 256}
        for task, params in (("LUT_CORRECTION", big_answer), ("BILINEAR_DEMOSAIC", big_input)):
            with socket.create_connection(("127.0.0.1", srv.port), timeout=60) as s:
                s.sendall(wire.encode_header(task, params, "x", has_data=True))
                h = wire.decode_header(wire._recv_exact(s, wire.HEADER_BYTES))
                assert h["params"]["status"] == "RC_ENOMEM" and not h["has_data"], task
                assert s.recv(1) == b""
        params, data, coeffs, dn = correction_case(3, B=1, N=8, D=64, L=256)
        h, res = wire.request("127.0.0.1", srv.port, "LUT_CORRECTION", params, data, "out.u16")
        check_correction(o, params, coeffs, dn, h, res)


def test_stop_with_idle_connection():
    with wire.WireServer(port=0) as srv:
        s = socket.create_connection(("127.0.0.1", srv.port), timeout=60)
        h, _ = wire.exchange(s, "GPU_INFO")
        assert h["params"]["status"] == "RC_OK"
    # the server stopped while the connection was open and idle
    assert s.recv(1) == b""
    s.close()
