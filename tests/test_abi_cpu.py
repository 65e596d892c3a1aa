"""The C-ABI library loads, exports every function include/rc.h declares, and
rejects bad arguments on the host before touching the GPU. CPU only: no
compute call is made here."""
import ctypes
import os
import re

import pytest

import paper_1505_05655_amd as rc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        for m in re.finditer(r"\b(rc_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("rc_lut_build", "rc_correct", "rc_status_str", "rc_last_hip_error"):
        assert must in names


@pytest.mark.parametrize("name", declared_functions())
def test_symbol_exported(name):
    assert hasattr(rc.lib(), name), f"librc.so does not export {name}"


def test_status_strings():
    lib = rc.lib()
    for s in range(6):
        assert lib.rc_status_str(s).startswith(b"RC_")


L = rc.lib()
FAKE = 0x10000  # never dereferenced: every call below fails validation first


@pytest.mark.parametrize("args", [
    (None, 1, 1, 1024, FAKE),            # NULL coeffs
    (FAKE, 1, 1, 1024, None),            # NULL lut
    (FAKE, -1, 1, 1024, FAKE),           # negative bands
    (FAKE, 1, -5, 1024, FAKE),           # negative detectors
    (FAKE, 1, 1, 1, FAKE),               # levels < 2
    (FAKE, 1, 1, 65537, FAKE),           # levels > 65536
    (FAKE + 4, 1, 1, 1024, FAKE + 64),   # coeffs not 8-byte aligned
    (FAKE, 1, 1, 1024, FAKE + 4097),     # lut not 2-byte aligned
    (FAKE, 1, 1, 1024, FAKE + 16),       # lut overlaps coeffs
    (FAKE, 1 << 30, 1 << 30, 1024, FAKE * 4),  # byte count overflows
])
def test_lut_build_rejects(args):
    assert L.rc_lut_build(*args, None) == rc.RC_EINVAL


def test_lut_build_empty_is_noop():
    assert L.rc_lut_build(None, 0, 5, 1024, None, None) == rc.RC_OK
    assert L.rc_lut_build(None, 3, 0, 1024, None, None) == rc.RC_OK


WS4096 = 3 * 64 * 6000 * 10  # rc_correct_ws_bytes(6000, 3, 4096)
WSA = FAKE * 4096  # past the 147 MB LUT at FAKE * 64 and the coefficients at FAKE


@pytest.mark.parametrize("args", [
    (FAKE, 3, 6000, 1024, FAKE * 64, WSA, WS4096),      # levels below the workspace range
    (FAKE, 3, 6000, 8256, FAKE * 64, WSA, WS4096),      # levels above it
    (None, 3, 6000, 4096, FAKE * 64, WSA, WS4096),      # NULL coeffs
    (FAKE, 3, 6000, 4096, None, WSA, WS4096),           # NULL lut
    (FAKE, 3, 6000, 4096, FAKE * 64, None, WS4096),             # NULL workspace
    (FAKE, 3, 6000, 4096, FAKE * 64, WSA + 16, WS4096),  # workspace not 256-byte aligned
    (FAKE, 3, 6000, 4096, FAKE * 64, WSA, WS4096 - 1),  # workspace too short
    (FAKE, 3, 6000, 4096, FAKE * 64, FAKE * 64, WS4096),        # workspace overlaps the LUT
    (FAKE, -3, 6000, 4096, FAKE * 64, WSA, WS4096),     # negative bands
])
def test_lut_build_ws_rejects(args):
    assert L.rc_lut_build_ws(*args, None) == rc.RC_EINVAL


def test_correct_pre_rejects():
    """Levels outside the workspace range, and a missing workspace."""
    assert L.rc_correct_pre(FAKE, FAKE * 64, 4, 4, 1, 1024, FAKE * 128, FAKE * 1024, 1 << 20,
                            None, None) == rc.RC_EINVAL
    assert L.rc_correct_pre(FAKE, FAKE * 64, 4, 4, 1, 4096, FAKE * 128, None, 1 << 20,
                            None, None) == rc.RC_EINVAL


BIG = 1 << 24


@pytest.mark.parametrize("args", [
    (None, FAKE, 4, 4, 1, 1024, FAKE * 64),         # NULL dn
    (FAKE, None, 4, 4, 1, 1024, FAKE * 64),         # NULL lut
    (FAKE, FAKE * 64, 4, 4, 1, 1024, None),         # NULL out
    (FAKE, FAKE * 64, -1, 4, 1, 1024, FAKE * 128),  # negative lines
    (FAKE, FAKE * 64, 4, -4, 1, 1024, FAKE * 128),  # negative detectors
    (FAKE, FAKE * 64, 4, 4, -1, 1024, FAKE * 128),  # negative bands
    (FAKE, FAKE * 64, 4, 4, 1, 1, FAKE * 128),      # levels < 2
    (FAKE, FAKE * 64, 4, 4, 1, 70000, FAKE * 128),  # levels > 65536
    (FAKE + 1, FAKE * 64, 4, 4, 1, 1024, FAKE * 128),   # dn odd address
    (FAKE, FAKE * 64, 4, 4, 1, 1024, FAKE * 128 + 1),   # out odd address
    (FAKE, FAKE * 64, 4, 4, 1, 1024, FAKE + 2),     # out partially overlaps dn
    (FAKE, FAKE * 64, 4, 4, 1, 1024, FAKE * 64 + 8),  # out overlaps lut
    (FAKE, FAKE * 64, 1 << 40, 1 << 30, 4, 1024, FAKE * 128),  # pixel count overflows
])
def test_correct_rejects(args):
    assert L.rc_correct(*args, None) == rc.RC_EINVAL


def test_correct_empty_is_noop():
    assert L.rc_correct(None, None, 0, 100, 2, 1024, None, None) == rc.RC_OK
    assert L.rc_correct(None, None, 10, 0, 2, 1024, None, None) == rc.RC_OK
    assert L.rc_correct(None, None, 10, 100, 0, 1024, None, None) == rc.RC_OK


@pytest.mark.parametrize("args", [
    # x, y, bands, points, detectors, order, coeffs
    (None, FAKE, 1, 6, 4, 2, FAKE * 64),               # NULL x
    (FAKE, None, 1, 6, 4, 2, FAKE * 64),               # NULL y
    (FAKE, FAKE * 32, 1, 6, 4, 2, None),               # NULL coeffs
    (FAKE, FAKE * 32, 1, 6, 4, -1, FAKE * 64),         # order < 0
    (FAKE, FAKE * 32, 1, 6, 4, 4, FAKE * 64),          # order > 3
    (FAKE, FAKE * 32, 1, 2, 4, 2, FAKE * 64),          # points < order + 1
    (FAKE, FAKE * 32, -1, 6, 4, 2, FAKE * 64),         # negative bands
    (FAKE, FAKE * 32, 1, 6, -4, 2, FAKE * 64),         # negative detectors
    (FAKE + 4, FAKE * 32, 1, 6, 4, 2, FAKE * 64),      # x not 8-byte aligned
    (FAKE, FAKE * 32 + 2, 1, 6, 4, 2, FAKE * 64),      # y not 8-byte aligned
    (FAKE, FAKE * 32, 1, 6, 4, 2, FAKE * 64 + 4),      # coeffs not 8-byte aligned
    (FAKE, FAKE * 32, 1, 6, 4, 2, FAKE + 64),          # coeffs overlap x
    (FAKE, FAKE * 32, 1, 6, 4, 2, FAKE * 32 + 8),      # coeffs overlap y
    (FAKE, FAKE * 32, 1 << 20, 1 << 20, 1 << 20, 1, FAKE * 64),  # sizes overflow
])
def test_fit_rejects(args):
    assert L.rc_fit(*args, None) == rc.RC_EINVAL


def test_fit_empty_is_noop():
    assert L.rc_fit(None, None, 0, 6, 100, 2, None, None) == rc.RC_OK
    assert L.rc_fit(None, None, 3, 6, 0, 2, None, None) == rc.RC_OK


@pytest.mark.parametrize("args", [
    # raw, images, height, width, rgb
    (None, 1, 4, 8, FAKE * 64),            # NULL raw
    (FAKE, 1, 4, 8, None),                 # NULL rgb
    (FAKE, -1, 4, 8, FAKE * 64),           # negative images
    (FAKE, 1, -4, 8, FAKE * 64),           # negative height
    (FAKE, 1, 3, 8, FAKE * 64),            # odd height
    (FAKE, 1, 4, 6, FAKE * 64),            # width not a multiple of 4
    (FAKE + 2, 1, 4, 8, FAKE * 64),        # raw not 8-byte aligned
    (FAKE, 1, 4, 8, FAKE * 64 + 4),        # rgb not 8-byte aligned
    (FAKE, 1, 4, 8, FAKE + 32),            # rgb overlaps raw
    (FAKE, 1 << 20, 1 << 20, 1 << 20, FAKE * 64),  # sizes overflow
])
def test_demosaic_rejects(args):
    assert L.rc_demosaic(*args, None) == rc.RC_EINVAL


def test_demosaic_empty_is_noop():
    assert L.rc_demosaic(None, 0, 4, 8, None, None) == rc.RC_OK
    assert L.rc_demosaic(None, 2, 0, 8, None, None) == rc.RC_OK


def test_correct_plan_requires_plan():
    assert L.rc_correct_plan(FAKE, FAKE * 64, 4, 4, 1, 1024, FAKE * 128, None, None) == rc.RC_EINVAL


def _req(coeffs, dn, lut, out, lines=4, det=4, bands=1, levels=1024, reserved=0):
    return rc.Request(coeffs, dn, lut, out, lines, det, bands, levels, reserved)


# Request buffers (never dereferenced): coeffs 128 B at C, lut 8 KiB at T,
# dn/out 32 B at I/O, second request shifted by S.
C, T, I, O, S = 0x100000, 0x200000, 0x300000, 0x400000, 0x1000000


@pytest.mark.parametrize("reqs", [
    [_req(C, I, T, O, reserved=1)],                       # reserved field set
    [_req(None, I, T, O)],                                # NULL coeffs
    [_req(C, I, T, O, levels=1)],                         # bad levels
    [_req(C, I, T, O, lines=-1)],                         # negative lines
    [_req(C, I, T, I + 2)],                               # out partially overlaps dn
    [_req(C, I, C + 8, O)],                               # lut overlaps coeffs
    [_req(C, T, T, O)],                                   # lut overlaps dn
    [_req(C, I, T, O), _req(C + S, I + S, T + S, O)],     # two requests write one out
    [_req(C, I, T, O), _req(C + S, O, T + S, O + S)],     # output of one is input of another
    [_req(C, I, T, O), _req(C + S, I + S, T, O + S)],     # shared LUT written twice
    [_req(C, I, T, C)],                                   # out is its own coeffs
    [_req(C, I, T, C + 64)],                              # out overlaps its own coeffs
    [_req(C, I, T, T + 16)],                              # out overlaps its own LUT
])
def test_batch_rejects(reqs):
    arr = (rc.Request * len(reqs))(*reqs)
    h = ctypes.c_void_p()
    assert L.rc_batch_create(arr, len(reqs), 0, ctypes.byref(h)) == rc.RC_EINVAL
    assert not h.value
    # The tuner validates the same way, before it touches the device.
    n = ctypes.c_int32(-1)
    assert L.rc_batch_tune(arr, len(reqs), 0, ctypes.byref(n), None) == rc.RC_EINVAL
    assert n.value == 0


def test_batch_null_args():
    h = ctypes.c_void_p()
    assert L.rc_batch_tune(None, 3, 0, None, None) == rc.RC_EINVAL
    assert L.rc_batch_create(None, 3, 0, ctypes.byref(h)) == rc.RC_EINVAL
    assert L.rc_batch_create(None, -1, 0, ctypes.byref(h)) == rc.RC_EINVAL
    assert L.rc_batch_run(None, None) == rc.RC_EINVAL
    L.rc_batch_destroy(None)


def test_server_argument_checks():
    h = ctypes.c_void_p()
    bad = rc.ServerOpts(0, 0, 0, 0, 0, 7)  # reserved must be 0
    assert L.rc_server_create(ctypes.byref(bad), ctypes.byref(h)) == rc.RC_EINVAL
    bad = rc.ServerOpts(0, -1, 0, 0, 0, 0)
    assert L.rc_server_create(ctypes.byref(bad), ctypes.byref(h)) == rc.RC_EINVAL
    assert L.rc_server_create(None, None) == rc.RC_EINVAL
    jid = ctypes.c_uint64()
    job = rc.HostJob(FAKE, FAKE, FAKE, None, 4, 4, 1, 1024, 0)
    assert L.rc_server_submit(None, ctypes.byref(job), ctypes.byref(jid)) == rc.RC_EINVAL
    assert L.rc_server_wait(None, 1, None) == rc.RC_EINVAL
    assert L.rc_server_poll(None, 1, None) == rc.RC_EINVAL
    L.rc_server_destroy(None)


@pytest.mark.parametrize("args", [
    # raw, images, height, width, rgb
    (None, 1, 4, 8, FAKE * 64),            # NULL raw
    (FAKE, 1, 4, 8, None),                 # NULL rgb
    (FAKE, -1, 4, 8, FAKE * 64),           # negative images
    (FAKE, 1, -4, 8, FAKE * 64),           # negative height
    (FAKE, 1, 5, 8, FAKE * 64),            # odd height
    (FAKE, 1, 2, 8, FAKE * 64),            # height 2: the stencil reaches two rows
    (FAKE, 1, 4, 6, FAKE * 64),            # width not a multiple of 4
    (FAKE + 2, 1, 4, 8, FAKE * 64),        # raw not 8-byte aligned
    (FAKE, 1, 4, 8, FAKE * 64 + 4),        # rgb not 8-byte aligned
    (FAKE, 1, 4, 8, FAKE + 32),            # rgb overlaps raw
    (FAKE, 1 << 20, 1 << 20, 1 << 20, FAKE * 64),  # sizes overflow
])
def test_demosaic_gradient_rejects(args):
    assert L.rc_demosaic_gradient(*args, None) == rc.RC_EINVAL


def test_demosaic_gradient_empty_is_noop():
    assert L.rc_demosaic_gradient(None, 0, 4, 8, None, None) == rc.RC_OK
    assert L.rc_demosaic_gradient(None, 2, 0, 8, None, None) == rc.RC_OK


def test_plan_cache_file_roundtrip(tmp_path):
    """The plan cache file (host only): valid lines load, malformed ones are
    skipped, a save reloads to the same entries, a missing file empties the
    cache."""
    good = ('{"arch":"gfx950","cus":256,"levels":1024,"dclass":14,"nclass":14,"bands":4,'
            '"vmax":4,"path":2,"strip":256,"vec":4,"threads":512,"unroll":4,"chunks":1,'
            '"xcd_remap":1,"nontemporal":2,"us":482.1}')
    lines = [good,
             good.replace('"levels":1024', '"levels":4096'),
             good.replace('"strip":256,', ''),                  # missing key
             good.replace('"cus":256', '"cus":1e300'),          # out of int range
             good.replace('"vec":4', '"vec":nan'),              # not a number
             good.replace('"unroll":4', '"unroll":'),           # no value
             "garbage", ""]
    path = tmp_path / "cache.json"
    path.write_text("\n".join(lines) + "\n")
    try:
        assert rc.rc_tune_load(str(path)) == 2
        assert rc.rc_tune_count() == 2
        saved = tmp_path / "saved.json"
        assert rc.rc_tune_save(str(saved)) == 2
        assert rc.rc_tune_load(str(saved)) == 2
        assert rc.rc_tune_load(str(tmp_path / "missing.json")) == -1
        assert rc.rc_tune_count() == 0
        assert rc.rc_tune_load(str(saved)) == 2
        rc.rc_tune_clear()
        assert rc.rc_tune_count() == 0
    finally:
        rc.rc_tune_load(None)  # back to the packaged cache


def test_ws_bytes_host():
    """Workspace size of rc_correct_ws (host only): 10 bytes per 64-level
    block of every LUT row for 2048 <= levels <= 8192, in 256-byte pieces."""
    assert rc.rc_correct_ws_bytes(6000, 3, 4096) == 3 * 64 * 6000 * 8 + 3 * 64 * 6000 * 2
    assert rc.rc_correct_ws_bytes(7, 1, 2048) == 1792 + 512  # 224 blocks: 1792 B + 448 B -> 512
    assert rc.rc_correct_ws_bytes(100, 2, 1024) == 0
    assert rc.rc_correct_ws_bytes(100, 2, 8193) == 0
    assert rc.rc_correct_ws_bytes(0, 2, 4096) == 0


def test_tune_cache_reads_json_with_spaces(tmp_path):
    """Plan-cache lines may come from any JSON writer (spaces after colons);
    batch entries keep their kind through a save and a reload."""
    import json
    entry = {"arch": "gfx950", "cus": 256, "levels": 4096, "dclass": 12, "nclass": 0,
             "bands": 0, "vmax": 4, "path": rc.RC_PATH_DENSE, "strip": 128, "vec": 4,
             "threads": 1024, "unroll": 4, "chunks": 1, "xcd_remap": 1, "nontemporal": 0,
             "strips": 0, "lane_map": 0, "kind": 1, "us": 12.5}
    src = tmp_path / "in.json"
    src.write_text(json.dumps(entry) + "\n" + json.dumps(dict(entry, kind=7)) + "\n")
    try:
        assert rc.rc_tune_load(str(src)) == 1  # kind 7 is not a valid entry
        out = tmp_path / "out.json"
        assert rc.rc_tune_save(str(out)) == 1
        saved = json.loads(out.read_text().splitlines()[0])
        assert saved["kind"] == 1 and saved["path"] == rc.RC_PATH_DENSE and saved["strip"] == 128
        assert rc.rc_tune_load(str(out)) == 1
    finally:
        rc.rc_tune_load()
