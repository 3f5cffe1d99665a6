"""The C-ABI library loads, exports every symbol include/rfps.h declares, and
rejects invalid arguments on the host before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rfps.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rfps_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_2606_06255_amd as rf
    return rf.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name


def test_status_strings(L):
    import paper_2606_06255_amd as rf
    for code in range(8):
        s = L.rfps_status_str(code)
        assert isinstance(s, bytes) and len(s) > 0
    assert L.rfps_status_str(99) == b"unknown status"
    assert rf.STATUS_NAMES[7] == "RFPS_ERR_TIMEOUT"


def test_workspace_sizes(L):
    import paper_2606_06255_amd as rf
    p = rf.rfps_params(n_vox=16)
    a = L.rfps_index_workspace_size(1000, ctypes.byref(p))
    b = L.rfps_index_workspace_size(100000, ctypes.byref(p))
    assert 0 < a < b and a % 256 == 0
    assert L.rfps_index_workspace_size(0, ctypes.byref(p)) == 0
    assert L.rfps_index_workspace_size(-5, None) == 0
    for la in (2, 4, 8):
        ok = rf.rfps_params(n_vox=16, lookahead=la)
        assert L.rfps_index_workspace_size(1000, ctypes.byref(ok)) == a
    for bad in (rf.rfps_params(n_vox=2000), rf.rfps_params(n_vox=16, tile=65), rf.rfps_params(groups=257),
                rf.rfps_params(flags=0x100), rf.rfps_params(n_vox=-1), rf.rfps_params(lookahead=3),
                rf.rfps_params(lookahead=16), rf.rfps_params(lookahead=-1)):
        assert L.rfps_index_workspace_size(1000, ctypes.byref(bad)) == 0
    assert L.rfps_fps_plain_workspace_size(1000, 0) > 0
    assert L.rfps_fps_plain_workspace_size(1000, 2) == 0
    assert L.rfps_fps_plain_workspace_size(0, 0) == 0


def test_default_n_vox(L):
    vals = [L.rfps_default_n_vox(n) for n in (1, 4096, 80000, 114624, 1 << 20)]
    assert vals == sorted(vals) and all(8 <= v <= 256 for v in vals)


def test_invalid_arguments_return_before_device_work(L):
    import paper_2606_06255_amd as rf
    h = rf.rfps_index()
    p = rf.rfps_params(16, 0, 0, 0)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    # build: NULL input, n < 1, bad params, NULL / misaligned / small workspace
    assert L.rfps_build_index(None, 10, None, fake, 1 << 30, None, ctypes.byref(h)) == 1
    assert L.rfps_build_index(fake, 0, None, fake, 1 << 30, None, ctypes.byref(h)) == 1
    bad = rf.rfps_params(0, 100, 0, 0)
    assert L.rfps_build_index(fake, 10, ctypes.byref(bad), fake, 1 << 30, None, ctypes.byref(h)) == 1
    assert L.rfps_build_index(fake, 10, ctypes.byref(p), None, 1 << 30, None, ctypes.byref(h)) == 3
    assert L.rfps_build_index(fake, 10, ctypes.byref(p), ctypes.c_void_p(0x1001), 1 << 30, None,
                              ctypes.byref(h)) == 3
    assert L.rfps_build_index(fake, 10, ctypes.byref(p), fake, 64, None, ctypes.byref(h)) == 3
    # sample: NULL handle, bad handle, m / start out of range
    out = ctypes.c_void_p(0x2000)
    assert L.rfps_sample(None, 1, 0, None, out, None, None) == 1
    h.n, h.n_vox, h.tile, h.ws, h.ws_bytes = 100, 16, 64, 0x1000, 1 << 30
    assert L.rfps_sample(ctypes.byref(h), 0, 0, None, out, None, None) == 1
    assert L.rfps_sample(ctypes.byref(h), 101, 0, None, out, None, None) == 1
    assert L.rfps_sample(ctypes.byref(h), 10, 100, None, out, None, None) == 1
    assert L.rfps_sample(ctypes.byref(h), 10, -1, None, out, None, None) == 1
    assert L.rfps_sample(ctypes.byref(h), 10, 0, None, None, None, None) == 1
    h.ws_bytes = 10
    assert L.rfps_sample(ctypes.byref(h), 10, 0, None, out, None, None) == 3
    h.ws = 0x1001
    h.ws_bytes = 1 << 30
    assert L.rfps_sample(ctypes.byref(h), 10, 0, None, out, None, None) == 3
    # plain
    assert L.rfps_fps_plain(None, 10, 5, 0, 0, 0, fake, 1 << 30, out, None, None) == 1
    assert L.rfps_fps_plain(fake, 10, 11, 0, 0, 0, fake, 1 << 30, out, None, None) == 1
    assert L.rfps_fps_plain(fake, 10, 5, 0, 3, 0, fake, 1 << 30, out, None, None) == 1
    assert L.rfps_fps_plain(fake, 10, 5, 0, 0, 300, fake, 1 << 30, out, None, None) == 1
    assert L.rfps_fps_plain(fake, 10, 5, 0, 0, 0, None, 1 << 30, out, None, None) == 3
    assert L.rfps_fps_plain(fake, 10, 5, 0, 0, 0, fake, 16, out, None, None) == 3
    assert L.rfps_read_plain_status(None, 0, None) == 3
    # readers reject bad handles without touching the device
    t = rf.rfps_telemetry()
    assert L.rfps_read_telemetry(None, None, ctypes.byref(t)) == 1
    assert L.rfps_read_status(None, None) == 1
    assert L.rfps_read_trace(None, None, out, 4, None) == -1
