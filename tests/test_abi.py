"""The C-ABI library loads, exports every symbol include/rfps.h declares, and
rejects invalid arguments on the host before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(rfps_[a-z_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    import paper_2606_06255_amd as rf
    return rf.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 28
    assert "rfps_gather_xyz" in names and "rfps_mlp_train_step" in names and "rfps_sample_batched" in names
    for name in names:
        assert hasattr(L, name), name


def test_status_strings(L):
    import paper_2606_06255_amd as rf
    for code in range(10):
        s = L.rfps_status_str(code)
        assert isinstance(s, bytes) and len(s) > 0
    assert L.rfps_status_str(99) == b"unknown status"
    assert rf.STATUS_NAMES[7] == "RFPS_ERR_TIMEOUT"
    assert rf.STATUS_NAMES[9] == "RFPS_ERR_SCRATCH_LIMIT"


def test_workspace_sizes(L):
    import paper_2606_06255_amd as rf
    p = rf.rfps_params(n_vox=16)
    a = L.rfps_index_workspace_size(1000, ctypes.byref(p))
    b = L.rfps_index_workspace_size(100000, ctypes.byref(p))
    assert 0 < a < b and a % 256 == 0
    assert L.rfps_index_workspace_size(0, ctypes.byref(p)) == 0
    assert L.rfps_index_workspace_size(-5, None) == 0
    for la in (2, 3, 4, 8):
        ok = rf.rfps_params(n_vox=16, lookahead=la)
        assert L.rfps_index_workspace_size(1000, ctypes.byref(ok)) == a
    for bad in (rf.rfps_params(n_vox=2000), rf.rfps_params(n_vox=16, tile=65), rf.rfps_params(groups=257),
                rf.rfps_params(flags=0x100), rf.rfps_params(n_vox=-1), rf.rfps_params(lookahead=5),
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
    assert L.rfps_sample(ctypes.byref(h), 10, 0, None, out, None, None) == 1   # shells = 0 is no handle
    h.shells = 65
    assert L.rfps_sample(ctypes.byref(h), 10, 0, None, out, None, None) == 1
    h.shells = 1
    assert L.rfps_sample(ctypes.byref(h), 0, 0, None, out, None, None) == 1
    assert L.rfps_sample(ctypes.byref(h), 101, 0, None, out, None, None) == 1
    assert L.rfps_sample(ctypes.byref(h), 10, 100, None, out, None, None) == 1
    assert L.rfps_sample(ctypes.byref(h), 10, -1, None, out, None, None) == 1
    assert L.rfps_sample(ctypes.byref(h), 10, 0, None, None, None, None) == 1
    for fl in (rf.F_UNFUSED | rf.F_TELEMETRY, rf.F_UNFUSED | rf.F_TRACE):
        assert L.rfps_sample(ctypes.byref(h), 10, 0, ctypes.byref(rf.rfps_params(flags=fl)), out, None, None) == 5
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
    # stage gather: NULL pointers and sizes
    assert L.rfps_gather_xyz(None, 10, fake, 5, out, None) == 1
    assert L.rfps_gather_xyz(fake, 10, None, 5, out, None) == 1
    assert L.rfps_gather_xyz(fake, 10, fake, 5, None, None) == 1
    assert L.rfps_gather_xyz(fake, 0, fake, 5, out, None) == 1
    assert L.rfps_gather_xyz(fake, 10, fake, 0, out, None) == 1
    # readers reject bad handles without touching the device
    t = rf.rfps_telemetry()
    assert L.rfps_read_telemetry(None, None, ctypes.byref(t)) == 1
    assert L.rfps_read_status(None, None) == 1
    assert L.rfps_read_trace(None, None, out, 4, None) == -1


def test_batched_workspace_and_host_checks(L):
    import paper_2606_06255_amd as rf
    p = rf.rfps_params()
    a = L.rfps_batched_workspace_size(100000, 32, ctypes.byref(p))
    single = L.rfps_index_workspace_size(100000, ctypes.byref(rf.rfps_params(n_vox=64)))
    assert a > 0 and a % 256 == 0 and a >= single
    fixed = rf.rfps_params(n_vox=16)
    assert 0 < L.rfps_batched_workspace_size(100000, 32, ctypes.byref(fixed)) <= a
    assert L.rfps_batched_workspace_size(100000, 0, None) == 0
    assert L.rfps_batched_workspace_size(100000, 4097, None) == 0
    assert L.rfps_batched_workspace_size(10, 11, None) == 0
    assert L.rfps_batched_workspace_size(0, 1, None) == 0
    assert L.rfps_batched_workspace_size(1000, 2, ctypes.byref(rf.rfps_params(lookahead=5))) == 0
    fake = ctypes.c_void_p(0x1000)
    out = ctypes.c_void_p(0x2000)
    args = dict(xyz=fake, n=100, off=fake, m=fake, st=None, b=4, mt=20, p=None, ws=fake, wsb=1 << 30, oi=out)

    def call(**kw):
        a = dict(args)
        a.update(kw)
        return L.rfps_sample_batched(a["xyz"], a["n"], a["off"], a["m"], a["st"], a["b"], a["mt"], a["p"],
                                     a["ws"], a["wsb"], a["oi"], None, None)
    assert call(xyz=None) == 1
    assert call(off=None) == 1
    assert call(m=None) == 1
    assert call(oi=None) == 1
    assert call(b=0) == 1
    assert call(b=101) == 1
    assert call(mt=3) == 1        # fewer outputs than clouds
    assert call(mt=101) == 1      # more outputs than points
    assert call(n=0) == 1
    for fl in (rf.F_NO_PRUNE, rf.F_SINGLE_PICK, rf.F_TRACE, rf.F_UNFUSED):
        assert call(p=ctypes.byref(rf.rfps_params(flags=fl))) == 5
    assert call(ws=None) == 3
    assert call(ws=ctypes.c_void_p(0x1001)) == 3
    assert call(wsb=64) == 3
    assert L.rfps_batched_read_status(None, 0, None) == 3
    t = rf.rfps_telemetry()
    assert L.rfps_batched_read_telemetry(fake, 1 << 20, None, None) == 1
    best = rf.rfps_params()
    assert L.rfps_autotune_batched(fake, 100, fake, fake, None, 4, 20, None, 0, fake, 1 << 30, out, None, None,
                                   ctypes.byref(best), None) == 1
    assert L.rfps_autotune_batched(fake, 100, fake, fake, None, 4, 20, None, 3, fake, 1 << 30, out, None, None,
                                   None, None) == 1


def test_shell_parameter(L):
    import paper_2606_06255_amd as rf
    base = L.rfps_index_workspace_size(5000, ctypes.byref(rf.rfps_params(n_vox=16)))
    for sh in (5.0, 0.25, float("inf")):
        assert L.rfps_index_workspace_size(5000, ctypes.byref(rf.rfps_params(n_vox=16, shell_spacing=sh))) >= base
    for bad in (-1.0, float("nan")):
        assert L.rfps_index_workspace_size(5000, ctypes.byref(rf.rfps_params(n_vox=16, shell_spacing=bad))) == 0
    fake = ctypes.c_void_p(0x1000)
    h = rf.rfps_index()
    p = rf.rfps_params(n_vox=16, shell_spacing=-2.0)
    assert L.rfps_build_index(fake, 10, ctypes.byref(p), fake, 1 << 30, None, ctypes.byref(h)) == 1


def test_mlp_host_checks(L):
    import paper_2606_06255_amd as rf
    assert rf.mlp_candidate(0) == (12, 0.0) and rf.mlp_candidate(35) == (192, 20.0)
    assert rf.mlp_candidate(13) == (32, 5.0)
    with pytest.raises(ValueError):
        rf.mlp_candidate(36)
    assert L.rfps_mlp_state_size() >= 4 * 3 * rf.MLP_PARAMS
    assert L.rfps_mlp_workspace_size(0) == 0 and L.rfps_mlp_workspace_size(1 << 17) == 0
    assert L.rfps_mlp_workspace_size(64) > L.rfps_mlp_workspace_size(1) > 0
    fake = ctypes.c_void_p(0x1000)
    big = 1 << 30
    # state / workspace checks come before any device work
    assert L.rfps_mlp_forward(None, big, fake, 1, fake, big, fake, None) == 3
    assert L.rfps_mlp_forward(fake, 16, fake, 1, fake, big, fake, None) == 3
    assert L.rfps_mlp_forward(fake, big, fake, 0, fake, big, fake, None) == 1
    assert L.rfps_mlp_forward(fake, big, fake, 4, fake, 64, fake, None) == 3
    assert L.rfps_mlp_forward(fake, big, None, 1, fake, big, fake, None) == 1
    assert L.rfps_mlp_train_step(fake, big, fake, fake, None, 4, 0.0, fake, big, None, None) == 1
    assert L.rfps_mlp_train_step(fake, big, fake, fake, None, 4, float("nan"), fake, big, None, None) == 1
    assert L.rfps_mlp_choose(fake, big, fake, 36, 0.0, fake, big, fake, None, None) == 1
    assert L.rfps_mlp_choose(fake, big, fake, 3, -1.0, fake, big, fake, None, None) == 1
    assert L.rfps_mlp_features(None, 10, fake, big, fake, None) == 1
    assert L.rfps_mlp_features(fake, 0, fake, big, fake, None) == 1
    assert L.rfps_mlp_load(fake, big, None, None) == 1
    assert L.rfps_mlp_save(None, big, fake, None) == 3


def test_noalloc_host_checks(L):
    """rfps_sample_batched_noalloc rejects bad arguments and inputs beyond its
    fixed array on the host, before any device work."""
    import paper_2606_06255_amd as rf
    cap = L.rfps_noalloc_scratch_bytes()
    assert cap == 128 << 20
    fake = ctypes.c_void_p(0x1000)
    out = ctypes.c_void_p(0x2000)

    def call(xyz=fake, n=100, off=fake, m=fake, b=4, mt=20, p=None, oi=out):
        return L.rfps_sample_batched_noalloc(xyz, n, off, m, None, b, mt, p, oi, None, None)
    assert call(xyz=None) == 1
    assert call(off=None) == 1
    assert call(oi=None) == 1
    assert call(b=0) == 1
    assert call(mt=3) == 1
    assert call(n=0) == 1
    assert call(p=ctypes.byref(rf.rfps_params(lookahead=5))) == 1
    # the largest batch that fits and the first that does not
    assert 0 < L.rfps_batched_workspace_size(1_500_000, 32, None) <= cap
    big = 1 << 26
    assert L.rfps_batched_workspace_size(big, 1, None) > cap
    assert call(n=big, b=1, mt=1) == 9
    assert call(n=big, b=32, mt=64) == 9
