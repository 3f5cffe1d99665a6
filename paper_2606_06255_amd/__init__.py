"""RadiusFPS-G for AMD Instinct MI355X: Python binding of librfps.so.

Thin ctypes marshalling over the C ABI in include/rfps.h, with the same
names.  PyTorch supplies device memory (input, outputs, workspace) and the
stream; every step of the sampling path runs in the library's HIP kernels.
The binding fails loudly when the library is missing or no GPU is present:
there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librfps.so")

RFPS_OK = 0
STATUS_NAMES = {
    0: "RFPS_OK", 1: "RFPS_ERR_INVALID_ARG", 2: "RFPS_ERR_NONFINITE", 3: "RFPS_ERR_WORKSPACE",
    4: "RFPS_ERR_DEVICE", 5: "RFPS_ERR_UNSUPPORTED", 6: "RFPS_ERR_CAPACITY", 7: "RFPS_ERR_TIMEOUT",
    8: "RFPS_ERR_INTERNAL",
}
F_NO_PRUNE = 0x01
F_NO_POINT_SKIP = 0x02
F_TELEMETRY = 0x04
F_TRACE = 0x08
F_SINGLE_PICK = 0x10
WS_ALIGN = 256


class rfps_params(ctypes.Structure):
    _fields_ = [("n_vox", ctypes.c_int32), ("tile", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("lookahead", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class rfps_index(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_vox", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t)]


class rfps_telemetry(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "iters", "tiles", "tile_tests", "tiles_pruned", "points_visited", "points_skipped",
        "points_updated", "tiles_resynced", "exchanges", "ticks_lookahead", "ticks_exchange",
        "ticks_merge", "ticks_apply", "tick_hz", "reserved0", "reserved1")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_ if not k.startswith("reserved")}


class rfps_index_info(ctypes.Structure):
    _fields_ = [("n_voxels", ctypes.c_int64), ("n_tiles", ctypes.c_int64), ("pmin", ctypes.c_double * 3),
                ("voxel_edge", ctypes.c_double)]


class RfpsError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__("%s: %s (%d)" % (where, STATUS_NAMES.get(status, "unknown"), status))
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Loads librfps.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librfps.so is not built: run paper_2606_06255_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        i32, u32, sz, vp = ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_void_p
        L.rfps_index_workspace_size.argtypes = [i32, P(rfps_params)]
        L.rfps_index_workspace_size.restype = sz
        L.rfps_build_index.argtypes = [vp, i32, P(rfps_params), vp, sz, vp, P(rfps_index)]
        L.rfps_build_index.restype = ctypes.c_int
        L.rfps_sample.argtypes = [P(rfps_index), i32, i32, P(rfps_params), vp, vp, vp]
        L.rfps_sample.restype = ctypes.c_int
        L.rfps_read_status.argtypes = [P(rfps_index), vp]
        L.rfps_read_status.restype = ctypes.c_int
        L.rfps_read_index_info.argtypes = [P(rfps_index), vp, P(rfps_index_info)]
        L.rfps_read_index_info.restype = ctypes.c_int
        L.rfps_read_telemetry.argtypes = [P(rfps_index), vp, P(rfps_telemetry)]
        L.rfps_read_telemetry.restype = ctypes.c_int
        L.rfps_read_trace.argtypes = [P(rfps_index), vp, vp, i32, P(ctypes.c_double)]
        L.rfps_read_trace.restype = i32
        L.rfps_fps_plain_workspace_size.argtypes = [i32, i32]
        L.rfps_fps_plain_workspace_size.restype = sz
        L.rfps_fps_plain.argtypes = [vp, i32, i32, i32, i32, i32, vp, sz, vp, vp, vp]
        L.rfps_fps_plain.restype = ctypes.c_int
        L.rfps_read_plain_status.argtypes = [vp, sz, vp]
        L.rfps_read_plain_status.restype = ctypes.c_int
        L.rfps_status_str.argtypes = [ctypes.c_int]
        L.rfps_status_str.restype = ctypes.c_char_p
        L.rfps_default_n_vox.argtypes = [i32]
        L.rfps_default_n_vox.restype = i32
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != RFPS_OK:
        raise RfpsError(status, where)


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _workspace(nbytes: int, device) -> tuple[torch.Tensor, int]:
    buf = torch.empty(nbytes + WS_ALIGN, dtype=torch.uint8, device=device)
    ptr = buf.data_ptr()
    return buf, ptr + (-ptr) % WS_ALIGN


def _check_xyz(xyz: torch.Tensor):
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the RadiusFPS-G path runs only on a gfx950 device")
    if not (isinstance(xyz, torch.Tensor) and xyz.is_cuda and xyz.dtype == torch.float32 and xyz.dim() == 2
            and xyz.shape[1] == 3 and xyz.is_contiguous()):
        raise ValueError("xyz must be a contiguous float32 CUDA tensor of shape [N, 3]")


def _params(n_vox=0, tile=0, groups=0, flags=0, lookahead=0) -> rfps_params:
    return rfps_params(int(n_vox), int(tile), int(groups), int(lookahead), int(flags))


def default_n_vox(n: int) -> int:
    return int(lib().rfps_default_n_vox(int(n)))


class Index:
    """A voxel index in a torch-owned workspace (rfps_index + its memory)."""

    def __init__(self, handle: rfps_index, ws: torch.Tensor, device):
        self.handle = handle
        self.ws = ws
        self.device = device

    @property
    def n(self) -> int:
        return int(self.handle.n)

    @property
    def n_vox(self) -> int:
        return int(self.handle.n_vox)


def index_workspace_size(n: int, n_vox: int = 0, tile: int = 0) -> int:
    p = _params(n_vox, tile)
    return int(lib().rfps_index_workspace_size(int(n), ctypes.byref(p)))


def build_index(xyz: torch.Tensor, n_vox: int = 0, tile: int = 0, reuse: Index | None = None) -> Index:
    """rfps_build_index on torch's current stream.

    With `reuse`, the workspace of that index is rebuilt in place when it is
    large enough (the old index is then invalid); nothing is allocated.
    """
    _check_xyz(xyz)
    L = lib()
    n = xyz.shape[0]
    p = _params(n_vox, tile)
    nbytes = L.rfps_index_workspace_size(n, ctypes.byref(p))
    if nbytes == 0:
        raise RfpsError(1, "rfps_index_workspace_size")
    if reuse is not None and reuse.ws_bytes >= nbytes and reuse.device == xyz.device:
        ws, ptr, nbytes = reuse.ws, reuse.ws_ptr, reuse.ws_bytes
    else:
        ws, ptr = _workspace(nbytes, xyz.device)
    h = rfps_index()
    _check(L.rfps_build_index(xyz.data_ptr(), n, ctypes.byref(p), ptr, nbytes, _stream(xyz.device),
                              ctypes.byref(h)), "rfps_build_index")
    idx = Index(h, ws, xyz.device)
    idx.ws_ptr, idx.ws_bytes = ptr, nbytes
    return idx


def sample(index: Index, m: int, start: int = 0, groups: int = 0, flags: int = 0, lookahead: int = 0,
           out_idx: torch.Tensor | None = None, out_d2: torch.Tensor | None = None):
    """rfps_sample: returns (idx int32 [m], d2 float32 [m]) on the index's device."""
    dev = index.device
    if out_idx is None:
        out_idx = torch.empty(m, dtype=torch.int32, device=dev)
    if out_d2 is None:
        out_d2 = torch.empty(m, dtype=torch.float32, device=dev)
    p = _params(0, 0, groups, flags, lookahead)
    _check(lib().rfps_sample(ctypes.byref(index.handle), int(m), int(start), ctypes.byref(p),
                             out_idx.data_ptr(), out_d2.data_ptr(), _stream(dev)), "rfps_sample")
    return out_idx, out_d2


def read_status(index: Index) -> int:
    return int(lib().rfps_read_status(ctypes.byref(index.handle), _stream(index.device)))


def read_index_info(index: Index) -> dict:
    info = rfps_index_info()
    _check(lib().rfps_read_index_info(ctypes.byref(index.handle), _stream(index.device), ctypes.byref(info)),
           "rfps_read_index_info")
    return {"n_voxels": int(info.n_voxels), "n_tiles": int(info.n_tiles), "pmin": list(info.pmin),
            "voxel_edge": float(info.voxel_edge)}


def read_telemetry(index: Index) -> dict:
    t = rfps_telemetry()
    _check(lib().rfps_read_telemetry(ctypes.byref(index.handle), _stream(index.device), ctypes.byref(t)),
           "rfps_read_telemetry")
    return t.as_dict()


def read_trace(index: Index, cap: int = 1 << 17):
    """Per-selection (publish, winner known) wall-clock ticks of workgroup 0 and the tick rate."""
    import numpy as np
    buf = np.zeros(2 * cap, dtype=np.uint64)
    hz = ctypes.c_double(0.0)
    cnt = lib().rfps_read_trace(ctypes.byref(index.handle), _stream(index.device), buf.ctypes.data, cap,
                                ctypes.byref(hz))
    if cnt < 0:
        raise RfpsError(4, "rfps_read_trace")
    return buf[:2 * cnt].reshape(cnt, 2), hz.value


def fps(xyz: torch.Tensor, m: int, start: int = 0, n_vox: int = 0, tile: int = 0, groups: int = 0,
        flags: int = 0, lookahead: int = 0):
    """Build the index and sample: exact FPS with spherical-voxel pruning."""
    idx = build_index(xyz, n_vox=n_vox, tile=tile)
    out = sample(idx, m, start, groups=groups, flags=flags, lookahead=lookahead)
    st = read_status(idx)
    _check(st, "device status")
    return out


class PlainWorkspace:
    def __init__(self, n: int, device):
        self.nbytes = int(lib().rfps_fps_plain_workspace_size(int(n), 0))
        if self.nbytes == 0:
            raise RfpsError(1, "rfps_fps_plain_workspace_size")
        self.buf, self.ptr = _workspace(self.nbytes, device)
        self.device = device


def fps_plain(xyz: torch.Tensor, m: int, start: int = 0, variant: int = 0, groups: int = 0,
              ws: PlainWorkspace | None = None, out_idx=None, out_d2=None, check: bool = True):
    """rfps_fps_plain: plain FPS (variant 0 persistent, 1 one workgroup)."""
    _check_xyz(xyz)
    dev = xyz.device
    n = xyz.shape[0]
    if ws is None:
        ws = PlainWorkspace(n, dev)
    if out_idx is None:
        out_idx = torch.empty(m, dtype=torch.int32, device=dev)
    if out_d2 is None:
        out_d2 = torch.empty(m, dtype=torch.float32, device=dev)
    _check(lib().rfps_fps_plain(xyz.data_ptr(), n, int(m), int(start), int(variant), int(groups), ws.ptr,
                                ws.nbytes, out_idx.data_ptr(), out_d2.data_ptr(), _stream(dev)),
           "rfps_fps_plain")
    if check:
        _check(lib().rfps_read_plain_status(ws.ptr, ws.nbytes, _stream(dev)), "device status")
    return out_idx, out_d2
