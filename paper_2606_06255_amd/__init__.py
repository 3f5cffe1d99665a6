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
    8: "RFPS_ERR_INTERNAL", 9: "RFPS_ERR_SCRATCH_LIMIT",
}
F_NO_PRUNE = 0x01
F_NO_POINT_SKIP = 0x02
F_TELEMETRY = 0x04
F_TRACE = 0x08
F_SINGLE_PICK = 0x10
F_SQRT = 0x20
F_UNFUSED = 0x40
F_CLOCKS = 0x80
WS_ALIGN = 256


class rfps_params(ctypes.Structure):
    _fields_ = [("n_vox", ctypes.c_int32), ("tile", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("lookahead", ctypes.c_int32), ("flags", ctypes.c_uint32), ("shell_spacing", ctypes.c_float)]


class rfps_index(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_vox", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("shells", ctypes.c_int32), ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t)]


class rfps_telemetry(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "iters", "tiles", "tile_tests", "tiles_pruned", "points_visited", "points_skipped",
        "points_updated", "tiles_resynced", "exchanges", "ticks_lookahead", "ticks_exchange",
        "ticks_merge", "ticks_apply", "tick_hz", "ticks_wait", "reserved",
        "ticks_merge_list", "ticks_merge_rank", "ticks_merge_walk", "ticks_merge_picks", "ticks_lookahead_copy",
        "ticks_lookahead_steps", "ticks_exchange_poll", "ticks_exchange_keys", "merge_above", "merge_listed",
        "merge_failures", "ticks_apply_loop", "ticks_lookahead_select", "ticks_apply_update", "apply_pairs",
        "apply_rekeys")]

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
        L.rfps_probe_exchange.argtypes = [P(rfps_index), i32, i32, i32, vp, P(ctypes.c_double)]
        L.rfps_probe_exchange.restype = ctypes.c_int
        L.rfps_read_trace.argtypes = [P(rfps_index), vp, vp, i32, P(ctypes.c_double)]
        L.rfps_read_trace.restype = i32
        L.rfps_fps_plain_workspace_size.argtypes = [i32, i32]
        L.rfps_fps_plain_workspace_size.restype = sz
        L.rfps_fps_plain.argtypes = [vp, i32, i32, i32, i32, i32, vp, sz, vp, vp, vp]
        L.rfps_fps_plain.restype = ctypes.c_int
        L.rfps_gather_xyz.argtypes = [vp, i32, vp, i32, vp, vp]
        L.rfps_gather_xyz.restype = ctypes.c_int
        L.rfps_cpu_sample.argtypes = [vp, i32, i32, i32, P(rfps_params), i32, vp, vp]
        L.rfps_cpu_sample.restype = ctypes.c_int
        L.rfps_read_plain_status.argtypes = [vp, sz, vp]
        L.rfps_read_plain_status.restype = ctypes.c_int
        L.rfps_batched_workspace_size.argtypes = [i32, i32, P(rfps_params)]
        L.rfps_batched_workspace_size.restype = sz
        L.rfps_sample_batched.argtypes = [vp, i32, vp, vp, vp, i32, i32, P(rfps_params), vp, sz, vp, vp, vp]
        L.rfps_sample_batched.restype = ctypes.c_int
        L.rfps_sample_batched_noalloc.argtypes = [vp, i32, vp, vp, vp, i32, i32, P(rfps_params), vp, vp, vp]
        L.rfps_sample_batched_noalloc.restype = ctypes.c_int
        L.rfps_noalloc_scratch_bytes.argtypes = []
        L.rfps_noalloc_scratch_bytes.restype = sz
        L.rfps_batched_read_status.argtypes = [vp, sz, vp]
        L.rfps_batched_read_status.restype = ctypes.c_int
        L.rfps_batched_read_telemetry.argtypes = [vp, sz, vp, P(rfps_telemetry)]
        L.rfps_batched_read_telemetry.restype = ctypes.c_int
        L.rfps_autotune_batched.argtypes = [vp, i32, vp, vp, vp, i32, i32, P(rfps_params), i32, vp, sz, vp, vp,
                                            vp, P(rfps_params), P(ctypes.c_float)]
        L.rfps_autotune_batched.restype = ctypes.c_int
        f32 = ctypes.c_float
        L.rfps_mlp_candidate.argtypes = [i32, P(i32), P(f32)]
        L.rfps_mlp_candidate.restype = i32
        L.rfps_mlp_state_size.argtypes = []
        L.rfps_mlp_state_size.restype = sz
        L.rfps_mlp_workspace_size.argtypes = [i32]
        L.rfps_mlp_workspace_size.restype = sz
        L.rfps_mlp_load.argtypes = [vp, sz, vp, vp]
        L.rfps_mlp_load.restype = ctypes.c_int
        L.rfps_mlp_save.argtypes = [vp, sz, vp, vp]
        L.rfps_mlp_save.restype = ctypes.c_int
        L.rfps_mlp_features.argtypes = [vp, i32, vp, sz, vp, vp]
        L.rfps_mlp_features.restype = ctypes.c_int
        L.rfps_mlp_forward.argtypes = [vp, sz, vp, i32, vp, sz, vp, vp]
        L.rfps_mlp_forward.restype = ctypes.c_int
        L.rfps_mlp_gradient.argtypes = [vp, sz, vp, vp, vp, i32, vp, sz, vp, vp, vp]
        L.rfps_mlp_gradient.restype = ctypes.c_int
        L.rfps_mlp_train_step.argtypes = [vp, sz, vp, vp, vp, i32, f32, vp, sz, vp, vp]
        L.rfps_mlp_train_step.restype = ctypes.c_int
        L.rfps_mlp_choose.argtypes = [vp, sz, vp, i32, f32, vp, sz, vp, vp, vp]
        L.rfps_mlp_choose.restype = ctypes.c_int
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


def _params(n_vox=0, tile=0, groups=0, flags=0, lookahead=0, shell=0.0) -> rfps_params:
    return rfps_params(int(n_vox), int(tile), int(groups), int(lookahead), int(flags), float(shell))


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


def index_workspace_size(n: int, n_vox: int = 0, tile: int = 0, shell: float = 0.0) -> int:
    p = _params(n_vox, tile, shell=shell)
    return int(lib().rfps_index_workspace_size(int(n), ctypes.byref(p)))


def build_index(xyz: torch.Tensor, n_vox: int = 0, tile: int = 0, reuse: Index | None = None,
                shell: float = 0.0) -> Index:
    """rfps_build_index on torch's current stream.

    With `reuse`, the workspace of that index is rebuilt in place when it is
    large enough (the old index is then invalid); nothing is allocated.
    """
    _check_xyz(xyz)
    L = lib()
    n = xyz.shape[0]
    p = _params(n_vox, tile, shell=shell)
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


def probe_exchange(index: Index, words: int, rounds: int = 2000, groups: int = 0) -> float:
    """rfps_probe_exchange: microseconds per bare exchange round of `words`
    words per workgroup among `groups` workgroups (0 = one per compute unit)."""
    us = ctypes.c_double(0.0)
    _check(lib().rfps_probe_exchange(ctypes.byref(index.handle), int(groups), int(words), int(rounds),
                                     _stream(index.device), ctypes.byref(us)), "rfps_probe_exchange")
    return float(us.value)


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
        flags: int = 0, lookahead: int = 0, shell: float = 0.0):
    """Build the index and sample: exact FPS with spherical-voxel pruning."""
    idx = build_index(xyz, n_vox=n_vox, tile=tile, shell=shell)
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


def gather_xyz(xyz: torch.Tensor, idx: torch.Tensor, out=None):
    """rfps_gather_xyz: the coordinates of the samples in sample order (the next
    stage's input when down-sampling in stages)."""
    _check_xyz(xyz)
    if not (idx.is_cuda and idx.dtype == torch.int32 and idx.dim() == 1 and idx.is_contiguous()):
        raise ValueError("idx must be a contiguous int32 CUDA tensor")
    m = idx.shape[0]
    if out is None:
        out = torch.empty((m, 3), dtype=torch.float32, device=xyz.device)
    _check(lib().rfps_gather_xyz(xyz.data_ptr(), xyz.shape[0], idx.data_ptr(), m, out.data_ptr(),
                                 _stream(xyz.device)), "rfps_gather_xyz")
    return out


def cpu_fps(xyz, m: int, start: int = 0, n_vox: int = 0, tile: int = 0, flags: int = 0, threads: int = 0):
    """rfps_cpu_sample: CPU RadiusFPS on the host cores.  xyz is a float32
    [N, 3] array (numpy, or a CPU tensor); returns (idx int32 [m], d2 float32 [m])
    as numpy arrays."""
    import numpy as np
    if isinstance(xyz, torch.Tensor):
        xyz = xyz.detach().cpu().numpy()
    a = np.ascontiguousarray(xyz, dtype=np.float32)
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("xyz must be [N, 3]")
    idx = np.empty(m, dtype=np.int32)
    d2 = np.empty(m, dtype=np.float32)
    p = _params(n_vox, tile, flags=flags)
    _check(lib().rfps_cpu_sample(a.ctypes.data, a.shape[0], int(m), int(start), ctypes.byref(p), int(threads),
                                 idx.ctypes.data, d2.ctypes.data), "rfps_cpu_sample")
    return idx, d2


# ---------------------------------------------------------------------------
# Batches of clouds
# ---------------------------------------------------------------------------
class BatchWorkspace:
    """Device workspace of rfps_sample_batched for up to n points in `batch` clouds."""

    def __init__(self, n: int, batch: int, device, n_vox: int = 0, shell: float = 0.0):
        p = _params(n_vox, shell=shell)
        self.nbytes = int(lib().rfps_batched_workspace_size(int(n), int(batch), ctypes.byref(p)))
        if self.nbytes == 0:
            raise RfpsError(1, "rfps_batched_workspace_size")
        self.buf, self.ptr = _workspace(self.nbytes, device)
        self.device = device
        self.n, self.batch, self.n_vox = int(n), int(batch), int(n_vox)

    def fits(self, n: int, batch: int, n_vox: int, shell: float = 0.0) -> bool:
        p = _params(n_vox, shell=shell)
        need = int(lib().rfps_batched_workspace_size(int(n), int(batch), ctypes.byref(p)))
        return 0 < need <= self.nbytes


def _i32_dev(x, device) -> torch.Tensor:
    t = torch.as_tensor(x, dtype=torch.int32)
    if not t.is_cuda:
        t = t.to(device)
    if t.device != device or not t.is_contiguous():
        t = t.to(device).contiguous()
    return t


def sample_batched(xyz: torch.Tensor, offsets, m, starts=None, m_total: int | None = None, n_vox: int = 0,
                   tile: int = 0, groups: int = 0, lookahead: int = 0, flags: int = 0,
                   ws: BatchWorkspace | None = None, out_idx=None, out_d2=None, check: bool = True,
                   shell: float = 0.0):
    """rfps_sample_batched on torch's current stream.

    offsets (int32 [B+1]), m (int32 [B]) and starts (int32 [B] or None) may be
    host sequences or device tensors; m_total is read from m when m is on the
    host, else it must be given.  Returns (idx, d2), both [m_total]: the
    selections of cloud c follow those of clouds 0..c-1, as local indices.
    With check=False nothing waits for the device (graph capture).
    """
    _check_xyz(xyz)
    dev = xyz.device
    n = xyz.shape[0]
    if m_total is None:
        if isinstance(m, torch.Tensor) and m.is_cuda:
            raise ValueError("m_total is required when m is a device tensor")
        m_total = int(sum(int(v) for v in m))
    offsets_d = _i32_dev(offsets, dev)
    m_d = _i32_dev(m, dev)
    starts_d = None if starts is None else _i32_dev(starts, dev)
    batch = offsets_d.numel() - 1
    if m_d.numel() != batch or (starts_d is not None and starts_d.numel() != batch):
        raise ValueError("offsets, m and starts disagree on the batch size")
    if ws is None or not ws.fits(n, batch, n_vox, shell):
        ws = BatchWorkspace(n, batch, dev, n_vox=n_vox, shell=shell)
    if out_idx is None:
        out_idx = torch.empty(m_total, dtype=torch.int32, device=dev)
    if out_d2 is None:
        out_d2 = torch.empty(m_total, dtype=torch.float32, device=dev)
    p = _params(n_vox, tile, groups, flags, lookahead, shell)
    _check(lib().rfps_sample_batched(xyz.data_ptr(), n, offsets_d.data_ptr(), m_d.data_ptr(),
                                     0 if starts_d is None else starts_d.data_ptr(), batch, int(m_total),
                                     ctypes.byref(p), ws.ptr, ws.nbytes, out_idx.data_ptr(), out_d2.data_ptr(),
                                     _stream(dev)), "rfps_sample_batched")
    if check:
        _check(lib().rfps_batched_read_status(ws.ptr, ws.nbytes, _stream(dev)), "device status")
    return out_idx, out_d2


def sample_batched_noalloc(xyz: torch.Tensor, offsets: torch.Tensor, m: torch.Tensor, m_total: int,
                           out_idx: torch.Tensor, out_d2: torch.Tensor, starts: torch.Tensor | None = None,
                           n_vox: int = 0, tile: int = 0, groups: int = 0, lookahead: int = 0, flags: int = 0,
                           shell: float = 0.0):
    """rfps_sample_batched_noalloc on torch's current stream: the batched call
    with the library's fixed scratch array as its workspace.  Every tensor
    (offsets, m, starts, outputs) must already be on the device: nothing is
    allocated and nothing waits for the device."""
    _check_xyz(xyz)
    dev = xyz.device
    for name, t, dt in (("offsets", offsets, torch.int32), ("m", m, torch.int32), ("out_idx", out_idx, torch.int32),
                        ("out_d2", out_d2, torch.float32), ("starts", starts, torch.int32)):
        if t is None and name == "starts":
            continue
        if not (isinstance(t, torch.Tensor) and t.device == dev and t.dtype == dt and t.is_contiguous()):
            raise ValueError("%s must be a contiguous %s tensor on %s" % (name, dt, dev))
    batch = offsets.numel() - 1
    p = _params(n_vox, tile, groups, flags, lookahead, shell)
    _check(lib().rfps_sample_batched_noalloc(xyz.data_ptr(), xyz.shape[0], offsets.data_ptr(), m.data_ptr(),
                                             0 if starts is None else starts.data_ptr(), batch, int(m_total),
                                             ctypes.byref(p), out_idx.data_ptr(), out_d2.data_ptr(), _stream(dev)),
           "rfps_sample_batched_noalloc")
    return out_idx, out_d2


def noalloc_scratch_bytes() -> int:
    return int(lib().rfps_noalloc_scratch_bytes())


def batched_read_status(ws: BatchWorkspace) -> int:
    return int(lib().rfps_batched_read_status(ws.ptr, ws.nbytes, _stream(ws.device)))


def batched_read_telemetry(ws: BatchWorkspace) -> dict:
    t = rfps_telemetry()
    _check(lib().rfps_batched_read_telemetry(ws.ptr, ws.nbytes, _stream(ws.device), ctypes.byref(t)),
           "rfps_batched_read_telemetry")
    return t.as_dict()


def autotune_batched(xyz: torch.Tensor, offsets, m, starts=None, n_vox: int = 0, tile: int = 0,
                     groups: int = 0, lookahead: int = 0, flags: int = 0, reps: int = 3,
                     ws: BatchWorkspace | None = None):
    """rfps_autotune_batched: returns ({n_vox, tile, groups, lookahead, flags}, median ms, (idx, d2))."""
    _check_xyz(xyz)
    dev = xyz.device
    n = xyz.shape[0]
    m_host = [int(v) for v in (m.tolist() if isinstance(m, torch.Tensor) else m)]
    m_total = sum(m_host)
    offsets_d, m_d = _i32_dev(offsets, dev), _i32_dev(m_host, dev)
    starts_d = None if starts is None else _i32_dev(starts, dev)
    batch = offsets_d.numel() - 1
    if ws is None or not ws.fits(n, batch, n_vox):
        ws = BatchWorkspace(n, batch, dev, n_vox=n_vox)
    out_idx = torch.empty(m_total, dtype=torch.int32, device=dev)
    out_d2 = torch.empty(m_total, dtype=torch.float32, device=dev)
    base = _params(n_vox, tile, groups, flags, lookahead)
    best = rfps_params()
    ms = ctypes.c_float(0.0)
    _check(lib().rfps_autotune_batched(xyz.data_ptr(), n, offsets_d.data_ptr(), m_d.data_ptr(),
                                       0 if starts_d is None else starts_d.data_ptr(), batch, m_total,
                                       ctypes.byref(base), int(reps), ws.ptr, ws.nbytes, out_idx.data_ptr(),
                                       out_d2.data_ptr(), _stream(dev), ctypes.byref(best), ctypes.byref(ms)),
           "rfps_autotune_batched")
    chosen = {k: int(getattr(best, k)) for k, _ in rfps_params._fields_}
    return chosen, float(ms.value), (out_idx, out_d2)


# ---------------------------------------------------------------------------
# Voxel-parameter network (include/rfps_mlp.h)
# ---------------------------------------------------------------------------
MLP_INPUTS, MLP_OUTPUTS, MLP_CANDIDATES, MLP_PARAMS = 516, 72, 36, 41928


def mlp_candidate(k: int):
    """(n_vox, shell spacing) of candidate k."""
    nv = ctypes.c_int32(0)
    sh = ctypes.c_float(0.0)
    if lib().rfps_mlp_candidate(int(k), ctypes.byref(nv), ctypes.byref(sh)) != 0:
        raise ValueError("candidate out of range")
    return int(nv.value), float(sh.value)


class MLP:
    """Model state and a workspace for up to `rows` rows, in device memory."""

    def __init__(self, device, rows: int = 1):
        L = lib()
        self.device = device
        self.state_bytes = int(L.rfps_mlp_state_size())
        self.state, self.state_ptr = _workspace(self.state_bytes, device)
        self.rows = 0
        self._reserve(max(1, int(rows)))

    def _reserve(self, rows: int):
        if rows <= self.rows:
            return
        nbytes = int(lib().rfps_mlp_workspace_size(int(rows)))
        if nbytes == 0:
            raise RfpsError(1, "rfps_mlp_workspace_size")
        self.ws, self.ws_ptr = _workspace(nbytes, self.device)
        self.ws_bytes, self.rows = nbytes, int(rows)

    def load(self, params):
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        if p.size != MLP_PARAMS:
            raise ValueError("expected %d parameters" % MLP_PARAMS)
        _check(lib().rfps_mlp_load(self.state_ptr, self.state_bytes, p.ctypes.data, _stream(self.device)),
               "rfps_mlp_load")

    def save(self):
        import numpy as np
        p = np.empty(MLP_PARAMS, dtype=np.float32)
        _check(lib().rfps_mlp_save(self.state_ptr, self.state_bytes, p.ctypes.data, _stream(self.device)),
               "rfps_mlp_save")
        return p

    def features(self, xyz: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        _check_xyz(xyz)
        if out is None:
            out = torch.empty(MLP_INPUTS, dtype=torch.float32, device=self.device)
        _check(lib().rfps_mlp_features(xyz.data_ptr(), xyz.shape[0], self.ws_ptr, self.ws_bytes, out.data_ptr(),
                                       _stream(self.device)), "rfps_mlp_features")
        return out

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        x = x.reshape(-1, MLP_INPUTS).contiguous()
        self._reserve(x.shape[0])
        y = torch.empty(x.shape[0], MLP_OUTPUTS, dtype=torch.float32, device=self.device)
        _check(lib().rfps_mlp_forward(self.state_ptr, self.state_bytes, x.data_ptr(), x.shape[0], self.ws_ptr,
                                      self.ws_bytes, y.data_ptr(), _stream(self.device)), "rfps_mlp_forward")
        return y

    def gradient(self, x, t, w=None):
        x = x.reshape(-1, MLP_INPUTS).contiguous()
        self._reserve(x.shape[0])
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check(lib().rfps_mlp_gradient(self.state_ptr, self.state_bytes, x.data_ptr(), t.data_ptr(),
                                       0 if w is None else w.data_ptr(), x.shape[0], self.ws_ptr, self.ws_bytes,
                                       g.data_ptr(), loss.data_ptr(), _stream(self.device)), "rfps_mlp_gradient")
        return g, loss

    def train_step(self, x, t, w=None, lr: float = 1e-3, loss: torch.Tensor | None = None):
        x = x.reshape(-1, MLP_INPUTS)
        self._reserve(x.shape[0])
        _check(lib().rfps_mlp_train_step(self.state_ptr, self.state_bytes, x.data_ptr(), t.data_ptr(),
                                         0 if w is None else w.data_ptr(), x.shape[0], float(lr), self.ws_ptr,
                                         self.ws_bytes, 0 if loss is None else loss.data_ptr(),
                                         _stream(self.device)), "rfps_mlp_train_step")

    def choose(self, feat: torch.Tensor, default_cand: int, margin: float = 0.0):
        """(chosen candidate, predictions [72]) -- waits for the device."""
        choice = torch.empty(1, dtype=torch.int32, device=self.device)
        y = torch.empty(MLP_OUTPUTS, dtype=torch.float32, device=self.device)
        _check(lib().rfps_mlp_choose(self.state_ptr, self.state_bytes, feat.data_ptr(), int(default_cand),
                                     float(margin), self.ws_ptr, self.ws_bytes, choice.data_ptr(), y.data_ptr(),
                                     _stream(self.device)), "rfps_mlp_choose")
        return int(choice.item()), y
