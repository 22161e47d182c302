"""ctypes binding of ``libvsaogm.so`` (the C ABI in include/vsaogm.h).

Argument marshalling only: torch tensors provide device memory and the current HIP stream;
every step of the path runs in the library's kernels.  Loading fails loudly when the built
library is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvsaogm.so")

OK, EINVAL, ENOMEM, EDEVICE, EAGAIN, EBUSY, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2, "bf16x3": 3}

EXPORTED = [
    "vsaogm_version", "vsaogm_last_error", "vsaogm_map_create", "vsaogm_map_destroy",
    "vsaogm_map_info", "vsaogm_map_reset", "vsaogm_encode", "vsaogm_map_take_rejected",
    "vsaogm_decode", "vsaogm_classify", "vsaogm_memories", "vsaogm_fuse", "vsaogm_fuse_many",
    "vsaogm_profile_events", "vsaogm_server_create", "vsaogm_server_destroy",
    "vsaogm_server_add_map", "vsaogm_server_get_map", "vsaogm_submit", "vsaogm_poll",
    "vsaogm_wait", "vsaogm_server_drain", "vsaogm_server_stats", "vsaogm_server_memory", "vsaogm_submit_many",
    "vsaogm_classify_ex", "vsaogm_decode_incremental", "vsaogm_request_bytes",
    "vsaogm_volume_create", "vsaogm_volume_destroy", "vsaogm_volume_reset", "vsaogm_volume_encode",
    "vsaogm_volume_take_rejected", "vsaogm_volume_decode", "vsaogm_classify3",
    "vsaogm_classify3_noalloc",
]
ACTIVATIONS = {"entropy": 0, "relu": 1, "tanh": 2, "sigmoid": 3}


class VsaogmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"vsaogm error {code}: {msg}")
        self.code = code


class MapDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("theta", ctypes.c_void_p),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("x1", ctypes.c_double), ("y1", ctypes.c_double),
                ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32),
                ("device", ctypes.c_int32)]


class GridDesc(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("res", ctypes.c_double),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32)]


class VolumeDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("theta", ctypes.c_void_p),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("z0", ctypes.c_double),
                ("x1", ctypes.c_double), ("y1", ctypes.c_double), ("z1", ctypes.c_double),
                ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32), ("tiles_z", ctypes.c_int32),
                ("device", ctypes.c_int32)]


class Grid3Desc(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("z0", ctypes.c_double),
                ("res", ctypes.c_double), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32)]


def _host_out(shape, dtype):
    """Output array for a served update: in pinned memory (torch's caching host allocator) when
    a device is present, so that the server copies results into it straight from the device;
    the returned array keeps its memory alive."""
    try:
        import torch
        if torch.cuda.is_available():
            tdt = {np.dtype(np.uint8): torch.uint8, np.dtype(np.float32): torch.float32}[np.dtype(dtype)]
            return torch.empty(shape, dtype=tdt, pin_memory=True).numpy()
    except (ImportError, RuntimeError):
        pass
    return np.empty(shape, dtype=dtype)


class ServerDesc(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("max_queue", ctypes.c_int32), ("device", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("map_id", ctypes.c_int32), ("xy", ctypes.c_void_p), ("label", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("grid", GridDesc), ("precision", ctypes.c_int32),
                ("r_occ", ctypes.c_int32), ("r_emp", ctypes.c_int32), ("rho", ctypes.c_float),
                ("ogm", ctypes.c_void_p), ("label_out", ctypes.c_void_p), ("heat", ctypes.c_void_p),
                ("flags", ctypes.c_int32)]


REQUEST_LOCAL = 1


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("t_submit_ns", ctypes.c_int64), ("t_start_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64), ("hmax", ctypes.c_float * 2)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2408_09066_amd.build.build()")
    L = ctypes.CDLL(path)
    P, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    L.vsaogm_version.restype = i32
    L.vsaogm_last_error.restype = ctypes.c_char_p
    L.vsaogm_map_create.argtypes = [ctypes.POINTER(MapDesc), ctypes.POINTER(P)]
    L.vsaogm_map_destroy.argtypes = [P]
    L.vsaogm_map_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.vsaogm_map_reset.argtypes = [P, P]
    L.vsaogm_encode.argtypes = [P, P, P, i64, P]
    L.vsaogm_map_take_rejected.argtypes = [P, P, ctypes.POINTER(i64)]
    L.vsaogm_decode.argtypes = [P, ctypes.POINTER(GridDesc), i32, P, P, P]
    L.vsaogm_decode_incremental.argtypes = [P, ctypes.POINTER(GridDesc), i32, P, P, P]
    L.vsaogm_classify.argtypes = [ctypes.POINTER(GridDesc), P, P, i32, i32, f32, P, P, i32, P]
    L.vsaogm_memories.argtypes = [P, P, P]
    L.vsaogm_classify_ex.argtypes = [ctypes.POINTER(GridDesc), P, P, i32, i32, f32, i32, i32, i32,
                                     P, P, i32, P]
    L.vsaogm_fuse.argtypes = [P, P, P]
    L.vsaogm_fuse_many.argtypes = [P, ctypes.POINTER(P), ctypes.c_int32, P]
    L.vsaogm_profile_events.argtypes = [i32, P, P]
    L.vsaogm_server_create.argtypes = [ctypes.POINTER(ServerDesc), ctypes.POINTER(P)]
    L.vsaogm_server_destroy.argtypes = [P]
    L.vsaogm_server_add_map.argtypes = [P, ctypes.POINTER(MapDesc), ctypes.POINTER(i32)]
    L.vsaogm_server_get_map.argtypes = [P, i32, ctypes.POINTER(P)]
    L.vsaogm_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.vsaogm_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(Result)]
    L.vsaogm_submit_many.argtypes = [P, ctypes.POINTER(Request), i32, ctypes.POINTER(ctypes.c_uint64),
                                     ctypes.POINTER(i32)]
    L.vsaogm_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(Result)]
    L.vsaogm_server_drain.argtypes = [P]
    L.vsaogm_server_stats.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.vsaogm_server_memory.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.vsaogm_request_bytes.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(i64)]
    L.vsaogm_volume_create.argtypes = [ctypes.POINTER(VolumeDesc), ctypes.POINTER(P)]
    L.vsaogm_volume_destroy.argtypes = [P]
    L.vsaogm_volume_reset.argtypes = [P, P]
    L.vsaogm_volume_encode.argtypes = [P, P, P, i64, P]
    L.vsaogm_volume_take_rejected.argtypes = [P, P, ctypes.POINTER(i64)]
    L.vsaogm_volume_decode.argtypes = [P, ctypes.POINTER(Grid3Desc), i32, P, P, P]
    L.vsaogm_classify3.argtypes = [ctypes.POINTER(Grid3Desc), P, P, i32, i32, f32, P, P, i32, P]
    L.vsaogm_classify3_noalloc.argtypes = [ctypes.POINTER(Grid3Desc), P, P, i32, i32, f32, P, P, i32, P]
    for name in EXPORTED:
        if name not in ("vsaogm_version", "vsaogm_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(rc: int):
    if rc != OK:
        msg = load().vsaogm_last_error().decode(errors="replace")
        raise VsaogmError(rc, msg)


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _tensor(t, dtype: str, shape, name: str):
    """Check that t is a contiguous device tensor of the given dtype ("float32", "uint8") and
    shape; the kernels read and write it through a raw pointer."""
    if t is None or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if str(t.dtype) != "torch." + dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def grid_desc(grid: Tuple[float, float, float], nx: int, ny: int) -> GridDesc:
    return GridDesc(float(grid[0]), float(grid[1]), float(grid[2]), int(nx), int(ny))


class Map:
    """A set of 2*tiles_x*tiles_y memory vectors on one GPU (Sec. III-B)."""

    def __init__(self, theta: np.ndarray, layout: Sequence[float], tiles: Sequence[int],
                 device: int = 0):
        L = load()
        th = np.ascontiguousarray(theta, dtype=np.float64)
        self.D = int(th.shape[0])
        self.tiles = (int(tiles[0]), int(tiles[1]))
        self.device = int(device)
        d = MapDesc(self.D, th.ctypes.data, float(layout[0]), float(layout[1]), float(layout[2]),
                    float(layout[3]), self.tiles[0], self.tiles[1], self.device)
        h = ctypes.c_void_p()
        check(L.vsaogm_map_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.n_memories = 2 * self.tiles[0] * self.tiles[1]

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            load().vsaogm_map_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self, stream=None):
        check(load().vsaogm_map_reset(self._h, _stream(stream)))

    def encode(self, xy, label, stream=None):
        """xy: float32 [n][2] cuda tensor, label: uint8 [n] cuda tensor."""
        n = int(xy.shape[0])
        _tensor(xy, "float32", (n, 2), "xy")
        _tensor(label, "uint8", (n,), "label")
        check(load().vsaogm_encode(self._h, _ptr(xy), _ptr(label), n, _stream(stream)))

    def take_rejected(self, stream=None) -> int:
        v = ctypes.c_int64()
        check(load().vsaogm_map_take_rejected(self._h, _stream(stream), ctypes.byref(v)))
        return int(v.value)

    def decode(self, grid, nx: int, ny: int, precision: str = "fp32", heat=None, hmax=None,
               stream=None):
        import torch
        dev = torch.device("cuda", self.device)
        if heat is None:
            heat = torch.empty((2, ny, nx), dtype=torch.float32, device=dev)
        if hmax is None:
            hmax = torch.empty(2, dtype=torch.float32, device=dev)
        _tensor(heat, "float32", (2, ny, nx), "heat")
        _tensor(hmax, "float32", (2,), "hmax")
        g = grid_desc(grid, nx, ny)
        check(load().vsaogm_decode(self._h, ctypes.byref(g), PRECISIONS[precision], _ptr(heat),
                                   _ptr(hmax), _stream(stream)))
        return heat, hmax

    def decode_incremental(self, grid, nx: int, ny: int, heat, precision: str = "fp32", hmax=None,
                           stream=None):
        """Recompute only the tiles whose memories changed since the last call with this heat."""
        import torch
        if hmax is None:
            hmax = torch.empty(2, dtype=torch.float32, device=torch.device("cuda", self.device))
        _tensor(heat, "float32", (2, ny, nx), "heat")
        _tensor(hmax, "float32", (2,), "hmax")
        g = grid_desc(grid, nx, ny)
        check(load().vsaogm_decode_incremental(self._h, ctypes.byref(g), PRECISIONS[precision],
                                               _ptr(heat), _ptr(hmax), _stream(stream)))
        return heat, hmax

    def memories(self, out=None, stream=None):
        """Paper-frame memories, float32 [2R][D/2+1][2]."""
        import torch
        if out is None:
            out = torch.empty((self.n_memories, self.D // 2 + 1, 2), dtype=torch.float32,
                              device=torch.device("cuda", self.device))
        _tensor(out, "float32", (self.n_memories, self.D // 2 + 1, 2), "out")
        check(load().vsaogm_memories(self._h, _ptr(out), _stream(stream)))
        return out

    def fuse_from(self, other: "Map", stream=None):
        check(load().vsaogm_fuse(self._h, other._h, _stream(stream)))

    def fuse_many(self, others: Sequence["Map"], stream=None):
        hs = (ctypes.c_void_p * max(len(others), 1))(*[o._h for o in others])
        check(load().vsaogm_fuse_many(self._h, hs, len(others), _stream(stream)))


def classify(heat, hmax, r_occ: int, r_emp: int, rho: float = 0.0, ogm=None, label=None,
             device: int = 0, stream=None, normalize: bool = True, square: bool = True,
             act: str = "entropy"):
    import torch
    _, ny, nx = heat.shape
    dev = heat.device
    if label is None:
        label = torch.empty((ny, nx), dtype=torch.uint8, device=dev)
    if ogm is None:
        ogm = torch.empty((ny, nx), dtype=torch.float32, device=dev)
    _tensor(heat, "float32", (2, ny, nx), "heat")
    _tensor(hmax, "float32", (2,), "hmax")
    _tensor(ogm, "float32", (ny, nx), "ogm")
    _tensor(label, "uint8", (ny, nx), "label")
    g = GridDesc(0.0, 0.0, 1.0, int(nx), int(ny))
    if normalize and square and act == "entropy":
        check(load().vsaogm_classify(ctypes.byref(g), _ptr(heat), _ptr(hmax), int(r_occ),
                                     int(r_emp), float(rho), _ptr(ogm), _ptr(label), int(device),
                                     _stream(stream)))
    else:
        check(load().vsaogm_classify_ex(ctypes.byref(g), _ptr(heat), _ptr(hmax), int(r_occ),
                                        int(r_emp), float(rho), int(bool(normalize)),
                                        int(bool(square)), ACTIVATIONS[act], _ptr(ogm), _ptr(label),
                                        int(device), _stream(stream)))
    return ogm, label


def grid3_desc(grid, nx: int, ny: int, nz: int) -> Grid3Desc:
    return Grid3Desc(float(grid[0]), float(grid[1]), float(grid[2]), float(grid[3]), int(nx), int(ny), int(nz))


class Volume:
    """2*tiles_x*tiles_y*tiles_z memory vectors of a 3-D map on one GPU."""

    def __init__(self, theta: np.ndarray, layout: Sequence[float], tiles: Sequence[int], device: int = 0):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        self.D = int(th.shape[0])
        self.device = int(device)
        d = VolumeDesc(self.D, th.ctypes.data, *[float(v) for v in layout], int(tiles[0]), int(tiles[1]),
                       int(tiles[2]), self.device)
        h = ctypes.c_void_p()
        check(load().vsaogm_volume_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().vsaogm_volume_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self, stream=None):
        check(load().vsaogm_volume_reset(self._h, _stream(stream)))

    def encode(self, xyz, label, stream=None):
        n = int(xyz.shape[0])
        _tensor(xyz, "float32", (n, 3), "xyz")
        _tensor(label, "uint8", (n,), "label")
        check(load().vsaogm_volume_encode(self._h, _ptr(xyz), _ptr(label), n, _stream(stream)))

    def take_rejected(self, stream=None) -> int:
        n = ctypes.c_int64()
        check(load().vsaogm_volume_take_rejected(self._h, _stream(stream), ctypes.byref(n)))
        return int(n.value)

    def decode(self, grid, nx: int, ny: int, nz: int, precision: str = "bf16x3", heat=None, hmax=None,
               stream=None):
        import torch
        dev = torch.device("cuda", self.device)
        if heat is None:
            heat = torch.empty((2, nz, ny, nx), dtype=torch.float32, device=dev)
        if hmax is None:
            hmax = torch.empty(2, dtype=torch.float32, device=dev)
        _tensor(heat, "float32", (2, nz, ny, nx), "heat")
        _tensor(hmax, "float32", (2,), "hmax")
        g = grid3_desc(grid, nx, ny, nz)
        check(load().vsaogm_volume_decode(self._h, ctypes.byref(g), PRECISIONS[precision], _ptr(heat), _ptr(hmax),
                                          _stream(stream)))
        return heat, hmax


def classify3(heat, hmax, r_occ: int, r_emp: int, rho: float = 0.0, ogm=None, label=None, device: int = 0,
              stream=None, noalloc: bool = False):
    """noalloc: call vsaogm_classify3_noalloc (fixed per-device scratch, no device allocation)."""
    import torch
    _, nz, ny, nx = heat.shape
    if label is None:
        label = torch.empty((nz, ny, nx), dtype=torch.uint8, device=heat.device)
    if ogm is None:
        ogm = torch.empty((nz, ny, nx), dtype=torch.float32, device=heat.device)
    _tensor(heat, "float32", (2, nz, ny, nx), "heat")
    _tensor(hmax, "float32", (2,), "hmax")
    _tensor(ogm, "float32", (nz, ny, nx), "ogm")
    _tensor(label, "uint8", (nz, ny, nx), "label")
    g = Grid3Desc(0.0, 0.0, 0.0, 1.0, int(nx), int(ny), int(nz))
    fn = load().vsaogm_classify3_noalloc if noalloc else load().vsaogm_classify3
    check(fn(ctypes.byref(g), _ptr(heat), _ptr(hmax), int(r_occ), int(r_emp), float(rho), _ptr(ogm), _ptr(label),
             int(device), _stream(stream)))
    return ogm, label


STAGES = {"encode": 0, "decode": 1, "classify": 2}


def profile_events(stage: str, begin=None, end=None):
    """Record torch.cuda.Event objects around every launch of a stage's main kernel."""
    b = ctypes.c_void_p(begin.cuda_event if begin is not None else 0)
    e = ctypes.c_void_p(end.cuda_event if end is not None else 0)
    check(load().vsaogm_profile_events(STAGES[stage], b, e))


class ServerMap:
    """A map owned by a Server (a view for memories, decoding and fusion once the server is
    drained)."""

    def __init__(self, handle, D, n_memories, device):
        self._h, self.D, self.n_memories, self.device = handle, D, n_memories, device

    def memories(self, out=None, stream=None):
        return Map.memories(self, out, stream)

    def decode(self, grid, nx: int, ny: int, precision: str = "fp32", heat=None, hmax=None, stream=None):
        return Map.decode(self, grid, nx, ny, precision, heat, hmax, stream)


class Server:
    """The request loop of the C ABI: submit map updates, poll for their results."""

    def __init__(self, device: int = 0, max_inflight: int = 4, max_queue: int = 1024,
                 hbm_budget_bytes: int = 0, max_batch: int = 0):
        L = load()
        d = ServerDesc(int(hbm_budget_bytes), int(max_inflight), int(max_queue), int(device), int(max_batch))
        h = ctypes.c_void_p()
        check(L.vsaogm_server_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.device = int(device)
        self._keep = {}
        self._maps = {}

    def close(self):
        if getattr(self, "_h", None):
            load().vsaogm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_map(self, theta, layout, tiles) -> int:
        th = np.ascontiguousarray(theta, dtype=np.float64)
        d = MapDesc(int(th.shape[0]), th.ctypes.data, float(layout[0]), float(layout[1]),
                    float(layout[2]), float(layout[3]), int(tiles[0]), int(tiles[1]), self.device)
        mid = ctypes.c_int32()
        check(load().vsaogm_server_add_map(self._h, ctypes.byref(d), ctypes.byref(mid)))
        self._maps[mid.value] = (int(th.shape[0]), 2 * int(tiles[0]) * int(tiles[1]))
        return int(mid.value)

    def get_map(self, map_id: int) -> ServerMap:
        h = ctypes.c_void_p()
        check(load().vsaogm_server_get_map(self._h, int(map_id), ctypes.byref(h)))
        D, nmem = self._maps[map_id]
        return ServerMap(h, D, nmem, self.device)

    def submit(self, map_id: int, xy: np.ndarray, label: np.ndarray, grid, nx: int, ny: int,
               r_occ: int, r_emp: int, rho: float = 0.0, precision: str = "fp32",
               want=("label",), block_when_busy: bool = True, local: bool = False):
        """Queue one update; returns (ticket, outputs dict of numpy arrays filled on completion).
        local: decode only the tiles whose memories changed, into a heat buffer the server keeps."""
        import time
        xy = np.ascontiguousarray(xy, dtype=np.float32).reshape(-1, 2)
        label = np.ascontiguousarray(label, dtype=np.uint8).reshape(-1)
        out = {}
        if "label" in want:
            out["label"] = _host_out((ny, nx), np.uint8)
        if "ogm" in want:
            out["ogm"] = _host_out((ny, nx), np.float32)
        if "heat" in want:
            out["heat"] = _host_out((2, ny, nx), np.float32)
        req = Request(int(map_id), xy.ctypes.data, label.ctypes.data, int(xy.shape[0]),
                      grid_desc(grid, nx, ny), PRECISIONS[precision], int(r_occ), int(r_emp),
                      float(rho),
                      out["ogm"].ctypes.data if "ogm" in out else None,
                      out["label"].ctypes.data if "label" in out else None,
                      out["heat"].ctypes.data if "heat" in out else None,
                      REQUEST_LOCAL if local else 0)
        t = ctypes.c_uint64()
        while True:
            rc = load().vsaogm_submit(self._h, ctypes.byref(req), ctypes.byref(t))
            if rc == EBUSY and block_when_busy:
                time.sleep(50e-6)
                continue
            check(rc)
            break
        self._keep[t.value] = out
        return int(t.value), out

    def prepare_many(self, items, want=("label",)):
        """Build the request structs and output arrays of a list of requests (no server call).
        items: dicts with keys map_id, xy, label, grid, nx, ny, r_occ, r_emp and optionally rho,
        precision, local.  Returns an object for submit_prepared."""
        n = len(items)
        arr = (Request * n)()
        keep, outs = [], []
        for i, it in enumerate(items):
            xy = np.ascontiguousarray(it["xy"], dtype=np.float32).reshape(-1, 2)
            lab = np.ascontiguousarray(it["label"], dtype=np.uint8).reshape(-1)
            nx, ny = int(it["nx"]), int(it["ny"])
            out = {}
            if "label" in want:
                out["label"] = _host_out((ny, nx), np.uint8)
            if "ogm" in want:
                out["ogm"] = _host_out((ny, nx), np.float32)
            if "heat" in want:
                out["heat"] = _host_out((2, ny, nx), np.float32)
            keep.append((xy, lab))
            outs.append(out)
            arr[i] = Request(int(it["map_id"]), xy.ctypes.data, lab.ctypes.data, int(xy.shape[0]),
                             grid_desc(it["grid"], nx, ny), PRECISIONS[it.get("precision", "fp32")],
                             int(it["r_occ"]), int(it["r_emp"]), float(it.get("rho", 0.0)),
                             out["ogm"].ctypes.data if "ogm" in out else None,
                             out["label"].ctypes.data if "label" in out else None,
                             out["heat"].ctypes.data if "heat" in out else None,
                             REQUEST_LOCAL if it.get("local") else 0)
        return (n, arr, keep, outs)

    def submit_prepared(self, prepared):
        """Queue requests built by prepare_many with one call (inputs are staged by the server
        before it returns).  Returns [(ticket, outputs)]."""
        n, arr, _keep, outs = prepared
        tk = (ctypes.c_uint64 * max(n, 1))()
        nq = ctypes.c_int32()
        rc = load().vsaogm_submit_many(self._h, arr, n, tk, ctypes.byref(nq))
        res = []
        for i in range(nq.value):
            self._keep[int(tk[i])] = outs[i]
            res.append((int(tk[i]), outs[i]))
        check(rc)
        return res

    def submit_many(self, items, want=("label",)):
        """Queue a list of requests with one call (prepare_many + submit_prepared).
        Returns [(ticket, outputs)]."""
        return self.submit_prepared(self.prepare_many(items, want))

    def poll(self, ticket: int):
        """None while running; else a dict with status, slot, times (ns) and maxima."""
        r = Result()
        rc = load().vsaogm_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(r))
        if rc == EAGAIN:
            return None
        check(rc)
        self._keep.pop(ticket, None)
        return {"status": r.status, "slot": r.slot, "t_submit_ns": r.t_submit_ns,
                "t_start_ns": r.t_start_ns, "t_done_ns": r.t_done_ns,
                "hmax": (r.hmax[0], r.hmax[1])}

    def wait(self, ticket: int):
        r = Result()
        check(load().vsaogm_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(r)))
        self._keep.pop(ticket, None)
        return {"status": r.status, "slot": r.slot, "t_submit_ns": r.t_submit_ns,
                "t_start_ns": r.t_start_ns, "t_done_ns": r.t_done_ns,
                "hmax": (r.hmax[0], r.hmax[1])}

    def drain(self):
        check(load().vsaogm_server_drain(self._h))

    def request_bytes(self, map_id: int, n_points: int, grid, nx: int, ny: int) -> int:
        """Device bytes admission reserves for such a request."""
        req = Request(int(map_id), None, None, int(n_points), grid_desc(grid, nx, ny), 0, 0, 0, 0.0,
                      None, None, None, 0)
        b = ctypes.c_int64()
        check(load().vsaogm_request_bytes(self._h, ctypes.byref(req), ctypes.byref(b)))
        return int(b.value)

    def stats(self):
        c, p, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(load().vsaogm_server_stats(self._h, ctypes.byref(c), ctypes.byref(p), ctypes.byref(b)))
        return {"completed": c.value, "peak_bytes": p.value, "budget_bytes": b.value}

    def memory(self):
        """Budget bytes now: in flight, resident in the maps, the slots' fixed buffers; reclaims."""
        v = [ctypes.c_int64() for _ in range(4)]
        check(load().vsaogm_server_memory(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("in_flight", "resident", "fixed", "reclaims"), (x.value for x in v)))
