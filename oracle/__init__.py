"""Python entry points of the FP64 CPU oracle (test infrastructure only).

Loads ``liboracle.so`` built from ``vsaogm_oracle.c`` (plain C, double precision, no code
shared with the GPU library).  Only tests, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  See the C file's header for the method passages each
function follows and for the readings of points the paper leaves open.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vsaogm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, -O2 -fopenmp, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.vo_tile_center.argtypes = [P, P, i32, P, P]
        L.vo_assign_tile.argtypes = [P, P, f64, f64]
        L.vo_assign_tile.restype = i32
        L.vo_assign_tiles.argtypes = [P, P, P, i64, P]
        L.vo_num_memories.argtypes = [P]
        L.vo_num_memories.restype = i64
        L.vo_encode.argtypes = [i32, P, P, P, P, P, i64, P]
        L.vo_encode.restype = i64
        L.vo_norm.argtypes = [i32, P]
        L.vo_norm.restype = f64
        L.vo_similarity.argtypes = [i32, P, P, P, P, P, i32, i32, P]
        L.vo_similarity_cells.argtypes = [i32, P, P, P, P, P, i32, P, i64, P]
        L.vo_disk_count.argtypes = [i32]
        L.vo_disk_count.restype = i64
        L.vo_postprocess.argtypes = [P, i32, i32, i32, i32, f64, P, P, P, P]
        L.vo_postprocess_cells.argtypes = [P, P, i64, i32, i32, P, f64, P, P, P]
        L.vo_fuse.argtypes = [i32, i64, i32, P, P, P, P]
        L.vo_postprocess_ex.argtypes = [P, i32, i32, i32, i32, f64, i32, i32, i32, P, P, P, P]
        L.vo_num_threads.restype = i32
        L.vo_set_threads.argtypes = [i32]
        L.vo3_tile_center.argtypes = [P, P, i32, P, P, P]
        L.vo3_assign_tile.argtypes = [P, P, f64, f64, f64]
        L.vo3_assign_tile.restype = i32
        L.vo3_assign_tiles.argtypes = [P, P, P, i64, P]
        L.vo3_encode.argtypes = [i32, P, P, P, P, P, i64, P]
        L.vo3_encode.restype = i64
        L.vo3_similarity_cells.argtypes = [i32, P, P, P, P, P, i32, i32, P, i64, P]
        L.vo3_ball_count.argtypes = [i32]
        L.vo3_ball_count.restype = i64
        L.vo3_postprocess.argtypes = [P, i32, i32, i32, i32, i32, f64, P, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _lay(layout, tiles):
    return (np.ascontiguousarray(layout, dtype=np.float64),
            np.ascontiguousarray(tiles, dtype=np.int32))


def num_threads() -> int:
    return int(lib().vo_num_threads())


def set_threads(n: int) -> None:
    """Host threads of the following calls (for timing; results do not depend on it)."""
    lib().vo_set_threads(int(n))


def num_memories(tiles) -> int:
    t = np.ascontiguousarray(tiles, dtype=np.int32)
    return int(lib().vo_num_memories(_p(t)))


def tile_center(layout, tiles, beta: int) -> Tuple[float, float]:
    lay, t = _lay(layout, tiles)
    mx, my = ctypes.c_double(), ctypes.c_double()
    lib().vo_tile_center(_p(lay), _p(t), int(beta), ctypes.byref(mx), ctypes.byref(my))
    return mx.value, my.value


def assign_tiles(layout, tiles, xy: np.ndarray) -> np.ndarray:
    lay, t = _lay(layout, tiles)
    pts = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    out = np.empty(pts.shape[0], dtype=np.int32)
    lib().vo_assign_tiles(_p(lay), _p(t), _p(pts), pts.shape[0], _p(out))
    return out


def new_memories(D: int, tiles) -> np.ndarray:
    return np.zeros((num_memories(tiles), D, 2), dtype=np.float64)


def encode(theta: np.ndarray, layout, tiles, xy: np.ndarray, label: np.ndarray,
           omega: Optional[np.ndarray] = None) -> Tuple[np.ndarray, int]:
    """Algorithm 1 into memories omega [2R][D][2] (complex spectra, world frame)."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    D = th.shape[0]
    lay, t = _lay(layout, tiles)
    if omega is None:
        omega = new_memories(D, tiles)
    assert omega.dtype == np.float64 and omega.flags.c_contiguous
    assert omega.shape == (num_memories(tiles), D, 2)
    pts = np.ascontiguousarray(xy, dtype=np.float32).reshape(-1, 2)
    lab = np.ascontiguousarray(label, dtype=np.uint8).reshape(-1)
    assert lab.shape[0] == pts.shape[0]
    bad = lib().vo_encode(D, _p(th), _p(lay), _p(t), _p(pts), _p(lab), pts.shape[0], _p(omega))
    return omega, int(bad)


def norm(omega_key: np.ndarray) -> float:
    w = np.ascontiguousarray(omega_key, dtype=np.float64)
    return float(lib().vo_norm(w.shape[0], _p(w)))


def similarity(theta, layout, tiles, omega, grid, nx: int, ny: int) -> np.ndarray:
    """Eq. loc-query for every cell: float64 [2][ny][nx]."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    lay, t = _lay(layout, tiles)
    g = np.ascontiguousarray(grid, dtype=np.float64)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    P = np.empty((2, ny, nx), dtype=np.float64)
    lib().vo_similarity(th.shape[0], _p(th), _p(lay), _p(t), _p(om), _p(g), nx, ny, _p(P))
    return P


def similarity_cells(theta, layout, tiles, omega, grid, nx: int, cells: np.ndarray) -> np.ndarray:
    """Eq. loc-query at flat cell indices j*nx+i: float64 [2][ncells]."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    lay, t = _lay(layout, tiles)
    g = np.ascontiguousarray(grid, dtype=np.float64)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    c = np.ascontiguousarray(cells, dtype=np.int64).reshape(-1)
    P = np.empty((2, c.shape[0]), dtype=np.float64)
    lib().vo_similarity_cells(th.shape[0], _p(th), _p(lay), _p(t), _p(om), _p(g), nx, _p(c),
                              c.shape[0], _p(P))
    return P


def disk_count(r: int) -> int:
    return int(lib().vo_disk_count(int(r)))


def postprocess(P: np.ndarray, r_occ: int, r_emp: int, rho: float):
    """Max-normalise, square, local entropy, softmax, signed difference, threshold.

    Returns (m[2], H[2][ny][nx], ogm[ny][nx], label[ny][nx])."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    _, ny, nx = P.shape
    m = np.empty(2, dtype=np.float64)
    H = np.empty((2, ny, nx), dtype=np.float64)
    ogm = np.empty((ny, nx), dtype=np.float64)
    lab = np.empty((ny, nx), dtype=np.uint8)
    lib().vo_postprocess(_p(P), nx, ny, int(r_occ), int(r_emp), float(rho), _p(m), _p(H),
                         _p(ogm), _p(lab))
    return m, H, ogm, lab


ACTIVATIONS = {"entropy": 0, "relu": 1, "tanh": 2, "sigmoid": 3}


def postprocess_ex(P: np.ndarray, r_occ: int, r_emp: int, rho: float, normalize: bool = True,
                   square: bool = True, act: str = "entropy"):
    """Decoding ablation (Sec. IV-B): (m[2], A[2][ny][nx] pre-softmax values, ogm, label)."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    _, ny, nx = P.shape
    m = np.empty(2, dtype=np.float64)
    A = np.empty((2, ny, nx), dtype=np.float64)
    ogm = np.empty((ny, nx), dtype=np.float64)
    lab = np.empty((ny, nx), dtype=np.uint8)
    lib().vo_postprocess_ex(_p(P), nx, ny, int(r_occ), int(r_emp), float(rho), int(bool(normalize)),
                            int(bool(square)), ACTIVATIONS[act], _p(m), _p(A), _p(ogm), _p(lab))
    return m, A, ogm, lab


def postprocess_cells(nb: np.ndarray, valid: np.ndarray, r_occ: int, r_emp: int,
                      m: Sequence[float], rho: float):
    """Entropy/softmax/threshold at listed cells from their similarity neighbourhoods.

    nb: float64 [ncells][2][w][w], valid: uint8 [ncells][w][w] with w = 2*max(r)+1."""
    nb = np.ascontiguousarray(nb, dtype=np.float64)
    valid = np.ascontiguousarray(valid, dtype=np.uint8)
    nc = nb.shape[0]
    mm = np.ascontiguousarray(m, dtype=np.float64)
    H = np.empty((2, nc), dtype=np.float64)
    ogm = np.empty(nc, dtype=np.float64)
    lab = np.empty(nc, dtype=np.uint8)
    lib().vo_postprocess_cells(_p(nb), _p(valid), nc, int(r_occ), int(r_emp), _p(mm),
                               float(rho), _p(H), _p(ogm), _p(lab))
    return H, ogm, lab


def fuse(omegas: Sequence[np.ndarray], present: Optional[np.ndarray] = None):
    """Algorithm 3 over agents' memory sets [nmem][D][2]; returns (fused, present)."""
    om = np.ascontiguousarray(np.stack(omegas), dtype=np.float64)
    na, nmem, D, _ = om.shape
    if present is None:
        present = np.ones((na, nmem), dtype=np.uint8)
    pr = np.ascontiguousarray(present, dtype=np.uint8)
    out = np.zeros((nmem, D, 2), dtype=np.float64)
    out_p = np.zeros(nmem, dtype=np.uint8)
    lib().vo_fuse(na, nmem, D, _p(om), _p(pr), _p(out), _p(out_p))
    return out, out_p


def pipeline(w, P_only: bool = False):
    """Whole decode of a synth.Workload: (omega, P, m, H, ogm, label)."""
    omega, bad = encode(w.theta, w.layout, w.tiles, w.xy, w.label)
    assert bad == 0
    P = similarity(w.theta, w.layout, w.tiles, omega, w.grid, w.nx, w.ny)
    if P_only:
        return omega, P
    m, H, ogm, lab = postprocess(P, w.r_occ, w.r_emp, w.rho)
    return omega, P, m, H, ogm, lab


# ---- three dimensions (the 3-D extension: Sec. III with a third axis) -----------------

def num_memories3(tiles) -> int:
    return 2 * int(tiles[0]) * int(tiles[1]) * int(tiles[2])


def tile_center3(layout, tiles, beta: int):
    lay, t = _lay(layout, tiles)
    out = [ctypes.c_double(), ctypes.c_double(), ctypes.c_double()]
    lib().vo3_tile_center(_p(lay), _p(t), int(beta), *[ctypes.byref(o) for o in out])
    return tuple(o.value for o in out)


def assign_tiles3(layout, tiles, xyz: np.ndarray) -> np.ndarray:
    lay, t = _lay(layout, tiles)
    pts = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    out = np.empty(pts.shape[0], dtype=np.int32)
    lib().vo3_assign_tiles(_p(lay), _p(t), _p(pts), pts.shape[0], _p(out))
    return out


def encode3(theta: np.ndarray, layout, tiles, xyz: np.ndarray, label: np.ndarray,
            omega: Optional[np.ndarray] = None):
    """Algorithm 1 in 3-D: memories float64 [2R][D][2] (accumulated into omega if given)."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    D = th.shape[0]
    lay, t = _lay(layout, tiles)
    if omega is None:
        omega = np.zeros((num_memories3(tiles), D, 2), dtype=np.float64)
    p = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
    lab = np.ascontiguousarray(label, dtype=np.uint8).reshape(-1)
    bad = lib().vo3_encode(D, _p(th), _p(lay), _p(t), _p(p), _p(lab), p.shape[0], _p(omega))
    return omega, int(bad)


def similarity3_cells(theta, layout, tiles, omega, grid, nx: int, ny: int, cells: np.ndarray) -> np.ndarray:
    """Eq. loc-query at flat voxel indices (l*ny + j)*nx + i: float64 [2][ncells]."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    lay, t = _lay(layout, tiles)
    g = np.ascontiguousarray(grid, dtype=np.float64)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    c = np.ascontiguousarray(cells, dtype=np.int64).reshape(-1)
    P = np.empty((2, c.shape[0]), dtype=np.float64)
    lib().vo3_similarity_cells(th.shape[0], _p(th), _p(lay), _p(t), _p(om), _p(g), int(nx), int(ny),
                               _p(c), c.shape[0], _p(P))
    return P


def similarity3(theta, layout, tiles, omega, grid, nx: int, ny: int, nz: int) -> np.ndarray:
    """Similarity of every voxel: float64 [2][nz][ny][nx]."""
    P = similarity3_cells(theta, layout, tiles, omega, grid, nx, ny, np.arange(nx * ny * nz))
    return P.reshape(2, nz, ny, nx)


def ball_count(r: int) -> int:
    return int(lib().vo3_ball_count(int(r)))


def postprocess3(P: np.ndarray, r_occ: int, r_emp: int, rho: float):
    """(m[2], H[2][nz][ny][nx], ogm[nz][ny][nx], label[nz][ny][nx]) of a whole volume."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    _, nz, ny, nx = P.shape
    m = np.empty(2, dtype=np.float64)
    H = np.empty_like(P)
    ogm = np.empty((nz, ny, nx), dtype=np.float64)
    lab = np.empty((nz, ny, nx), dtype=np.uint8)
    lib().vo3_postprocess(_p(P), nx, ny, nz, int(r_occ), int(r_emp), float(rho), _p(m), _p(H), _p(ogm), _p(lab))
    return m, H, ogm, lab


def pipeline3(v):
    """Whole 3-D decode of a synth.Volume workload: (omega, P, m, H, ogm, label)."""
    omega, bad = encode3(v.theta, v.layout, v.tiles, v.xyz, v.label)
    assert bad == 0
    P = similarity3(v.theta, v.layout, v.tiles, omega, v.grid, v.nx, v.ny, v.nz)
    m, H, ogm, lab = postprocess3(P, v.r_occ, v.r_emp, v.rho)
    return omega, P, m, H, ogm, lab
