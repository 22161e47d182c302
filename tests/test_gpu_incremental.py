"""Localized decoding on the GPU: only tiles whose memories changed are recomputed.

Each cell reads only its own tile's memories (Sec. III-A), so after an update confined to a
few tiles the cells of every other tile keep their values.  Bars: the incremental heat and
maxima equal a full decode up to the order of the fp32 accumulation (the frequency reduction
is split among workgroups according to how many tiles are decoded): max-abs difference
<= ORDER_TOL; cells of untouched tiles are provably not rewritten (a planted sentinel
survives); and the result meets the fp32 oracle bar (relative L2 <= 1e-4).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2408_09066_amd import synth

pytestmark = pytest.mark.gpu

HEAT_TOL = 1e-4
SENTINEL = -7.0
# The absolute values of a cell's K terms sum to at most 1 (each memory is divided by its norm,
# and by Cauchy-Schwarz sum|Omega_k| <= (D/2) ||omega||), so the partial sums stay below 1 and
# a different split of the K-reduction moves a cell by a few ulps of them per split point
# (about 1e-6 measured at D = 16384 and a 4000 x 4000 grid).
ORDER_TOL = 1e-5


def same(a, b):
    """Equal up to accumulation order."""
    return bool(torch_max_abs(a, b) <= ORDER_TOL)


def torch_max_abs(a, b):
    return float((a - b).abs().max()) if a.numel() else 0.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_09066_amd import native
    native.load()
    return torch


def tile_box(w, tx, ty, frac):
    """Axis-aligned box of half-width frac * tile side around the centre of tile (tx, ty)."""
    x0, y0, x1, y1 = w.layout
    sx, sy = (x1 - x0) / w.tiles[0], (y1 - y0) / w.tiles[1]
    cx, cy = x0 + (tx + 0.5) * sx, y0 + (ty + 0.5) * sy
    return cx - frac * sx, cy - frac * sy, cx + frac * sx, cy + frac * sy


def inside(xy, box):
    return (xy[:, 0] > box[0]) & (xy[:, 0] < box[2]) & (xy[:, 1] > box[1]) & (xy[:, 1] < box[3])


def cell_in(w, box):
    """(row, col) of a grid cell whose centre lies in the box."""
    gx, gy, res = w.grid
    c = int(((box[0] + box[2]) / 2 - gx) / res)
    r = int(((box[1] + box[3]) / 2 - gy) / res)
    assert 0 <= c < w.nx and 0 <= r < w.ny
    return r, c


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("name", ["mini4x4", "ragged3x3"])
def test_incremental_equals_full(torch_cuda, name, precision):
    say(f"[gpu] incremental decode {name} {precision}")
    from paper_2408_09066_amd import native
    torch = torch_cuda
    w = synth.workload(name)
    last_t = (w.tiles[0] - 1, w.tiles[1] - 1)
    upd = tile_box(w, *last_t, 0.3)
    sel = inside(w.xy, upd)
    assert sel.sum() > 10 and (~sel).sum() > 10
    xy_all = torch.from_numpy(w.xy).cuda()
    lb_all = torch.from_numpy(w.label).cuda()
    xy_a = torch.from_numpy(np.ascontiguousarray(w.xy[~sel])).cuda()
    lb_a = torch.from_numpy(np.ascontiguousarray(w.label[~sel])).cuda()
    xy_b = torch.from_numpy(np.ascontiguousarray(w.xy[sel])).cuda()
    lb_b = torch.from_numpy(np.ascontiguousarray(w.label[sel])).cuda()

    m = native.Map(w.theta, w.layout, w.tiles)
    heat = torch.empty((2, w.ny, w.nx), dtype=torch.float32, device="cuda")
    hmax = torch.empty(2, dtype=torch.float32, device="cuda")

    def full():
        h, mx = m.decode(w.grid, w.nx, w.ny, precision)
        return h.clone(), mx.clone()

    # first call decodes every cell
    m.encode(xy_a, lb_a)
    heat.fill_(float("nan"))
    m.decode_incremental(w.grid, w.nx, w.ny, heat, precision, hmax)
    ref, ref_max = full()
    torch.cuda.synchronize()
    assert same(heat, ref) and same(hmax, ref_max)

    # an update inside one tile: a cell of the first tile is not rewritten
    r, c = cell_in(w, tile_box(w, 0, 0, 0.3))
    keep = heat[:, r, c].clone()
    ur, uc = cell_in(w, upd)
    before_u = heat[:, ur, uc].clone()
    heat[:, r, c] = SENTINEL
    m.encode(xy_b, lb_b)
    m.decode_incremental(w.grid, w.nx, w.ny, heat, precision, hmax)
    ref, ref_max = full()
    torch.cuda.synchronize()
    assert torch.all(heat[:, r, c] == SENTINEL)
    heat[:, r, c] = keep
    assert same(heat, ref) and same(hmax, ref_max)
    assert torch_max_abs(heat[:, ur, uc], before_u) > 1e-4  # the updated tile did change

    # nothing changed: nothing is recomputed, maxima stay
    heat[:, ur, uc] = SENTINEL
    m.decode_incremental(w.grid, w.nx, w.ny, heat, precision, hmax)
    torch.cuda.synchronize()
    assert torch.all(heat[:, ur, uc] == SENTINEL) and same(hmax, ref_max)
    heat[:, ur, uc] = ref[:, ur, uc]

    # the full point set against the oracle (fp32 bar)
    if precision == "fp32":
        _, P = oracle.pipeline(w, P_only=True)
        h = heat.cpu().numpy().astype(np.float64)
        for p in range(2):
            e = np.linalg.norm(h[p] - P[p]) / np.linalg.norm(P[p])
            say(f"  class {p} rel-L2 vs oracle {e:.2e}")
            assert e <= HEAT_TOL

    # a reset and a fusion mark every memory of the target as changed
    m.reset()
    m.decode_incremental(w.grid, w.nx, w.ny, heat, precision, hmax)
    torch.cuda.synchronize()
    assert torch.all(heat == 0) and torch.all(hmax == 0)
    other = native.Map(w.theta, w.layout, w.tiles)
    other.encode(xy_all, lb_all)
    m.fuse_from(other)
    m.decode_incremental(w.grid, w.nx, w.ny, heat, precision, hmax)
    ref, ref_max = full()
    torch.cuda.synchronize()
    assert same(heat, ref) and same(hmax, ref_max)

    # another heat buffer decodes every cell
    heat2 = torch.full_like(heat, float("nan"))
    m.decode_incremental(w.grid, w.nx, w.ny, heat2, precision, hmax)
    torch.cuda.synchronize()
    assert same(heat2, ref) and same(hmax, ref_max)
    other.close()
    m.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x3"])
def test_incremental_many_tiles(torch_cuda, precision):
    """A 2560 x 2560 grid of 10 x 10 memory tiles (400 GEMM tiles of 256 x 64 cells), D = 1536
    (24 K steps per tile): updates that touch 7 tile rows (about 280 GEMM tiles, more than the
    workgroups: ranges of 27 steps that split tiles anywhere in the list, also past the 256th),
    two neighbouring tiles (a few tiles split over many workgroups) and none.  The plan is made
    on the device; every result equals a full decode up to accumulation order."""
    say(f"[gpu] incremental decode, many tiles, {precision}")
    from paper_2408_09066_amd import native
    torch = torch_cuda
    rng = np.random.default_rng(2408)
    D, res, side, T = 1536, 0.05, 2560, 10
    half = side * res / 2.0
    layout = (-half, -half, half, half)
    grid = (-half, -half, res)
    theta = synth.make_theta(D, 0.25, rng)
    m = native.Map(theta, layout, (T, T))
    heat = torch.empty((2, side, side), dtype=torch.float32, device="cuda")
    hmax = torch.empty(2, dtype=torch.float32, device="cuda")

    def points(x0, y0, x1, y1, n):
        xy = np.stack([rng.uniform(x0, x1, n), rng.uniform(y0, y1, n)], 1).astype(np.float32)
        lb = rng.integers(0, 2, n).astype(np.uint8)
        return torch.from_numpy(xy).cuda(), torch.from_numpy(lb).cuda()

    def check_full(tag):
        ref, ref_max = m.decode(grid, side, side, precision)
        torch.cuda.synchronize()
        d = torch_max_abs(heat, ref)
        say(f"  {tag}: max-abs vs full decode {d:.2e}")
        assert d <= ORDER_TOL and same(hmax, ref_max)

    m.encode(*points(-half, -half, half, half, 20000))
    heat.fill_(float("nan"))
    m.decode_incremental(grid, side, side, heat, precision, hmax)
    check_full("first call (all tiles)")
    tile = 2 * half / T
    m.encode(*points(-half, -half + 2 * tile, half, -half + 9 * tile, 30000))   # tile rows 2..8
    m.decode_incremental(grid, side, side, heat, precision, hmax)
    check_full("7 tile rows")
    m.encode(*points(-half + 3 * tile, -half + 5 * tile, -half + 5 * tile, -half + 6 * tile, 5000))
    m.decode_incremental(grid, side, side, heat, precision, hmax)
    check_full("2 tiles")
    heat[:, 0, 0] = SENTINEL
    m.decode_incremental(grid, side, side, heat, precision, hmax)
    torch.cuda.synchronize()
    assert torch.all(heat[:, 0, 0] == SENTINEL)
    m.close()
