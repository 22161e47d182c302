"""GPU parity at the edges of the method: exact ties of the nearest-tile rule, and disk radii
beyond the compile-time set of the classification kernel.

Ties (Algorithm 1; Sec. III-B vector discretization): a point or a cell centre equidistant from
two or four tile centres belongs to the lowest tile index.  Each memory below receives exactly
one point, so a single misassigned point moves a whole unit phasor into another memory and
fails the memory bar by orders of magnitude; cell centres placed exactly on the tile borders
make the same test for the decode's row and column split.

Radii (Algorithm 2): the classification kernel unrolls disks of radius <= 6 and reads larger
disks from a per-row half-width table; radii 7, 11, 12 and 24 (the largest the library
accepts) are checked against the oracle on the oracle's own heat.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2408_09066_amd import synth

pytestmark = pytest.mark.gpu


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


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


# 2 x 2 tiles on [-2, 2]^2 (centres at +-1): x = 0 and y = 0 are exact ties, (0, 0) a four-way
# tie.  By the lowest-index rule the points below fill every memory exactly once.
TIE_LAYOUT = (-2.0, -2.0, 2.0, 2.0)
TIE_POINTS = np.array([
    [0.0, 0.0],     # 4-way tie -> tile 0, occupied
    [-0.5, 0.0],    # y tie -> tile 0, empty
    [0.5, 0.0],     # y tie -> tile 1, occupied
    [1.5, 0.0],     # y tie -> tile 1, empty
    [0.0, 0.5],     # x tie -> tile 2, occupied
    [0.0, 1.5],     # x tie -> tile 2, empty
    [0.5, 0.5],     # tile 3, occupied
    [2.0, 2.0],     # layout corner -> tile 3, empty
], dtype=np.float32)
TIE_LABELS = np.array([1, 0, 1, 0, 1, 0, 1, 0], dtype=np.uint8)
TIE_GRID = (-2.0, -2.0, 0.25)
TIE_N = 16


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_exact_tile_ties(torch_cuda, precision):
    say(f"[gpu] exact tile ties, 2x2 tiles, {precision}")
    from paper_2408_09066_amd import native
    torch = torch_cuda
    D = 256
    theta = synth.make_theta(D, 0.5, synth.rng_for(77, synth.STREAM_THETA))
    beta = oracle.assign_tiles(TIE_LAYOUT, (2, 2), TIE_POINTS.astype(np.float64))
    keys = 2 * beta + TIE_LABELS
    assert sorted(keys.tolist()) == list(range(8)), keys   # the fixture fills every memory once
    om, bad = oracle.encode(theta, TIE_LAYOUT, (2, 2), TIE_POINTS, TIE_LABELS)
    assert bad == 0
    P = oracle.similarity(theta, TIE_LAYOUT, (2, 2), om, TIE_GRID, TIE_N, TIE_N)

    m = native.Map(theta, TIE_LAYOUT, (2, 2))
    m.encode(torch.from_numpy(TIE_POINTS).cuda(), torch.from_numpy(TIE_LABELS).cuda())
    heat, hmax = m.decode(TIE_GRID, TIE_N, TIE_N, precision)
    mem = m.memories()
    torch.cuda.synchronize()
    mem = mem.cpu().numpy().astype(np.float64)
    heat = heat.cpu().numpy().astype(np.float64)
    assert m.take_rejected() == 0
    m.close()
    for key in range(8):
        e = rel_l2(mem[key], om[key, :D // 2 + 1, :])
        assert e <= 1e-4, (key, e)
    for p in range(2):
        e = rel_l2(heat[p], P[p])
        say(f"  heat[{p}] rel-L2 {e:.3e}")
        assert e <= 1e-4


def test_grid_on_tile_borders(torch_cuda):
    """A grid whose cell centres include x = 0 and y = 0 exactly (cells tied between tiles),
    four points per memory: whole heatmaps against the oracle."""
    say("[gpu] cell centres on tile borders")
    from paper_2408_09066_amd import native
    torch = torch_cuda
    D = 512
    theta = synth.make_theta(D, 0.3, synth.rng_for(78, synth.STREAM_THETA))
    rng = np.random.default_rng(np.random.SeedSequence([2408, 78, 1]))
    xy = rng.uniform(-2.0, 2.0, size=(64, 2)).astype(np.float32)
    lab = (rng.uniform(size=64) < 0.5).astype(np.uint8)
    grid = (-2.125, -2.125, 0.25)     # centres -2.0, -1.75, ..., 0.0, ..., 2.0: 17 per axis
    n = 17
    cen = grid[0] + (np.arange(n) + 0.5) * grid[2]
    assert 0.0 in cen.tolist()
    om, _ = oracle.encode(theta, TIE_LAYOUT, (2, 2), xy, lab)
    P = oracle.similarity(theta, TIE_LAYOUT, (2, 2), om, grid, n, n)
    m = native.Map(theta, TIE_LAYOUT, (2, 2))
    m.encode(torch.from_numpy(xy).cuda(), torch.from_numpy(lab).cuda())
    heat, hmax = m.decode(grid, n, n, "fp32")
    torch.cuda.synchronize()
    heat = heat.cpu().numpy().astype(np.float64)
    m.close()
    for p in range(2):
        e = rel_l2(heat[p], P[p])
        say(f"  heat[{p}] rel-L2 {e:.3e}")
        assert e <= 1e-4


@pytest.mark.parametrize("radii", [(7, 7), (11, 3), (24, 0), (12, 24)])
def test_classify_large_radii(torch_cuda, radii):
    """Disk radii read from the half-width table, on the oracle's heat of the 4 x 4-tile map."""
    say(f"[gpu] classify large radii {radii}")
    from paper_2408_09066_amd import native
    torch = torch_cuda
    w = synth.workload("mini4x4")
    _, P = oracle.pipeline(w, P_only=True)
    P32 = P.astype(np.float32)
    r_occ, r_emp = radii
    m_ref, H_ref, ogm_ref, lab_ref = oracle.postprocess(P32.astype(np.float64), r_occ, r_emp, 0.0)
    heat = torch.from_numpy(P32).cuda()
    hmax = torch.from_numpy(m_ref.astype(np.float32)).cuda()
    ogm_g, lab_g = native.classify(heat, hmax, r_occ, r_emp, 0.0)
    torch.cuda.synchronize()
    ogm_g = ogm_g.cpu().numpy().astype(np.float64)
    lab_g = lab_g.cpu().numpy()
    err = float(np.max(np.abs(ogm_g - ogm_ref)))
    bad = lab_g != lab_ref
    say(f"  ogm max-abs {err:.3e}, {int(bad.sum())} label flips")
    assert err < 1e-4
    assert not bad.any() or np.max(np.abs(ogm_ref[bad])) < 1e-4
