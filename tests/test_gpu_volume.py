"""Volumes (3-D) on the GPU against the 3-D FP64 oracle.

Bars as for plane maps: heatmaps within relative L2 1e-4 per class with the bf16 hi+lo operands
(single-rounding bf16 / fp16 within their mantissa bounds), class maxima within 1e-4 and equal
to the heatmap's own maxima, labels >= 99.9 % with every disagreement where the oracle's
|OGM - rho| < 1e-3; ball-mask classification of the oracle's own similarities within 1e-4."""
import functools
import sys

import numpy as np
import pytest

import oracle
from paper_2408_09066_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"bf16x3": 1e-4, "bf16": 2e-2, "fp16": 3e-3}


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


def eight_tiles():
    """room3d re-tiled 2 x 2 x 2 (two tile layers along z)."""
    v = synth.volume("room3d")
    v.tiles = (2, 2, 2)
    v.name = "room3d_222"
    return v


@functools.lru_cache(maxsize=None)
def oracle_volume(name):
    v = synth.volume("room3d") if name == "room3d" else eight_tiles()
    return v, oracle.pipeline3(v)


def gpu_volume(torch, v, precision):
    from paper_2408_09066_amd import native
    vol = native.Volume(v.theta, v.layout, v.tiles)
    vol.encode(torch.from_numpy(v.xyz).cuda(), torch.from_numpy(v.label).cuda())
    heat, hmax = vol.decode(v.grid, v.nx, v.ny, v.nz, precision)
    ogm, lab = native.classify3(heat, hmax, v.r_occ, v.r_emp, v.rho)
    torch.cuda.synchronize()
    out = dict(heat=heat.cpu().numpy().astype(np.float64), hmax=hmax.cpu().numpy().astype(np.float64),
               ogm=ogm.cpu().numpy().astype(np.float64), label=lab.cpu().numpy(), rejected=vol.take_rejected())
    vol.close()
    return out


@pytest.mark.parametrize("precision", ["bf16x3", "bf16", "fp16"])
@pytest.mark.parametrize("name", ["room3d", "room3d_222"])
def test_volume_pipeline_matches_oracle(torch_cuda, name, precision):
    v, (om, P, m, H, ogm, lab) = oracle_volume(name)
    g = gpu_volume(torch_cuda, v, precision)
    assert g["rejected"] == 0
    for psi in range(2):
        e = np.linalg.norm(g["heat"][psi] - P[psi]) / np.linalg.norm(P[psi])
        say(f"[gpu] volume {name} {precision} heat[{psi}] rel-L2 {e:.3e} max-abs {np.max(np.abs(g['heat'][psi] - P[psi])):.2e}")
        assert e <= TOL[precision]
        assert abs(g["hmax"][psi] - m[psi]) <= 2 * TOL[precision] * abs(m[psi])
        assert g["hmax"][psi] == np.max(g["heat"][psi])
    agree = float(np.mean(g["label"] == lab))
    say(f"  labels agree {agree * 100:.4f}%")
    if precision == "bf16x3":
        bad = g["label"] != lab
        assert agree >= 0.999
        assert not bad.any() or np.max(np.abs(ogm[bad] - v.rho)) < 1e-3
    else:
        assert agree >= 0.98


@pytest.mark.parametrize("radii", [(1, 1), (2, 1), (0, 3), (5, 2)])   # (5, 2): the two-pass path
def test_classify3_on_oracle_heat(torch_cuda, radii):
    from paper_2408_09066_amd import native
    torch = torch_cuda
    v, (om, P, m, H, ogm, lab) = oracle_volume("room3d")
    P32 = P.astype(np.float32)
    m_ref, _, ogm_ref, lab_ref = oracle.postprocess3(P32.astype(np.float64), radii[0], radii[1], 0.0)
    o, l = native.classify3(torch.from_numpy(P32).cuda(), torch.from_numpy(m_ref.astype(np.float32)).cuda(),
                            radii[0], radii[1], 0.0)
    torch.cuda.synchronize()
    o = o.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(o - ogm_ref)) < 1e-4
    bad = l.cpu().numpy() != lab_ref
    assert not bad.any() or np.max(np.abs(ogm_ref[bad])) < 1e-5


def test_volume_errors(torch_cuda):
    from paper_2408_09066_amd import native
    torch = torch_cuda
    v = synth.volume("room3d")
    vol = native.Volume(v.theta, v.layout, v.tiles)
    with pytest.raises(native.VsaogmError):
        vol.decode(v.grid, v.nx, v.ny, v.nz, "fp32")
    bad_theta = v.theta.copy()
    bad_theta[3, 2] += 1.0
    with pytest.raises(native.VsaogmError):
        native.Volume(bad_theta, v.layout, v.tiles)
    lab = v.label.copy()
    lab[:5] = 7
    vol.encode(torch.from_numpy(v.xyz).cuda(), torch.from_numpy(lab).cuda())
    assert vol.take_rejected() == 5
    with pytest.raises(native.VsaogmError):
        vol.decode(v.grid, 0, v.ny, v.nz, "bf16x3")                     # empty grid
    with pytest.raises(native.VsaogmError):
        vol.decode((v.grid[0], v.grid[1], v.grid[2], -0.1), v.nx, v.ny, v.nz, "bf16x3")   # negative res
    heat, hmax = vol.decode(v.grid, v.nx, v.ny, v.nz, "bf16x3")
    with pytest.raises(native.VsaogmError):
        native.classify3(heat, hmax, 25, 1, 0.0)                          # radius above the maximum
    torch.cuda.synchronize()
    vol.close()


def test_volume_wide_phases_and_padded_spectrum(torch_cuda):
    """One tile over the room with l = 0.05 m: local phases beyond 64 revolutions take the
    double-precision phase path of the encode; D = 200 pads the half spectrum (100 bins) to
    128."""
    v = synth.volume("room3d", D=200, ell=0.05, tiles=(1, 1, 1))
    v.name = "room3d_wide"
    centre = np.array(oracle.tile_center3(v.layout, v.tiles, 0))
    rev_per_m = np.abs(v.theta[: v.D // 2]).max(axis=0) / (2 * np.pi)
    reach = (np.abs(v.xyz.astype(np.float64) - centre) @ rev_per_m).max()
    assert reach > 64.0          # the encode's single-precision bound is exceeded
    _, P, m, H, ogm, lab = oracle.pipeline3(v)
    g = gpu_volume(torch_cuda, v, "bf16x3")
    for p in range(2):
        e = np.linalg.norm(g["heat"][p] - P[p]) / np.linalg.norm(P[p])
        say(f"[gpu] volume {v.name} heat[{p}] rel-L2 {e:.3e} (phase reach {reach:.0f} rev)")
        assert e <= 1e-4
    agree = float(np.mean(g["label"] == lab))
    assert agree >= 0.999
    bad = g["label"] != lab
    assert not bad.any() or np.max(np.abs(ogm[bad] - v.rho)) < 1e-3


def test_volume_empty_and_one_point(torch_cuda):
    """An empty volume decodes to zero heat and maxima (OGM 0, occupied at rho = 0); one point
    has unit self-similarity at its own voxel centre and leaves the other class empty."""
    from paper_2408_09066_amd import native
    torch = torch_cuda
    v = synth.volume("room3d")
    vol = native.Volume(v.theta, v.layout, v.tiles)
    vol.encode(torch.zeros((0, 3), dtype=torch.float32, device="cuda"),
               torch.zeros(0, dtype=torch.uint8, device="cuda"))
    heat, hmax = vol.decode(v.grid, v.nx, v.ny, v.nz, "bf16x3")
    ogm, lab = native.classify3(heat, hmax, v.r_occ, v.r_emp, 0.0)
    torch.cuda.synchronize()
    assert torch.all(heat == 0) and torch.all(hmax == 0)
    assert torch.all(ogm == 0) and torch.all(lab == 1)
    x0, y0, z0, res = v.grid
    i, j, l = 5, 9, 3
    c = [x0 + (i + 0.5) * res, y0 + (j + 0.5) * res, z0 + (l + 0.5) * res]
    vol.encode(torch.tensor([c], dtype=torch.float32, device="cuda"),
               torch.tensor([1], dtype=torch.uint8, device="cuda"))
    heat, hmax = vol.decode(v.grid, v.nx, v.ny, v.nz, "bf16x3")
    torch.cuda.synchronize()
    assert abs(float(heat[1, l, j, i]) - 1.0) < 1e-5
    assert abs(float(hmax[1]) - 1.0) < 1e-5
    assert torch.all(heat[0] == 0)
    vol.close()


def test_volume_reset(torch_cuda):
    """A reset volume re-encoded with the same points decodes as a fresh one (same grid cache,
    same kernels, so bit-identical)."""
    from paper_2408_09066_amd import native
    torch = torch_cuda
    v = synth.volume("room3d")
    xyz, lab = torch.from_numpy(v.xyz).cuda(), torch.from_numpy(v.label).cuda()
    vol = native.Volume(v.theta, v.layout, v.tiles)
    vol.encode(xyz, lab)
    h1, m1 = vol.decode(v.grid, v.nx, v.ny, v.nz, "bf16x3")
    h1, m1 = h1.clone(), m1.clone()
    vol.encode(xyz[::2].contiguous(), lab[::2].contiguous())   # memories now differ
    vol.reset()
    vol.encode(xyz, lab)
    h2, m2 = vol.decode(v.grid, v.nx, v.ny, v.nz, "bf16x3")
    torch.cuda.synchronize()
    assert torch.equal(h1, h2) and torch.equal(m1, m2)
    vol.close()


def test_volume_fullsize_sampled(torch_cuda):
    """The 3-D benchmark volume (480 000 points, D = 4096, 128 x 128 x 32) at 1 000 seeded voxels of
    one tile: the oracle encodes only that tile's points (its memories depend on nothing else)."""
    from paper_2408_09066_amd import native
    torch = torch_cuda
    v = synth.volume("hall3d")
    vol = native.Volume(v.theta, v.layout, v.tiles)
    vol.encode(torch.from_numpy(v.xyz).cuda(), torch.from_numpy(v.label).cuda())
    heat, hmax = vol.decode(v.grid, v.nx, v.ny, v.nz, "bf16x3")
    torch.cuda.synchronize()
    heat = heat.cpu().numpy()
    hmax = hmax.cpu().numpy()
    vol.close()
    for p in range(2):
        assert hmax[p] == heat[p].max()
    beta = oracle.assign_tiles3(v.layout, v.tiles, v.xyz)
    tile = int(np.argmin(np.bincount(beta, minlength=v.tiles[0] * v.tiles[1] * v.tiles[2])))
    sel = beta == tile
    omega, bad = oracle.encode3(v.theta, v.layout, v.tiles, v.xyz[sel], v.label[sel])
    assert bad == 0
    rng = np.random.default_rng(np.random.SeedSequence([2408, 32, 7]))
    cand = rng.choice(v.nx * v.ny * v.nz, size=40_000, replace=False)
    i, j, l = cand % v.nx, (cand // v.nx) % v.ny, cand // (v.nx * v.ny)
    gx, gy, gz, res = v.grid
    cb = oracle.assign_tiles3(v.layout, v.tiles, np.stack([gx + (i + .5) * res, gy + (j + .5) * res, gz + (l + .5) * res], 1))
    cells = cand[cb == tile][:1000]
    assert len(cells) == 1000
    P = oracle.similarity3_cells(v.theta, v.layout, v.tiles, omega, v.grid, v.nx, v.ny, cells)
    for p in range(2):
        g = heat[p].reshape(-1)[cells].astype(np.float64)
        e = np.linalg.norm(g - P[p]) / np.linalg.norm(P[p])
        say(f"[gpu] hall3d tile {tile} heat[{p}] sampled rel-L2 {e:.3e}")
        assert e <= 1e-4


@pytest.mark.parametrize("precision", ["bf16x3", "bf16", "fp16"])
def test_volume_ragged_grids(torch_cuda, precision):
    """The joint (z, y) row table is stored in blocks of 32 rows: volumes whose joint row count
    is not a multiple of 32 and whose (z, y) bands start inside a block, and a single voxel,
    each against the oracle's similarity of the same memories (every voxel within the format's
    bar of the volume's peak magnitude; relative L2 where the grid has at least 256 voxels)."""
    from paper_2408_09066_amd import native
    torch = torch_cuda
    v, (om, P, m, H, ogm, lab) = oracle_volume("room3d_222")
    vol = native.Volume(v.theta, v.layout, v.tiles)
    vol.encode(torch.from_numpy(v.xyz).cuda(), torch.from_numpy(v.label).cuda())
    x0, y0, z0, res = v.grid
    cases = [((x0 + 0.013, y0 + 0.031, z0 + 0.017, res), 13, 21, 5),
             ((x0 + 0.11, y0 + 0.07, z0 + 0.05, 0.9 * res), 29, 7, 11),
             ((x0, y0, z0, res), 1, 1, 1)]
    peak = [float(np.max(np.abs(P[psi]))) for psi in range(2)]
    for grid, nx, ny, nz in cases:
        heat, hmax = vol.decode(grid, nx, ny, nz, precision)
        torch.cuda.synchronize()
        ref = oracle.similarity3(v.theta, v.layout, v.tiles, om, grid, nx, ny, nz)
        got = heat.cpu().numpy().astype(np.float64)
        for psi in range(2):
            mab = float(np.max(np.abs(got[psi] - ref[psi])))
            say(f"[gpu] volume grid {nx}x{ny}x{nz} {precision} heat[{psi}] max-abs {mab:.2e}")
            assert mab <= TOL[precision] * peak[psi], (grid, psi, mab)
            if nx * ny * nz >= 256:
                assert np.linalg.norm(got[psi] - ref[psi]) / np.linalg.norm(ref[psi]) <= TOL[precision]
            assert hmax.cpu().numpy()[psi] == np.max(got[psi])
    vol.close()
