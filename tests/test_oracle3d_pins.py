"""Pins of the 3-D oracle (the method of Sec. III with a third axis, the paper's 3-D future
work): the literal real-vector construction with three axis vectors, reduction to the pinned
2-D oracle when the third axis carries no phase, invariance under a permutation of the axes,
unit self-similarity, the direct double sum, textbook ball counts and the entropy closed form."""
import numpy as np
import pytest

import oracle
from paper_2408_09066_amd import synth


def real_axis(theta_col):
    v = np.fft.ifft(np.exp(1j * theta_col))
    assert np.max(np.abs(v.imag)) < 1e-14
    return v.real


def location3(axes, p, ell):
    spec = np.ones(axes[0].shape[0], complex)
    for a, x in zip(axes, p):
        spec = spec * np.fft.fft(a) ** (x / ell)
    v = np.fft.ifft(spec)
    assert np.max(np.abs(v.imag)) < 1e-12
    return v.real


def tiny3(seed, D=48, ell=0.5, npts=14, tiles=(2, 1, 2), ext=1.5):
    rng = np.random.default_rng(seed)
    th = synth.make_theta3(D, ell, rng)
    xyz = rng.uniform(-ext, ext, size=(npts, 3)).astype(np.float32)
    lab = rng.integers(0, 2, size=npts).astype(np.uint8)
    return th, xyz, lab, (-ext, -ext, -ext, ext, ext, ext), tiles


@pytest.mark.parametrize("seed,tiles", [(0, (1, 1, 1)), (1, (2, 1, 2)), (2, (2, 2, 2))])
def test_matches_real_vector_construction(seed, tiles):
    D, ell = 48, 0.5
    th, xyz, lab, layout, tiles = tiny3(seed, D=D, ell=ell, tiles=tiles)
    axes = [real_axis(th[:, a] * ell) for a in range(3)]
    omega, bad = oracle.encode3(th, layout, tiles, xyz, lab)
    assert bad == 0
    grid, nx, ny, nz = (-1.5, -1.5, -1.5, 0.75), 4, 4, 4
    P = oracle.similarity3(th, layout, tiles, omega, grid, nx, ny, nz)
    beta = oracle.assign_tiles3(layout, tiles, xyz.astype(np.float64))
    mem = np.zeros((oracle.num_memories3(tiles), D))
    for p, b, psi in zip(xyz.astype(np.float64), beta, lab):
        mem[2 * b + psi] += location3(axes, p, ell)
    for l in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = np.array([grid[0] + (i + .5) * grid[3], grid[1] + (j + .5) * grid[3], grid[2] + (l + .5) * grid[3]])
                b = oracle.assign_tiles3(layout, tiles, c[None, :])[0]
                phi = location3(axes, c, ell)
                for psi in range(2):
                    w = mem[2 * b + psi]
                    nw = np.linalg.norm(w)
                    e = 0.0 if nw == 0 else np.dot(w / nw, phi)
                    assert abs(P[psi, l, j, i] - e) < 1e-10


def test_reduces_to_two_dimensions():
    """No phase on z and one tile along z: every z slice is the 2-D map of (x, y)."""
    rng = np.random.default_rng(4)
    D, ell = 64, 0.4
    th2 = synth.make_theta(D, ell, rng)
    th3 = np.zeros((D, 3))
    th3[:, :2] = th2
    xyz = np.c_[rng.uniform(-2, 2, size=(40, 2)), rng.uniform(0, 1, size=40)].astype(np.float32)
    lab = rng.integers(0, 2, size=40).astype(np.uint8)
    om3, _ = oracle.encode3(th3, (-2, -2, 0, 2, 2, 1), (2, 2, 1), xyz, lab)
    om2, _ = oracle.encode(th2, (-2, -2, 2, 2), (2, 2), xyz[:, :2].copy(), lab)
    assert np.max(np.abs(om3 - om2)) < 1e-10
    P3 = oracle.similarity3(th3, (-2, -2, 0, 2, 2, 1), (2, 2, 1), om3, (-2, -2, 0, 0.5), 8, 8, 2)
    P2 = oracle.similarity(th2, (-2, -2, 2, 2), (2, 2), om2, (-2, -2, 0.5), 8, 8)
    for l in range(2):
        assert np.max(np.abs(P3[:, l] - P2)) < 1e-12


def test_axis_permutation_invariance():
    """Relabelling the axes (x, y, z) -> (y, z, x) relabels the voxels and nothing else."""
    th, xyz, lab, layout, tiles = tiny3(9, D=64, tiles=(2, 3, 1))
    grid, n = (-1.5, -1.5, -1.5, 0.5), (6, 6, 6)
    om, _ = oracle.encode3(th, layout, tiles, xyz, lab)
    P = oracle.similarity3(th, layout, tiles, om, grid, *n)
    perm = [1, 2, 0]
    thp = th[:, perm]
    xyzp = np.ascontiguousarray(xyz[:, perm])
    layp = tuple(layout[a] for a in perm) + tuple(layout[3 + a] for a in perm)
    tilesp = tuple(tiles[a] for a in perm)
    omp, _ = oracle.encode3(thp, layp, tilesp, xyzp, lab)
    Pp = oracle.similarity3(thp, layp, tilesp, omp, grid, *n)
    # P[psi][z][y][x]; in the permuted problem axis 0 is old y, axis 1 old z, axis 2 old x
    assert np.max(np.abs(Pp - P.transpose(0, 3, 1, 2))) < 1e-12


def test_self_similarity_and_direct_sum():
    th, xyz, lab, layout, tiles = tiny3(3, D=128, tiles=(1, 1, 1))
    grid = (-1.5, -1.5, -1.5, 0.25)
    one = np.array([[-1.5 + 2.5 * 0.25, -1.5 + 3.5 * 0.25, -1.5 + 7.5 * 0.25]], np.float32)
    om, _ = oracle.encode3(th, layout, tiles, one, np.array([1], np.uint8))
    P = oracle.similarity3_cells(th, layout, tiles, om, grid, 12, 12, np.array([(7 * 12 + 3) * 12 + 2]))
    assert abs(P[1, 0] - 1.0) < 1e-12 and P[0, 0] == 0.0
    om, _ = oracle.encode3(th, layout, tiles, xyz, lab)
    cells = np.array([5, 77, 300, 1000])
    P = oracle.similarity3_cells(th, layout, tiles, om, grid, 12, 12, cells)
    for q, c in enumerate(cells):
        i, j, l = c % 12, (c // 12) % 12, c // 144
        cc = np.array([grid[0] + (i + .5) * grid[3], grid[1] + (j + .5) * grid[3], grid[2] + (l + .5) * grid[3]])
        for psi in range(2):
            pts = xyz[lab == psi].astype(np.float64)
            s = np.cos((th @ (cc[:, None] - pts.T))).sum()
            w = om[psi, :, 0] + 1j * om[psi, :, 1]
            nrm = np.sqrt(np.sum(np.abs(w) ** 2) / th.shape[0])
            assert abs(P[psi, q] - s / (th.shape[0] * nrm)) < 1e-10


@pytest.mark.parametrize("r,count", [(0, 1), (1, 7), (2, 33), (3, 123), (4, 257)])
def test_ball_counts(r, count):
    assert oracle.ball_count(r) == count
    g = np.arange(-r, r + 1)
    assert int(np.sum(g[:, None, None] ** 2 + g[None, :, None] ** 2 + g[None, None, :] ** 2 <= r * r)) == count


def test_entropy_closed_form_and_borders():
    """Q = 1/e everywhere gives H = |ball|/e inside and in-volume neighbours only at borders."""
    nx, ny, nz, r = 9, 8, 7, 2
    P = np.full((2, nz, ny, nx), 1.0)
    P[:, 0, 0, 0] = np.sqrt(np.e)          # the maximum; elsewhere Q = 1/e
    m, H, ogm, lab = oracle.postprocess3(P, r, r, 0.0)
    assert np.allclose(m, np.sqrt(np.e))
    q = 1.0 / np.e
    assert abs(H[1, 3, 4, 4] - oracle.ball_count(r) * (-q * np.log(q))) < 1e-12
    # a corner voxel sees the in-volume part of the ball only
    g = np.arange(-r, r + 1)
    inside = [(dx, dy, dz) for dx in g for dy in g for dz in g
              if dx * dx + dy * dy + dz * dz <= r * r and dx >= 0 and dy >= 0 and dz >= 0]
    expect = sum(0.0 if (dx, dy, dz) == (0, 0, 0) else -q * np.log(q) for dx, dy, dz in inside)
    assert abs(H[0, 0, 0, 0] - expect) < 1e-12
    assert np.allclose(ogm, 0.0) and np.all(lab == 1)


def test_tile_assignment_bruteforce_and_ties():
    layout, tiles = (-2.0, -1.0, 0.0, 2.0, 1.0, 3.0), (4, 2, 3)
    rng = np.random.default_rng(11)
    pts = np.r_[rng.uniform([-3, -2, -1], [3, 2, 4], size=(300, 3)),
                [[0.0, 0.0, 1.0], [-1.0, 0.0, 2.0], [1.0, 0.0, 0.0]]]   # exact ties between centres
    got = oracle.assign_tiles3(layout, tiles, pts)
    cen = np.array([oracle.tile_center3(layout, tiles, b) for b in range(24)])
    d2 = ((pts[:, None, :] - cen[None, :, :]) ** 2).sum(-1)
    assert np.array_equal(got, np.argmin(d2, axis=1))   # argmin takes the lowest index on ties
