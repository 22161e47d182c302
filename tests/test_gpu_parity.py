"""GPU parity: the HIP path through the C ABI against the FP64 oracle on identical inputs.

Bars (stated once here and used below):
  memories   relative L2 error per memory        <= 1e-4
  heatmaps   relative L2 error per class map     <= 1e-4   (fp32 path)
  maxima     relative error                      <= 1e-4
  labels     agreement with the oracle            >= 99.9 %, and every disagreement lies where
             the oracle's |OGM - rho| is below 1e-3 (the fp32 heatmap error cannot move
             OGM further than that)
"""
import functools
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2408_09066_amd import synth

pytestmark = pytest.mark.gpu

MEM_TOL = 1e-4
HEAT_TOL = 1e-4
LABEL_AGREE = 0.999
MARGIN = 1e-3


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


@functools.lru_cache(maxsize=None)
def oracle_result(name):
    w = synth.workload(name)
    return w, oracle.pipeline(w)


def gpu_run(torch, w, precision="fp32", xy=None, label=None):
    from paper_2408_09066_amd import native
    m = native.Map(w.theta, w.layout, w.tiles)
    xy_t = torch.from_numpy(w.xy if xy is None else xy).cuda()
    lab_t = torch.from_numpy(w.label if label is None else label).cuda()
    m.encode(xy_t, lab_t)
    heat, hmax = m.decode(w.grid, w.nx, w.ny, precision)
    ogm, lab = native.classify(heat, hmax, w.r_occ, w.r_emp, w.rho)
    mem = m.memories()
    torch.cuda.synchronize()
    out = dict(mem=mem.cpu().numpy().astype(np.float64), heat=heat.cpu().numpy().astype(np.float64),
               hmax=hmax.cpu().numpy().astype(np.float64), ogm=ogm.cpu().numpy().astype(np.float64),
               label=lab.cpu().numpy(), rejected=m.take_rejected())
    m.close()
    return out


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def check_labels(lab_gpu, lab_ref, ogm_ref, rho):
    agree = float(np.mean(lab_gpu == lab_ref))
    bad = lab_gpu != lab_ref
    worst = float(np.max(np.abs(ogm_ref[bad] - rho))) if bad.any() else 0.0
    say(f"  labels agree {agree * 100:.4f}% ({int(bad.sum())} flips, worst oracle margin {worst:.2e})")
    assert agree >= LABEL_AGREE
    assert worst < MARGIN


# Single-rounding 16-bit operands are reported, not held to the fp32 bar: their heatmap
# error is bounded by a few units of their 8- or 11-bit mantissa.
LOOSE_TOL = {"bf16": 2e-2, "fp16": 3e-3}


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "bf16", "fp16"])
@pytest.mark.parametrize("name", ["toy_room", "mini4x4", "ragged3x3"])
def test_pipeline_matches_oracle(torch_cuda, name, precision):
    say(f"[gpu] pipeline parity {name} {precision}")
    w, (om, P, m, H, ogm, lab) = oracle_result(name)
    g = gpu_run(torch_cuda, w, precision)
    assert g["rejected"] == 0
    half = w.D // 2
    ref_mem = om[:, :half + 1, :]
    for key in range(om.shape[0]):
        e = rel_l2(g["mem"][key], ref_mem[key])
        assert e <= MEM_TOL, (key, e)
    tol = LOOSE_TOL.get(precision, HEAT_TOL)
    for psi in range(2):
        e = rel_l2(g["heat"][psi], P[psi])
        mab = float(np.max(np.abs(g["heat"][psi] - P[psi])))
        say(f"  heat[{psi}] rel-L2 {e:.3e} max-abs {mab:.3e}; max {g['hmax'][psi]:.6f} vs {m[psi]:.6f}")
        assert e <= tol
        assert abs(g["hmax"][psi] - m[psi]) <= 2 * tol * max(abs(m[psi]), 1e-30)
        assert g["hmax"][psi] == np.max(g["heat"][psi])
    say(f"  ogm max-abs {np.max(np.abs(g['ogm'] - ogm)):.3e}")
    if precision in LOOSE_TOL:
        agree = float(np.mean(g["label"] == lab))
        say(f"  labels agree {agree * 100:.4f}% (reported)")
        assert agree >= 0.98
    else:
        check_labels(g["label"], lab, ogm, w.rho)


@pytest.mark.parametrize("name", ["toy_room", "mini4x4"])
@pytest.mark.parametrize("radii", [(2, 2), (3, 1), (0, 5)])
def test_classify_on_oracle_heat(torch_cuda, name, radii):
    """The classification stage alone, fed the oracle's own similarity maps."""
    say(f"[gpu] classify parity {name} radii {radii}")
    from paper_2408_09066_amd import native
    torch = torch_cuda
    w, (om, P, m, H, ogm, lab) = oracle_result(name)
    P32 = P.astype(np.float32)
    r_occ, r_emp = radii
    m_ref, H_ref, ogm_ref, lab_ref = oracle.postprocess(P32.astype(np.float64), r_occ, r_emp, 0.0)
    heat = torch.from_numpy(P32).cuda()
    hmax = torch.from_numpy(m_ref.astype(np.float32)).cuda()
    ogm_g, lab_g = native.classify(heat, hmax, r_occ, r_emp, 0.0)
    torch.cuda.synchronize()
    ogm_g = ogm_g.cpu().numpy().astype(np.float64)
    lab_g = lab_g.cpu().numpy()
    assert np.max(np.abs(ogm_g - ogm_ref)) < 1e-4
    bad = lab_g != lab_ref
    assert not bad.any() or np.max(np.abs(ogm_ref[bad])) < 1e-5


def test_incremental_encode_and_determinism(torch_cuda):
    """Memories accumulate across calls (eq. bundling); identical runs give identical bits."""
    say("[gpu] incremental encode + determinism mini4x4")
    from paper_2408_09066_amd import native
    torch = torch_cuda
    w = synth.workload("mini4x4")
    xy = torch.from_numpy(w.xy).cuda()
    lab = torch.from_numpy(w.label).cuda()
    outs = []
    for _ in range(2):
        m = native.Map(w.theta, w.layout, w.tiles)
        m.encode(xy, lab)
        heat, hmax = m.decode(w.grid, w.nx, w.ny)
        torch.cuda.synchronize()
        outs.append(heat.cpu().numpy())
        m.close()
    assert np.array_equal(outs[0], outs[1])
    m = native.Map(w.theta, w.layout, w.tiles)
    cut = [0, 1, 5000, 5001, w.n]
    for a, b in zip(cut[:-1], cut[1:]):
        m.encode(xy[a:b].contiguous(), lab[a:b].contiguous())
    heat2, _ = m.decode(w.grid, w.nx, w.ny)
    torch.cuda.synchronize()
    assert rel_l2(heat2.cpu().numpy().astype(np.float64), outs[0].astype(np.float64)) < 1e-5
    m.close()


def test_fusion_is_union(torch_cuda):
    """Algorithm 3 on the GPU: fusing maps of disjoint point subsets equals one map of all."""
    say("[gpu] fusion mini4x4")
    from paper_2408_09066_amd import native
    torch = torch_cuda
    w, (om, P, m, H, ogm, lab) = oracle_result("mini4x4")
    xy = torch.from_numpy(w.xy).cuda()
    lb = torch.from_numpy(w.label).cuda()
    a = native.Map(w.theta, w.layout, w.tiles)
    b = native.Map(w.theta, w.layout, w.tiles)
    a.encode(xy[:7000].contiguous(), lb[:7000].contiguous())
    b.encode(xy[7000:].contiguous(), lb[7000:].contiguous())
    a.fuse_from(b)
    heat, hmax = a.decode(w.grid, w.nx, w.ny)
    torch.cuda.synchronize()
    assert rel_l2(heat.cpu().numpy().astype(np.float64)[1], P[1]) <= HEAT_TOL
    assert rel_l2(heat.cpu().numpy().astype(np.float64)[0], P[0]) <= HEAT_TOL
    bad_theta = w.theta.copy()
    bad_theta[1] *= 1.0000001
    bad_theta[-1] = -bad_theta[1]
    c = native.Map(bad_theta, w.layout, w.tiles)
    with pytest.raises(native.VsaogmError):
        a.fuse_from(c)
    for mm in (a, b, c):
        mm.close()


def test_fusion_many_agents(torch_cuda):
    """Algorithm 3 over N agents in one pass: the same bits as N pairwise fusions in that order,
    the union's memories against the oracle, more than one launch's worth of sources, a repeated
    source, no sources, and refused sources leaving the destination untouched."""
    say("[gpu] fusion of N agents mini4x4")
    from paper_2408_09066_amd import native
    torch = torch_cuda
    w, (om, P, m, H, ogm, lab) = oracle_result("mini4x4")
    xy = torch.from_numpy(w.xy).cuda()
    lb = torch.from_numpy(w.label).cuda()
    n = xy.shape[0]
    cuts = [0, n // 5, 2 * n // 5, 3 * n // 5, 4 * n // 5, n]
    agents = []
    for i in range(5):
        a = native.Map(w.theta, w.layout, w.tiles)
        a.encode(xy[cuts[i]:cuts[i + 1]].contiguous(), lb[cuts[i]:cuts[i + 1]].contiguous())
        agents.append(a)
    seq = native.Map(w.theta, w.layout, w.tiles)
    many = native.Map(w.theta, w.layout, w.tiles)
    for a in agents:
        seq.fuse_from(a)
    many.fuse_many(agents)
    m_seq, m_many = seq.memories().cpu().numpy(), many.memories().cpu().numpy()
    assert np.array_equal(m_seq.view(np.uint32), m_many.view(np.uint32))
    half = w.D // 2
    got = m_many.astype(np.float64)
    for key in range(om.shape[0]):
        assert rel_l2(got[key], om[key, :half + 1, :]) <= MEM_TOL, key
    heat, _ = many.decode(w.grid, w.nx, w.ny)
    torch.cuda.synchronize()
    for psi in range(2):
        assert rel_l2(heat.cpu().numpy().astype(np.float64)[psi], P[psi]) <= HEAT_TOL
    # 17 sources (two launches, a repeated source) and no sources
    seq.reset()
    many.reset()
    srcs = [agents[i % 5] for i in range(17)]
    for a in srcs:
        seq.fuse_from(a)
    many.fuse_many(srcs)
    many.fuse_many([])
    m_seq, m_many = seq.memories().cpu().numpy(), many.memories().cpu().numpy()
    assert np.array_equal(m_seq.view(np.uint32), m_many.view(np.uint32))
    # refused: the destination among the sources, a different Theta; nothing is added
    bad_theta = w.theta.copy()
    bad_theta[1] *= 1.0000001
    bad_theta[-1] = -bad_theta[1]
    c = native.Map(bad_theta, w.layout, w.tiles)
    with pytest.raises(native.VsaogmError):
        many.fuse_many([agents[0], many])
    with pytest.raises(native.VsaogmError):
        many.fuse_many([agents[0], c])
    after = many.memories().cpu().numpy()
    assert np.array_equal(after.view(np.uint32), m_many.view(np.uint32))
    for mm in agents + [seq, many, c]:
        mm.close()


@pytest.mark.parametrize("precision", ["bf16x3", "bf16", "fp16"])
def test_small_and_ragged_grids_16bit(torch_cuda, precision):
    """The 16-bit row tables are stored in blocks of 32 rows: grids whose row count is not a
    multiple of 32, whose tile bands start inside a block, a single cell, and a grid narrower
    than one column slice, each against the oracle's similarity of the same memories."""
    say(f"[gpu] small and ragged grids {precision}")
    from paper_2408_09066_amd import native
    torch = torch_cuda
    w, (om, P, m, H, ogm, lab) = oracle_result("mini4x4")
    mp = native.Map(w.theta, w.layout, w.tiles)
    mp.encode(torch.from_numpy(w.xy).cuda(), torch.from_numpy(w.label).cuda())
    x0, y0, res = w.grid
    cases = [((x0, y0, res), 1, 1), ((x0 + 0.35, y0 + 0.95, res), 3, 5),
             ((x0 + 1.05, y0 + 2.15, res), 70, 33), ((x0 + 0.25, y0 + 0.45, res), 65, 97),
             ((x0, y0 + 0.05, 0.17), 41, 93)]
    # every cell within tol of the map's peak magnitude; the map-level relative L2 bar where a
    # grid has enough cells for it to mean one (for a single cell it is that cell's relative error)
    tol = LOOSE_TOL.get(precision, HEAT_TOL)
    peak = [float(np.max(np.abs(P[psi]))) for psi in range(2)]
    for grid, nx, ny in cases:
        heat, hmax = mp.decode(grid, nx, ny, precision)
        torch.cuda.synchronize()
        ref = oracle.similarity(w.theta, w.layout, w.tiles, om, grid, nx, ny)
        got = heat.cpu().numpy().astype(np.float64)
        for psi in range(2):
            mab = float(np.max(np.abs(got[psi] - ref[psi])))
            assert mab <= tol * peak[psi], (grid, nx, ny, psi, mab)
            if nx * ny >= 256:
                e = rel_l2(got[psi], ref[psi])
                assert e <= tol, (grid, nx, ny, psi, e)
            assert hmax.cpu().numpy()[psi] == np.max(got[psi])
    mp.close()


def test_edge_cases(torch_cuda):
    say("[gpu] edge cases")
    from paper_2408_09066_amd import native
    torch = torch_cuda
    D = 64
    th = synth.make_theta(D, 0.3, np.random.default_rng(3))
    layout, tiles = (-2.0, -2.0, 2.0, 2.0), (2, 2)
    grid, nx, ny = (-2.0, -2.0, 0.25), 16, 16
    # empty map: all-zero heat, zero maxima, ogm 0 -> occupied at rho = 0
    m = native.Map(th, layout, tiles)
    m.encode(torch.zeros((0, 2), dtype=torch.float32, device="cuda"),
             torch.zeros(0, dtype=torch.uint8, device="cuda"))
    heat, hmax = m.decode(grid, nx, ny)
    ogm, lab = native.classify(heat, hmax, 1, 1, 0.0)
    torch.cuda.synchronize()
    assert torch.all(heat == 0) and torch.all(hmax == 0)
    assert torch.all(ogm == 0) and torch.all(lab == 1)
    # one point: unit self-similarity at its own cell centre, other class empty
    cx, cy = grid[0] + 5.5 * grid[2], grid[1] + 9.5 * grid[2]
    m.encode(torch.tensor([[cx, cy]], dtype=torch.float32, device="cuda"),
             torch.tensor([1], dtype=torch.uint8, device="cuda"))
    heat, hmax = m.decode(grid, nx, ny)
    torch.cuda.synchronize()
    assert abs(float(heat[1, 9, 5]) - 1.0) < 1e-5
    assert torch.all(heat[0] == 0)
    # labels outside {0, 1} are rejected and counted, points far outside the layout bundle
    # into the nearest tile (double-precision phase path)
    xy = torch.tensor([[0.1, 0.2], [150.0, -90.0], [0.3, 0.3]], dtype=torch.float32, device="cuda")
    lb = torch.tensor([0, 1, 7], dtype=torch.uint8, device="cuda")
    m2 = native.Map(th, layout, tiles)
    m2.encode(xy, lb)
    assert m2.take_rejected() == 1
    mem = m2.memories()
    torch.cuda.synchronize()
    ref, bad = oracle.encode(th, layout, tiles, xy.cpu().numpy(), lb.cpu().numpy())
    assert bad == 1
    got = mem.cpu().numpy().astype(np.float64)
    for key in range(ref.shape[0]):
        assert rel_l2(got[key], ref[key, :D // 2 + 1]) < MEM_TOL
    # invalid arguments
    with pytest.raises(native.VsaogmError):
        native.Map(th[:-2], layout, tiles)            # not conjugate-symmetric
    with pytest.raises(native.VsaogmError):
        native.classify(heat, hmax, 25, 1, 0.0)       # radius above the maximum
    with pytest.raises(native.VsaogmError):
        m.decode(grid, 0, ny)                         # empty grid
    with pytest.raises(native.VsaogmError):
        m.decode((0.0, 0.0, -1.0), nx, ny)            # negative resolution
    # a 1 x 1 grid
    heat1, hmax1 = m.decode((cx - 0.125, cy - 0.125, 0.25), 1, 1)
    torch.cuda.synchronize()
    assert abs(float(heat1[1, 0, 0]) - 1.0) < 1e-5
    m.close()
    m2.close()


def test_wide_phase_path(torch_cuda):
    """One tile over a 40 m world: local phases exceed the single-precision bound."""
    say("[gpu] wide phase path")
    rec = synth.RECIPES["world40_d1"]
    import dataclasses
    small = dataclasses.replace(rec, name="world40_d1_small", n_poses=3, beams=240, empties=4,
                                D=1024, nx=100, ny=100, res=0.4)
    w = synth.build(small)
    om, P = oracle.pipeline(w, P_only=True)
    g = gpu_run(torch_cuda, w)
    for psi in range(2):
        e = rel_l2(g["heat"][psi], P[psi])
        say(f"  heat[{psi}] rel-L2 {e:.3e}")
        assert e <= HEAT_TOL


@pytest.mark.parametrize("act", ["entropy", "relu", "tanh", "sigmoid"])
@pytest.mark.parametrize("normalize,square", [(True, True), (True, False), (False, True), (False, False)])
def test_decoding_ablation_variants(torch_cuda, act, normalize, square):
    """The toggles of the decoding ablation (Sec. IV-B) on the oracle's similarity maps."""
    say(f"[gpu] ablation {act} normalize={normalize} square={square}")
    from paper_2408_09066_amd import native
    torch = torch_cuda
    w, (om, P, m, H, ogm, lab) = oracle_result("mini4x4")
    P32 = P.astype(np.float32)
    r_occ, r_emp = 3, 2
    m_ref, A_ref, ogm_ref, lab_ref = oracle.postprocess_ex(P32.astype(np.float64), r_occ, r_emp, 0.0,
                                                           normalize, square, act)
    heat = torch.from_numpy(P32).cuda()
    hmax = torch.from_numpy(m_ref.astype(np.float32)).cuda()
    ogm_g, lab_g = native.classify(heat, hmax, r_occ, r_emp, 0.0, normalize=normalize,
                                   square=square, act=act)
    torch.cuda.synchronize()
    ogm_g = ogm_g.cpu().numpy().astype(np.float64)
    lab_g = lab_g.cpu().numpy()
    assert np.max(np.abs(ogm_g - ogm_ref)) < 1e-4
    bad = lab_g != lab_ref
    assert not bad.any() or np.max(np.abs(ogm_ref[bad])) < 1e-5
