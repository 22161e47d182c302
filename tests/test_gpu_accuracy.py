"""The accuracy harness on GPU maps: held-out AUC / NLL (Sec. IV, 80 / 20 split of the labelled
points) from the HIP path against the same figures from the FP64 oracle's map.

AUC is a rank statistic, so it can move only through pairs (occupied, empty) whose
probabilities lie within twice the largest probability difference between the two maps; the
bar is that fraction of pairs (computed from the data).  NLL: relative 1e-3."""
import sys

import numpy as np
import pytest

import oracle
from paper_2408_09066_amd import metrics, synth

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


def gpu_ogm(torch, w, idx, precision):
    from paper_2408_09066_amd import native
    m = native.Map(w.theta, w.layout, w.tiles)
    m.encode(torch.from_numpy(np.ascontiguousarray(w.xy[idx])).cuda(),
             torch.from_numpy(np.ascontiguousarray(w.label[idx])).cuda())
    heat, hmax = m.decode(w.grid, w.nx, w.ny, precision)
    ogm, _ = native.classify(heat, hmax, w.r_occ, w.r_emp, w.rho)
    torch.cuda.synchronize()
    out = ogm.cpu().numpy().astype(np.float64)
    m.close()
    return out


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("name", ["toy_room", "mini4x4"])
def test_heldout_accuracy_matches_oracle(torch_cuda, name, precision):
    w = synth.workload(name)
    tr, te = metrics.split_points(w.n, 0.8, np.random.default_rng(np.random.SeedSequence([2408, 1, 6])))
    om, bad = oracle.encode(w.theta, w.layout, w.tiles, w.xy[tr], w.label[tr])
    P = oracle.similarity(w.theta, w.layout, w.tiles, om, w.grid, w.nx, w.ny)
    _, _, ogm_o, _ = oracle.postprocess(P, w.r_occ, w.r_emp, w.rho)
    ogm_g = gpu_ogm(torch_cuda, w, tr, precision)
    ro = metrics.evaluate(ogm_o, w.grid, w.xy[te], w.label[te])
    rg = metrics.evaluate(ogm_g, w.grid, w.xy[te], w.label[te])
    say(f"[gpu] held-out accuracy {name} {precision}: AUC {rg['auc']:.5f} (oracle {ro['auc']:.5f}), "
        f"NLL {rg['nll']:.5f} (oracle {ro['nll']:.5f}), {rg['points']} points")
    cells, inside = metrics.point_cells(w.xy[te], w.grid, w.nx, w.ny)
    po = metrics.occupancy_probability(ogm_o).ravel()[cells[inside]]
    pg = metrics.occupancy_probability(ogm_g).ravel()[cells[inside]]
    y = w.label[te][inside].astype(bool)
    d = float(np.max(np.abs(pg - po)))
    close = np.abs(po[y][:, None] - po[~y][None, :]) <= 2 * d
    bound = float(close.sum()) / (y.sum() * (~y).sum())
    assert abs(rg["auc"] - ro["auc"]) <= bound + 1e-12
    assert abs(rg["nll"] - ro["nll"]) <= 1e-3 * ro["nll"]


def test_heldout_accuracy_bench_workload(torch_cuda):
    """The benchmark's 40 m world trained on 80 % of its points (reported; sanity bounds)."""
    w = synth.workload("world40")
    tr, te = metrics.split_points(w.n, 0.8, np.random.default_rng(np.random.SeedSequence([2408, 2, 6])))
    r = metrics.evaluate(gpu_ogm(torch_cuda, w, tr, "bf16x3"), w.grid, w.xy[te], w.label[te])
    say(f"[gpu] held-out accuracy world40: AUC {r['auc']:.4f}, NLL {r['nll']:.4f}, {r['points']} points")
    assert r["auc"] > 0.8 and np.isfinite(r["nll"])
