"""Accuracy harness (AUC / NLL of held-out points, Sec. IV) pinned on the CPU: closed forms,
brute-force pair counting, the scikit-learn routine, and exact cell containment."""
import math

import numpy as np
import pytest

from paper_2408_09066_amd import metrics


def brute_auc(s, y):
    pos, neg = s[y], s[~y]
    gt = (pos[:, None] > neg[None, :]).sum()
    eq = (pos[:, None] == neg[None, :]).sum()
    return (gt + 0.5 * eq) / (len(pos) * len(neg))


def test_auc_closed_forms():
    y = np.array([0, 0, 1, 1], bool)
    assert metrics.auc(np.array([0.1, 0.2, 0.8, 0.9]), y) == 1.0
    assert metrics.auc(np.array([0.9, 0.8, 0.2, 0.1]), y) == 0.0
    assert metrics.auc(np.full(4, 0.3), y) == 0.5
    assert metrics.auc(np.array([0.1, 0.5, 0.5, 0.9]), y) == pytest.approx(0.875)
    with pytest.raises(ValueError):
        metrics.auc(np.ones(3), np.ones(3, bool))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_auc_brute_force_and_library(seed):
    rng = np.random.default_rng(seed)
    n = 300
    s = np.round(rng.normal(size=n), 1)  # many ties
    y = rng.random(n) < 0.3
    a = metrics.auc(s, y)
    assert a == pytest.approx(brute_auc(s, y), abs=1e-12)
    skm = pytest.importorskip("sklearn.metrics")
    assert a == pytest.approx(skm.roc_auc_score(y, s), abs=1e-12)


def test_nll():
    y = np.array([1, 0, 1, 0], bool)
    assert metrics.nll(np.full(4, 0.5), y) == pytest.approx(math.log(2))
    p = np.array([0.9, 0.2, 0.6, 0.35])
    ref = -np.mean([math.log(0.9), math.log(0.8), math.log(0.6), math.log(0.65)])
    assert metrics.nll(p, y) == pytest.approx(ref, rel=1e-12)
    # certainty on the wrong side is clipped, not infinite
    assert metrics.nll(np.array([0.0]), np.array([True])) == pytest.approx(-math.log(1e-7))


def test_split_and_probability():
    rng = np.random.default_rng(np.random.SeedSequence([2408, 1, 6]))
    tr, te = metrics.split_points(1001, 0.8, rng)
    assert len(tr) == 801 and len(te) == 200
    assert np.intersect1d(tr, te).size == 0
    assert np.array_equal(np.union1d(tr, te), np.arange(1001))
    tr2, te2 = metrics.split_points(1001, 0.8, np.random.default_rng(np.random.SeedSequence([2408, 1, 6])))
    assert np.array_equal(tr, tr2) and np.array_equal(te, te2)
    assert np.array_equal(metrics.occupancy_probability(np.array([-1.0, 0.0, 1.0])), [0.0, 0.5, 1.0])


def test_point_cells_brute_force():
    rng = np.random.default_rng(5)
    grid, nx, ny = (-2.0, -1.0, 0.25), 12, 9
    xy = rng.uniform(-3, 3, size=(500, 2)).astype(np.float32)
    cells, inside = metrics.point_cells(xy, grid, nx, ny)
    for (x, y), c, ok in zip(xy.astype(np.float64), cells, inside):
        hit = [(j * nx + i) for j in range(ny) for i in range(nx)
               if grid[0] + i * grid[2] <= x < grid[0] + (i + 1) * grid[2]
               and grid[1] + j * grid[2] <= y < grid[1] + (j + 1) * grid[2]]
        assert ok == (len(hit) == 1)
        if ok:
            assert c == hit[0]
