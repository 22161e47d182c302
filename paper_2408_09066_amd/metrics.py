"""Mapping accuracy as the paper reports it (Sec. IV: area under the ROC curve and negative
log-likelihood of the held-out labelled points, after training on 80 % of them).

The map's probability that a cell is occupied is the softmax probability of class 1,
Pr1 = (1 + OGM) / 2 (eqs. softmax and psd: OGM = Pr1 - Pr0 with Pr0 + Pr1 = 1).  A held-out
point is scored with the probability of the grid cell that contains it; points outside the grid
are not scored.  numpy only; nothing here runs on the GPU.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np


def split_points(n: int, train_frac: float, rng: np.random.Generator) -> Tuple[np.ndarray, np.ndarray]:
    """Random train / held-out split of n points: (train indices, test indices), each sorted."""
    if not 0.0 < train_frac < 1.0:
        raise ValueError("train_frac must be in (0, 1)")
    perm = rng.permutation(n)
    k = int(round(train_frac * n))
    return np.sort(perm[:k]), np.sort(perm[k:])


def point_cells(xy: np.ndarray, grid, nx: int, ny: int) -> Tuple[np.ndarray, np.ndarray]:
    """Flat cell index j*nx + i of each point and a mask of the points inside the grid."""
    x0, y0, res = grid
    i = np.floor((np.asarray(xy[:, 0], np.float64) - x0) / res).astype(np.int64)
    j = np.floor((np.asarray(xy[:, 1], np.float64) - y0) / res).astype(np.int64)
    inside = (i >= 0) & (i < nx) & (j >= 0) & (j < ny)
    return np.where(inside, j * nx + i, 0), inside


def occupancy_probability(ogm: np.ndarray) -> np.ndarray:
    """Pr1 = (1 + OGM) / 2, clipped to [0, 1] against rounding."""
    return np.clip(0.5 * (1.0 + np.asarray(ogm, np.float64)), 0.0, 1.0)


def auc(score: np.ndarray, label: np.ndarray) -> float:
    """Area under the ROC curve: the probability that a random positive scores above a random
    negative, ties counting one half (Mann-Whitney statistic from average ranks)."""
    s = np.asarray(score, np.float64).ravel()
    y = np.asarray(label).ravel().astype(bool)
    npos, nneg = int(y.sum()), int((~y).sum())
    if npos == 0 or nneg == 0:
        raise ValueError("AUC needs both classes")
    order = np.argsort(s, kind="mergesort")
    ranks = np.empty(len(s), np.float64)
    sorted_s = s[order]
    # average rank (1-based) over each run of equal scores
    starts = np.flatnonzero(np.r_[True, sorted_s[1:] != sorted_s[:-1]])
    ends = np.r_[starts[1:], len(s)]
    avg = (starts + ends + 1) / 2.0
    ranks[order] = np.repeat(avg, ends - starts)
    return float((ranks[y].sum() - npos * (npos + 1) / 2.0) / (npos * nneg))


def nll(prob: np.ndarray, label: np.ndarray, eps: float = 1e-7) -> float:
    """Mean negative log-likelihood of binary labels under probabilities clipped to [eps, 1-eps]."""
    p = np.clip(np.asarray(prob, np.float64).ravel(), eps, 1.0 - eps)
    y = np.asarray(label).ravel().astype(bool)
    return float(-np.mean(np.where(y, np.log(p), np.log1p(-p))))


def evaluate(ogm: np.ndarray, grid, xy: np.ndarray, label: np.ndarray) -> Dict[str, float]:
    """AUC and NLL of labelled points under a map (ogm: [ny][nx])."""
    ny, nx = ogm.shape
    cells, inside = point_cells(xy, grid, nx, ny)
    p = occupancy_probability(ogm).ravel()[cells[inside]]
    y = np.asarray(label)[inside]
    return {"auc": auc(p, y), "nll": nll(p, y), "points": int(inside.sum()),
            "occupied": int(y.astype(bool).sum())}
