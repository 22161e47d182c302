"""A map update captured in a HIP graph.

After one eager update with a given point count, grid and precision (which sizes the work
buffers and builds the grid's tables), reset, encode, decode and classify launch kernels only:
no allocation, no synchronisation, no memset.  The update can then be captured once and
replayed for later scans of the same size, with new points copied into the captured input
buffers.  Every replay, with eager work and synchronisation between replays, must equal the
eager update bit for bit.
"""
import sys

import numpy as np
import pytest

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


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_update_replays_in_a_graph(torch_cuda, precision):
    from paper_2408_09066_amd import native
    torch = torch_cuda
    w = synth.workload("mini4x4")
    n = w.n // 3
    parts = [(w.xy[k * n:(k + 1) * n], w.label[k * n:(k + 1) * n]) for k in range(3)]
    m = native.Map(w.theta, w.layout, w.tiles)
    xy = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    lb = torch.empty(n, dtype=torch.uint8, device="cuda")
    heat = torch.empty((2, w.ny, w.nx), dtype=torch.float32, device="cuda")
    hmax = torch.empty(2, dtype=torch.float32, device="cuda")
    ogm = torch.empty((w.ny, w.nx), dtype=torch.float32, device="cuda")
    lab = torch.empty((w.ny, w.nx), dtype=torch.uint8, device="cuda")

    def step():
        m.reset()
        m.encode(xy, lb)
        m.decode(w.grid, w.nx, w.ny, precision, heat=heat, hmax=hmax)
        native.classify(heat, hmax, w.r_occ, w.r_emp, w.rho, ogm=ogm, label=lab)

    def load(k):
        xy.copy_(torch.from_numpy(np.ascontiguousarray(parts[k][0])))
        lb.copy_(torch.from_numpy(np.ascontiguousarray(parts[k][1])))

    load(0)
    step()                       # eager warm-up: buffers sized, tables built
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for rep, k in enumerate([1, 2, 0, 1]):
        load(k)
        g.replay()
        torch.cuda.synchronize()
        got = [t.clone() for t in (heat, hmax, ogm, lab)]
        step()                   # the same update, eager
        torch.cuda.synchronize()
        for a, b in zip(got, (heat, hmax, ogm, lab)):
            assert torch.equal(a, b), (rep, k)
        say(f"[gpu] graph replay {rep} (scan {k}, {precision}) equals the eager update")
    m.close()
