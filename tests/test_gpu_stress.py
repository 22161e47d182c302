"""The large-map configuration at full size (D = 16384, 16 x 16 tiles, 4000 x 4000 grid, bf16 hi+lo
decode) through the request loop with localized decoding, on sampled outputs.

The oracle cannot encode millions of points at D = 16384 in seconds, but a tile's memories
depend only on the points nearest to it (Sec. III-A): encoding just the points of a few tiles
gives those tiles' memories exactly, and the similarity at cells of those tiles reads nothing
else.  So the oracle encodes all the points of four seeded random tiles (among those holding at
least 2 000 points) and checks 10 000 seeded cells of them, 2 500 per tile.  The served heat must also equal a full decode of the served map up to the
order of the fp32 accumulation (max-abs <= 1e-5), and the maxima must be the heat's own maxima.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2408_09066_amd import synth

pytestmark = pytest.mark.gpu

N_UPDATES = 30


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


def test_stress_map_sampled(torch_cuda):
    say(f"[gpu] large map, {N_UPDATES} updates through the request loop")
    from paper_2408_09066_amd import native
    torch = torch_cuda
    sc = synth.stress_scenario(n_poses=N_UPDATES * 10)
    ups = sc.updates()
    say(f"  generated {sum(len(x) for x, _ in ups)} points")
    srv = native.Server(max_inflight=2)
    mid = srv.add_map(sc.theta, sc.layout, sc.tiles)
    tickets = []
    for j, (xy, lb) in enumerate(ups):
        want = ("label", "heat") if j == len(ups) - 1 else ("label",)
        tickets.append(srv.submit(mid, xy, lb, sc.grid, sc.nx, sc.ny, sc.r, sc.r, 0.0, "bf16x3",
                                  want=want, local=True))
    res = [srv.wait(t) for t, _ in tickets]
    assert all(r["status"] == 0 for r in res)
    heat = tickets[-1][1]["heat"]
    hmax = np.array(res[-1]["hmax"], dtype=np.float32)
    say("  served")
    # localized decoding equals a full decode of the same map
    srv.drain()
    m = srv.get_map(mid)
    full, fmax = m.decode(sc.grid, sc.nx, sc.ny, "bf16x3")
    torch.cuda.synchronize()
    d = float(np.max(np.abs(full.cpu().numpy() - heat)))
    dm = float(np.max(np.abs(fmax.cpu().numpy() - hmax)))
    say(f"  localized vs full decode: max-abs {d:.3e}, maxima {dm:.3e}")
    assert d <= 1e-5 and dm <= 1e-5
    del full, fmax
    for p in range(2):
        assert hmax[p] == heat[p].max()

    # oracle at sampled cells of two tiles
    xy = np.concatenate([x for x, _ in ups])
    lb = np.concatenate([l for _, l in ups])
    beta = oracle.assign_tiles(sc.layout, sc.tiles, xy)
    counts = np.bincount(beta, minlength=sc.tiles[0] * sc.tiles[1])
    touched = np.flatnonzero(counts >= 2000)
    pick = np.sort(np.random.default_rng(np.random.SeedSequence([2408, 5, 78])).choice(touched, size=4,
                                                                                         replace=False))
    say(f"  tiles {pick.tolist()} with {counts[pick].tolist()} points")
    sel = np.isin(beta, pick)
    omega, bad = oracle.encode(sc.theta, sc.layout, sc.tiles, xy[sel], lb[sel])
    assert bad == 0
    gx, gy, res_ = sc.grid
    rng = np.random.default_rng(np.random.SeedSequence([2408, 5, 77]))
    cand = rng.choice(sc.nx * sc.ny, size=1_200_000, replace=False)
    jj, ii = np.divmod(cand, sc.nx)
    cbeta = oracle.assign_tiles(sc.layout, sc.tiles,
                                np.stack([gx + (ii + 0.5) * res_, gy + (jj + 0.5) * res_], axis=1))
    cells = np.concatenate([cand[cbeta == b][:2500] for b in pick])
    assert len(cells) == 10_000
    P = oracle.similarity_cells(sc.theta, sc.layout, sc.tiles, omega, sc.grid, sc.nx, cells)
    for p in range(2):
        g = heat[p].reshape(-1)[cells].astype(np.float64)
        e = np.linalg.norm(g - P[p]) / np.linalg.norm(P[p])
        say(f"  heat[{p}] sampled rel-L2 {e:.3e} max-abs {np.max(np.abs(g - P[p])):.3e}")
        assert e <= 1e-4
    srv.close()
