"""The request loop (vsaogm_submit / vsaogm_poll) on the GPU.

Every update a server runs must equal the same update run alone through the map API (same
kernels, same per-map order), bit for bit, whatever else shares the device; and it must match
the FP64 oracle within the fp32 bars.
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


@pytest.fixture(scope="module")
def stream():
    maps, reqs = synth.serving_stream(n_maps=4, n_requests=24, config_id=41, beams=(120, 600),
                                      grid_side=(40, 200), dims=(1024, 2048))
    return maps, reqs


def direct(torch, maps, reqs, precision):
    """Each request through the map API, in submission order."""
    from paper_2408_09066_amd import native
    objs = [native.Map(m.theta, m.layout, m.tiles) for m in maps]
    outs = []
    for q in reqs:
        spec = maps[q.map_id]
        mo = objs[q.map_id]
        mo.encode(torch.from_numpy(q.xy).cuda(), torch.from_numpy(q.label).cuda())
        heat, hmax = mo.decode(spec.grid, spec.side, spec.side, precision)
        ogm, lab = native.classify(heat, hmax, 3, 3, 0.0)
        torch.cuda.synchronize()
        outs.append({"heat": heat.cpu().numpy(), "ogm": ogm.cpu().numpy(), "label": lab.cpu().numpy()})
    for mo in objs:
        mo.close()
    return outs


def served(maps, reqs, precision, only_map=None, max_inflight=4, budget=0, local=False, max_batch=0):
    from paper_2408_09066_amd import native
    srv = native.Server(max_inflight=max_inflight, hbm_budget_bytes=budget, max_batch=max_batch)
    ids = [srv.add_map(m.theta, m.layout, m.tiles) for m in maps]
    tickets = []
    for i, q in enumerate(reqs):
        if only_map is not None and q.map_id != only_map:
            continue
        spec = maps[q.map_id]
        t, out = srv.submit(ids[q.map_id], q.xy, q.label, spec.grid, spec.side, spec.side, 3, 3,
                            0.0, precision, want=("label", "ogm", "heat"), local=local)
        tickets.append((i, t, out))
    results = {}
    for i, t, out in tickets:
        r = srv.wait(t)
        assert r["status"] == 0, r
        results[i] = (out, r)
    st = srv.stats()
    srv.close()
    return results, st


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_server_equals_direct_path(torch_cuda, stream, precision):
    say(f"[gpu] server vs direct path {precision}")
    maps, reqs = stream
    ref = direct(torch_cuda, maps, reqs, precision)
    res, st = served(maps, reqs, precision)
    assert st["completed"] == len(reqs)
    assert st["peak_bytes"] <= st["budget_bytes"]
    slots = set()
    for i, (out, r) in res.items():
        slots.add(r["slot"])
        for k in ("heat", "ogm", "label"):
            assert np.array_equal(out[k], ref[i][k]), (i, k)
        assert r["hmax"][1] == pytest.approx(float(ref[i]["heat"][1].max()), abs=0.0)
    say(f"  {len(res)} updates bitwise equal to the direct path, slots used {sorted(slots)}")


def test_alone_and_in_the_mix_agree(torch_cuda, stream):
    """A map's updates give the same bits alone on the server and mixed with other maps'."""
    say("[gpu] alone vs in the mix")
    maps, reqs = stream
    mix, _ = served(maps, reqs, "bf16x3", max_inflight=8, max_batch=8)   # batches of up to 8 maps
    for mid in range(len(maps)):
        alone, _ = served(maps, reqs, "bf16x3", only_map=mid, max_inflight=1)
        for i, (out, r) in alone.items():
            for k in ("heat", "ogm", "label"):
                assert np.array_equal(out[k], mix[i][0][k]), (mid, i, k)


def test_tight_budget_still_completes(torch_cuda, stream):
    """Admission waits for memory: a budget for the maps' own buffers and about one request at
    a time (no room for every grid's tables at once) still finishes, and the server's count
    stays within it."""
    say("[gpu] tight budget")
    maps, reqs = stream
    from paper_2408_09066_amd import native
    probe = native.Server(max_inflight=1)
    ids = [probe.add_map(m.theta, m.layout, m.tiles) for m in maps]
    base = probe.memory()["resident"]
    one = max(probe.request_bytes(ids[q.map_id], q.xy.shape[0], maps[q.map_id].grid, maps[q.map_id].side,
                                  maps[q.map_id].side) for q in reqs[:12])
    probe.close()
    budget = base + 2 * one + (256 << 20)
    res, st = served(maps, reqs[:12], "fp32", max_inflight=4, budget=budget)
    assert st["completed"] == 12
    assert st["peak_bytes"] <= budget


def test_budget_bounds_device_memory(torch_cuda):
    """What the server holds on the device -- maps, cached grids, workspaces, slot buffers,
    requests in flight -- stays within its budget, measured as the drop of the device's free
    memory, over a stream that decodes three grid sizes per map (more grid tables than the
    budget holds: the server must release cached grids to go on)."""
    say("[gpu] budget bounds device memory")
    torch = torch_cuda
    from paper_2408_09066_amd import native
    rng = np.random.default_rng(9066)
    D, T, res = 8192, 2, 0.05
    sides = (1200, 1500, 1800)
    nmaps = 4
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0, _ = torch.cuda.mem_get_info()
    probe = native.Server(max_inflight=4)
    half = max(sides) * res / 2.0
    layout = (-half, -half, half, half)
    thetas = [synth.make_theta(D, 0.25, rng) for _ in range(nmaps)]
    for th in thetas:
        probe.add_map(th, layout, (T, T))
    base = probe.memory()["resident"]
    probe.close()
    budget = base + (1 << 30)
    srv = native.Server(max_inflight=4, hbm_budget_bytes=budget)
    ids = [srv.add_map(th, layout, (T, T)) for th in thetas]
    items = []
    for i in range(36):
        side = sides[i % 3]
        h = side * res / 2.0
        n = 20000
        xy = np.stack([rng.uniform(-h, h, n), rng.uniform(-h, h, n)], 1).astype(np.float32)
        lb = rng.integers(0, 2, n).astype(np.uint8)
        items.append({"map_id": ids[(i // 3) % nmaps], "xy": xy, "label": lb, "grid": (-h, -h, res),
                      "nx": side, "ny": side, "r_occ": 2, "r_emp": 2,
                      "precision": ("bf16x3", "fp32", "bf16")[(i // 2) % 3]})
    tk = srv.submit_many(items)
    out = [srv.wait(t) for t, _ in tk]
    assert all(r["status"] == 0 for r in out)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    mem = srv.memory()
    st = srv.stats()
    held = free0 - free1
    say(f"  budget {budget / 2**20:.0f} MiB, peak counted {st['peak_bytes'] / 2**20:.0f} MiB, device drop "
        f"{held / 2**20:.0f} MiB, reclaims {mem['reclaims']}, resident {mem['resident'] / 2**20:.0f} MiB, "
        f"fixed {mem['fixed'] / 2**20:.0f} MiB")
    assert st["peak_bytes"] <= budget
    assert mem["reclaims"] >= 1
    # the allocator rounds blocks up and the runtime holds its own queues and events
    assert held <= budget + (128 << 20)
    srv.close()


def test_served_update_matches_oracle(torch_cuda):
    say("[gpu] served update vs oracle")
    from paper_2408_09066_amd import native
    w = synth.workload("mini4x4")
    srv = native.Server(max_inflight=2)
    mid = srv.add_map(w.theta, w.layout, w.tiles)
    t, out = srv.submit(mid, w.xy, w.label, w.grid, w.nx, w.ny, w.r_occ, w.r_emp, 0.0, "bf16x3",
                        want=("heat", "label"))
    r = srv.wait(t)
    assert r["status"] == 0
    _, P, m, H, ogm, lab = oracle.pipeline(w)
    for p in range(2):
        e = np.linalg.norm(out["heat"][p] - P[p]) / np.linalg.norm(P[p])
        assert e < 1e-4
    assert np.mean(out["label"] == lab) >= 0.999
    srv.close()


def test_server_errors(torch_cuda):
    say("[gpu] server errors")
    from paper_2408_09066_amd import native
    srv = native.Server(max_inflight=1, hbm_budget_bytes=128 << 20)
    w = synth.workload("toy_room")
    mid = srv.add_map(w.theta, w.layout, w.tiles)
    with pytest.raises(native.VsaogmError) as e:
        srv.submit(mid + 7, w.xy, w.label, w.grid, w.nx, w.ny, 2, 2)
    assert e.value.code == native.ENOTFOUND
    with pytest.raises(native.VsaogmError) as e:
        srv.submit(mid, w.xy, w.label, w.grid, 20000, 20000, 2, 2)   # beyond the budget
    assert e.value.code == native.EINVAL
    with pytest.raises(native.VsaogmError):
        srv.submit(mid, w.xy, w.label, w.grid, w.nx, w.ny, 30, 2)
    t, _ = srv.submit(mid, w.xy, w.label, w.grid, w.nx, w.ny, 2, 2)
    srv.wait(t)
    with pytest.raises(native.VsaogmError) as e:
        srv.poll(t)                                                     # retired
    assert e.value.code == native.ENOTFOUND
    srv.close()


def test_submit_many_matches_single_submits(torch_cuda, stream):
    say("[gpu] submit_many")
    from paper_2408_09066_amd import native
    maps, reqs = stream
    ref, _ = served(maps, reqs, "fp32")
    srv = native.Server(max_inflight=4)
    ids = [srv.add_map(m.theta, m.layout, m.tiles) for m in maps]
    items = [{"map_id": ids[q.map_id], "xy": q.xy, "label": q.label, "grid": maps[q.map_id].grid,
              "nx": maps[q.map_id].side, "ny": maps[q.map_id].side, "r_occ": 3, "r_emp": 3,
              "precision": "fp32"} for q in reqs]
    tk = srv.submit_many(items, want=("label", "ogm", "heat"))
    assert len(tk) == len(reqs)
    for i, (t, out) in enumerate(tk):
        assert srv.wait(t)["status"] == 0
        for k in ("heat", "ogm", "label"):
            assert np.array_equal(out[k], ref[i][0][k])
    # a bad request stops the batch; the ones before it are queued
    bad = dict(items[0], map_id=99)
    with pytest.raises(native.VsaogmError):
        srv.submit_many([items[0], bad, items[1]])
    srv.drain()
    srv.close()


# Localized and full decodes differ only in the order of the fp32 K-reduction: heat by at most
# ORDER_TOL (absolute), the OGM derived from it by at most the OGM bar used against the oracle,
# and labels only where the OGM lies within that bar of the threshold 0.
ORDER_TOL = 1e-5
OGM_TOL = 1e-3


def check_local(out, ref, tag):
    for k, tol in (("heat", ORDER_TOL), ("ogm", OGM_TOL)):
        d = float(np.max(np.abs(out[k] - ref[k]))) if out[k].size else 0.0
        assert d <= tol, (tag, k, d)
    flips = out["label"] != ref["label"]
    assert not flips.any() or float(np.max(np.abs(ref["ogm"][flips]))) <= OGM_TOL, tag


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_local_requests_equal_full_ones(torch_cuda, stream, precision):
    """Requests flagged local (map-kept heat, only changed tiles decoded) match full decodes up
    to the accumulation order of the similarity reduction (labels may differ only where the
    OGM is within that of the threshold 0)."""
    say(f"[gpu] local requests {precision}")
    maps, reqs = stream
    ref = direct(torch_cuda, maps, reqs, precision)
    got, _ = served(maps, reqs, precision, local=True)
    for i in range(len(reqs)):
        out, _ = got[i]
        check_local(out, ref[i], i)


def test_local_requests_switching_grids(torch_cuda):
    """One map, local requests alternating between two grids, against full decodes."""
    say("[gpu] local requests, two grids")
    from paper_2408_09066_amd import native
    torch = torch_cuda
    w = synth.workload("mini4x4")
    grids = [(w.grid, w.nx, w.ny), ((w.grid[0] + 0.35, w.grid[1] + 0.15, 0.1), 120, 96)]
    parts = np.array_split(np.arange(w.n), 6)
    srv = native.Server(max_inflight=2)
    mid = srv.add_map(w.theta, w.layout, w.tiles)
    ref_map = native.Map(w.theta, w.layout, w.tiles)
    for j, idx in enumerate(parts):
        g, nx, ny = grids[(j // 2) % 2]
        t, out = srv.submit(mid, w.xy[idx], w.label[idx], g, nx, ny, 3, 3, 0.0, "fp32",
                            want=("label", "ogm", "heat"), local=True)
        assert srv.wait(t)["status"] == 0
        ref_map.encode(torch.from_numpy(np.ascontiguousarray(w.xy[idx])).cuda(),
                       torch.from_numpy(np.ascontiguousarray(w.label[idx])).cuda())
        heat, hmax = ref_map.decode(g, nx, ny)
        ogm, lab = native.classify(heat, hmax, 3, 3, 0.0)
        torch.cuda.synchronize()
        check_local(out, {"heat": heat.cpu().numpy(), "ogm": ogm.cpu().numpy(),
                          "label": lab.cpu().numpy()}, j)
    ref_map.close()
    srv.close()


def test_request_stream_against_oracle(torch_cuda):
    """The benchmark's request stream (16 maps, 256 updates): every update of its two cheapest
    maps (D = 2048, the smallest grids), served interleaved in stream order, against the FP64
    oracle's memories accumulated update by update: whole heatmaps within the fp32 bar, labels
    >= 99.9 % with every disagreement within 1e-3 of the threshold."""
    say("[gpu] request stream vs oracle")
    from paper_2408_09066_amd import native
    maps, reqs = synth.serving_stream()
    small = sorted((m.side, i) for i, m in enumerate(maps) if m.D == 2048)[:2]
    chosen = [i for _, i in small]
    srv = native.Server(max_inflight=8)
    ids = {i: srv.add_map(maps[i].theta, maps[i].layout, maps[i].tiles) for i in chosen}
    tickets = []
    for q in reqs:
        if q.map_id in ids:
            spec = maps[q.map_id]
            t, out = srv.submit(ids[q.map_id], q.xy, q.label, spec.grid, spec.side, spec.side, 3, 3, 0.0,
                                "bf16x3", want=("label", "ogm", "heat"))
            tickets.append((q, t, out))
    omega = {i: None for i in chosen}
    worst, n = 0.0, 0
    for q, t, out in tickets:
        assert srv.wait(t)["status"] == 0
        spec = maps[q.map_id]
        omega[q.map_id], bad = oracle.encode(spec.theta, spec.layout, spec.tiles, q.xy, q.label,
                                             omega=omega[q.map_id])
        assert bad == 0
        P = oracle.similarity(spec.theta, spec.layout, spec.tiles, omega[q.map_id], spec.grid, spec.side,
                              spec.side)
        _, _, ogm, lab = oracle.postprocess(P, 3, 3, 0.0)
        for p in range(2):
            e = float(np.linalg.norm(out["heat"][p] - P[p]) / np.linalg.norm(P[p]))
            worst = max(worst, e)
            assert e <= 1e-4, (q.map_id, p, e)
        flips = out["label"] != lab
        assert float(np.mean(~flips)) >= 0.999
        assert not flips.any() or float(np.max(np.abs(ogm[flips]))) < 1e-3
        n += 1
    srv.close()
    say(f"  {n} updates of maps {chosen}: worst heat rel-L2 {worst:.2e}")


FULL_HEAT_MAX_WORK = 2.0e9   # cells x D above which the oracle checks sampled cells only
SAMPLED_CELLS = 4000


def test_request_stream_random_requests_against_oracle(torch_cuda):
    """The benchmark's whole request stream (16 maps, 256 updates of uneven scans and grids) served
    through the loop, and 32 seeded random requests of it checked against the FP64 oracle's
    memories accumulated update by update in stream order: maps of every D, the largest grid
    (916 x 916 cells) and the largest D = 8192 grid (829 x 829).  Where the oracle's whole map
    costs at most 2e9 cell-bins it is computed in full and the heatmaps (rel-L2 <= 1e-4) and
    labels (>= 99.9 %, every disagreement within 1e-3 of the threshold) are compared in full;
    above that, 4000 seeded random cells of the heatmaps are compared (rel-L2 <= 1e-4)."""
    say("[gpu] request stream, 32 random requests vs oracle")
    from paper_2408_09066_amd import native
    maps, reqs = synth.serving_stream()
    rng = np.random.default_rng(np.random.SeedSequence([2408, 4, 32]))
    chosen = set(rng.choice(len(reqs), size=32, replace=False).tolist())
    big = max(range(len(maps)), key=lambda i: maps[i].side)
    big8 = max((i for i in range(len(maps)) if maps[i].D == 8192), key=lambda i: maps[i].side)
    assert any(reqs[i].map_id == big for i in chosen) and any(reqs[i].map_id == big8 for i in chosen)
    assert {maps[reqs[i].map_id].D for i in chosen} == {2048, 4096, 8192}
    srv = native.Server(max_inflight=8)
    ids = [srv.add_map(m.theta, m.layout, m.tiles) for m in maps]
    tickets = []
    for j, q in enumerate(reqs):
        spec = maps[q.map_id]
        want = ("label", "heat") if j in chosen else ("label",)
        t, out = srv.submit(ids[q.map_id], q.xy, q.label, spec.grid, spec.side, spec.side, 3, 3, 0.0, "bf16x3",
                            want=want)
        tickets.append((t, out))
    res = [srv.wait(t) for t, _ in tickets]
    assert all(r["status"] == 0 for r in res)
    srv.close()
    say("  served 256 updates")
    last = {}
    for j in sorted(chosen):
        last[reqs[j].map_id] = j
    omega = {}
    worst, full, sampled = 0.0, 0, 0
    for j, q in enumerate(reqs):
        if q.map_id not in last or j > last[q.map_id]:
            continue
        spec = maps[q.map_id]
        omega[q.map_id], bad = oracle.encode(spec.theta, spec.layout, spec.tiles, q.xy, q.label,
                                             omega=omega.get(q.map_id))
        assert bad == 0
        if j not in chosen:
            continue
        out = tickets[j][1]
        n = spec.side
        if n * n * spec.D <= FULL_HEAT_MAX_WORK:
            P = oracle.similarity(spec.theta, spec.layout, spec.tiles, omega[q.map_id], spec.grid, n, n)
            _, _, ogm, lab = oracle.postprocess(P, 3, 3, 0.0)
            for p in range(2):
                e = float(np.linalg.norm(out["heat"][p] - P[p]) / np.linalg.norm(P[p]))
                worst = max(worst, e)
                assert e <= 1e-4, (j, q.map_id, p, e)
            flips = out["label"] != lab
            assert float(np.mean(~flips)) >= 0.999, j
            assert not flips.any() or float(np.max(np.abs(ogm[flips]))) < 1e-3, j
            full += 1
        else:
            cells = np.random.default_rng(np.random.SeedSequence([2408, 4, 33, j])).choice(
                n * n, size=SAMPLED_CELLS, replace=False)
            P = oracle.similarity_cells(spec.theta, spec.layout, spec.tiles, omega[q.map_id], spec.grid, n, cells)
            for p in range(2):
                g = out["heat"][p].reshape(-1)[cells].astype(np.float64)
                e = float(np.linalg.norm(g - P[p]) / np.linalg.norm(P[p]))
                worst = max(worst, e)
                assert e <= 1e-4, (j, q.map_id, p, e)
            sampled += 1
        say(f"  request {j}: map {q.map_id} D={spec.D} {n}x{n} checked")
    say(f"  {full} requests in full, {sampled} at sampled cells; worst heat rel-L2 {worst:.2e}")
