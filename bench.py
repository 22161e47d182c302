#!/usr/bin/env python3
"""Benchmark of the VSA-OGM hot path on one MI355X.

Headline (one JSON line): the large-map configuration "stress200" -- a 200 m x 200 m world with
400 obstacles mapped by a random walk of 1 080-beam scans, D = 16384, l = 0.1 m, 16 x 16 tiles
(512 memories), a 4000 x 4000 grid at 0.05 m, disk radius 3 and the similarity contraction in
bf16 hi+lo operands (which meet the fp32 accuracy bar).  One step is one incremental map update
with its inputs already resident in HBM: encode and bundle the update's 118 800 points (10
poses x 1 080 beams x (1 hit + 10 empty samples)) into the map's memories, decode both class
heatmaps over the whole grid, classify every cell (entropy, softmax difference, threshold).
The memories accumulate from step to step, as the map of a moving robot does.

Timed: K plain steps (throughput: cells decoded per second, points encoded per second), then K
steps whose stage kernels carry HIP timing events (per-kernel durations for the rooflines,
per-update latency percentiles).  Sections beside it: the same step through the request loop
(host inputs, labels returned per update: PCIe-inclusive), the 40 m world of the plain method in
fp32 and bf16 hi+lo, the request-loop benchmark (256 updates of 16 uneven maps against the plain
per-request fp32 path), the 3-D extension, held-out accuracy, and the FP64 CPU oracle timed on a
bounded sample of the headline workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks: HBM3E bandwidth, dense matrix rates per operand type, fp32 vector rate
PEAK_HBM_GBS = 8000.0
PEAK_MFMA_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0, "bf16x3": 2500.0}
PEAK_FP32_TFLOPS = 157.3
# Algorithmic work of the encode per point and spectrum bin: the phase Theta_x x + Theta_y y
# (two fused multiply-adds, 4 flops), one sine and one cosine (1 op each), and the accumulation
# of the real and imaginary parts (2 adds): 8 ops, priced against the fp32 vector rate (which
# counts a fused multiply-add as 2).  A 3-D point adds one fused multiply-add (10 ops).
ENCODE_OPS_PER_BIN = 8
ENCODE3_OPS_PER_BIN = 10
# Context only (not a peak): the VALU issue bound of the pair-form encode kernels, 256 CUs x
# 2.4 GHz x 64 lanes / (issue slots per complex exponential): 4.5 for planes, 5.5 for volumes.
ISSUE_CEXP_TPS = 256 * 2.4e9 * 64 / 4.5 / 1e12
ISSUE_CEXP3_TPS = 256 * 2.4e9 * 64 / 5.5 / 1e12


# HBM bytes per launch of a stage's main kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE counters
# of an earlier profiled run (scaled by what they read for a device-to-device copy of known size),
# one file per workload; a figure is used only while the kernel sources it was taken on are
# unchanged (SHA-256 recorded with it).
def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.json")


def source_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, stage):
    try:
        with open(traffic_file(workload)) as fh:
            rec = json.load(fh).get(stage)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha256") != source_digest(rec["sources"]):
        return None
    return rec["bytes_per_launch"]


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q))


def measured_hbm_copy_gbs() -> float:
    """Device-to-device copy of 1 GiB (bytes read plus bytes written per second): the HBM rate
    a streaming kernel can reach on this device, beside the 8 TB/s of the datasheet."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    reps = 5
    t = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * 4 * n * reps / dt / 1e9


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, xy, label, budget_s: float):
    """The FP64 oracle on a bounded sample of one update of the headline workload, scaled to one
    whole update (cells/s): encode a prefix of the update's points, the similarity at random
    cells, and the entropy / softmax / threshold post-processing of a sub-grid of the oracle's own
    heat; the same kinds of work on one host thread beside it."""
    import oracle
    oracle.lib()
    rng = np.random.default_rng(np.random.SeedSequence([2408, 99]))
    n = len(xy)
    ncell = sc.nx * sc.ny
    # encode: a prefix of the points, sized from a short probe to about budget/2 seconds
    probe = 200
    t = time.perf_counter()
    oracle.encode(sc.theta, sc.layout, sc.tiles, xy[:probe], label[:probe])
    dt = max(time.perf_counter() - t, 1e-6)
    n_enc = int(min(n, max(probe, probe * (0.5 * budget_s) / dt)))
    t = time.perf_counter()
    omega, _ = oracle.encode(sc.theta, sc.layout, sc.tiles, xy[:n_enc], label[:n_enc])
    t_enc = time.perf_counter() - t
    # similarity at random cells, sized to about budget/3 seconds
    cells = rng.choice(ncell, size=32, replace=False)
    t = time.perf_counter()
    oracle.similarity_cells(sc.theta, sc.layout, sc.tiles, omega, sc.grid, sc.nx, cells)
    dt = max(time.perf_counter() - t, 1e-6)
    n_dec = int(min(ncell, max(32, 32 * (budget_s / 3) / dt)))
    cells = rng.choice(ncell, size=n_dec, replace=False)
    t = time.perf_counter()
    oracle.similarity_cells(sc.theta, sc.layout, sc.tiles, omega, sc.grid, sc.nx, cells)
    t_dec = time.perf_counter() - t
    # post-processing of the oracle's heat of a 40 x 40 sub-grid around the first pose
    sub = 40
    px, py = sc.poses[0]
    gx, gy, res = sc.grid
    i0 = int(min(max((px - gx) / res - sub // 2, 0), sc.nx - sub))
    j0 = int(min(max((py - gy) / res - sub // 2, 0), sc.ny - sub))
    sub_grid = (gx + i0 * res, gy + j0 * res, res)
    P = oracle.similarity(sc.theta, sc.layout, sc.tiles, omega, sub_grid, sub, sub)
    t = time.perf_counter()
    oracle.postprocess(P, sc.r, sc.r, 0.0)
    t_cls = max(time.perf_counter() - t, 1e-6)
    step = t_enc * (n / n_enc) + t_dec * (ncell / n_dec) + t_cls * (ncell / (sub * sub))
    threads = oracle.num_threads()
    oracle.set_threads(1)
    n1 = min(n, max(16, int(n_enc * (budget_s / 8) / max(t_enc * threads, 1e-6))))
    t = time.perf_counter()
    om1, _ = oracle.encode(sc.theta, sc.layout, sc.tiles, xy[:n1], label[:n1])
    t_enc1 = time.perf_counter() - t
    c1 = cells[:max(8, int(n_dec * (budget_s / 8) / max(t_dec * threads, 1e-6)))]
    t = time.perf_counter()
    oracle.similarity_cells(sc.theta, sc.layout, sc.tiles, om1, sc.grid, sc.nx, c1)
    t_dec1 = time.perf_counter() - t
    t = time.perf_counter()
    oracle.postprocess(P, sc.r, sc.r, 0.0)
    t_cls1 = max(time.perf_counter() - t, 1e-6)
    oracle.set_threads(threads)
    step1 = t_enc1 * (n / n1) + t_dec1 * (ncell / len(c1)) + t_cls1 * (ncell / (sub * sub))
    return {
        "value": ncell / step,
        "unit": "cells/s",
        "cores": threads,
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": (f"one {n}-point update of {sc.name}: encode of its first {n_enc} points ({t_enc:.2f} s), "
                   f"similarity at {n_dec} random cells of {ncell} ({t_dec:.2f} s), entropy/softmax/threshold "
                   f"of the oracle's heat on a {sub}x{sub} sub-grid ({t_cls * 1e3:.1f} ms); scaled to one whole "
                   f"update ({step:.0f} s)"),
        "points_per_s": n_enc / t_enc,
        "single_thread": {"value": ncell / step1, "points_per_s": n1 / t_enc1, "cores": 1,
                          "sample": f"encode of {n1} points ({t_enc1:.2f} s), similarity at {len(c1)} cells "
                                    f"({t_dec1:.2f} s), the same sub-grid post-processing"},
    }


# Passes of the serving stream: untimed (tables, work buffers and pinned pools reach their sizes,
# clocks settle), then timed, of which the median is reported.
WARM_PASSES = 2
TIMED_PASSES = 5


def serving_benchmark(n_requests: int = 256, slots: int = 8, precision: str = "bf16x3", max_batch: int = 0,
                      plain: bool = True):
    """256 map updates of 16 uneven maps: plain per-request fp32 path vs the request loop.

    Plain path: one update at a time through the map API (copy in, encode, fp32 decode,
    classify, copy the labels out, synchronise).  Request loop: the server with `slots`
    execution slots and the bf16 hi+lo decode (fp32-level accuracy).  Both paths first run the
    whole stream WARM_PASSES times untimed, then TIMED_PASSES timed passes, of which the median
    is reported.  Throughput is measured with every request queued at once; latency percentiles
    with Poisson arrivals at 0.5x, 1x and 2x the plain path's throughput, measured on both paths
    (the plain path serves the arrivals one at a time in arrival order, each as soon as it has
    arrived and the previous one is done)."""
    import torch
    from paper_2408_09066_amd import native, synth

    maps, reqs = synth.serving_stream(n_requests=n_requests)
    dev = torch.device("cuda", 0)
    R = 3

    # ---- plain per-request path
    objs = [native.Map(m.theta, m.layout, m.tiles) for m in maps]

    def plain_one(q):
        spec, o = maps[q.map_id], objs[q.map_id]
        xy = torch.from_numpy(q.xy).to(dev)
        lb = torch.from_numpy(q.label).to(dev)
        o.encode(xy, lb)
        heat, hmax = o.decode(spec.grid, spec.side, spec.side, "fp32")
        _, lab = native.classify(heat, hmax, R, R, 0.0)
        out = lab.cpu().numpy()
        torch.cuda.synchronize()
        return out

    def plain_pass():
        t_all = time.perf_counter()
        labels = [plain_one(q) for q in reqs]
        return time.perf_counter() - t_all, labels

    for _ in range(WARM_PASSES):
        plain_pass()
    # median of the timed passes; memories accumulate pass after pass, so labels are compared
    # between the last passes of both paths (the same updates applied the same number of times)
    runs = [plain_pass() for _ in range(TIMED_PASSES)]
    plain_total = sorted(r[0] for r in runs)[TIMED_PASSES // 2]
    plain_labels = runs[-1][1]
    plain_ups = len(reqs) / plain_total

    # ---- request loop
    srv = native.Server(max_inflight=slots, max_batch=max_batch)
    ids = [srv.add_map(m.theta, m.layout, m.tiles) for m in maps]

    def submit(q):
        spec = maps[q.map_id]
        return srv.submit(ids[q.map_id], q.xy, q.label, spec.grid, spec.side, spec.side, R, R, 0.0,
                          precision)

    items = [{"map_id": ids[q.map_id], "xy": q.xy, "label": q.label, "grid": maps[q.map_id].grid,
              "nx": maps[q.map_id].side, "ny": maps[q.map_id].side, "r_occ": R, "r_emp": R,
              "precision": precision} for q in reqs]

    def saturated():
        # the client builds its request structs before the clock starts; the server's own
        # staging of the inputs (copies into pinned memory) is timed
        prepared = srv.prepare_many(items)
        t0 = time.perf_counter()
        tk = srv.submit_prepared(prepared)
        res = [srv.wait(t) for t, _ in tk]
        assert all(r["status"] == 0 for r in res)
        return time.perf_counter() - t0, [out["label"] for _, out in tk]

    for _ in range(WARM_PASSES):
        saturated()
    sruns = [saturated() for _ in range(TIMED_PASSES)]
    served_total = sorted(r[0] for r in sruns)[TIMED_PASSES // 2]
    served_labels = sruns[-1][1]
    agree = min(float(np.mean(a == b)) for a, b in zip(served_labels, plain_labels))
    served_ups = len(reqs) / served_total

    # ---- latency under Poisson arrivals
    arrivals = np.array([q.arrival_s for q in reqs])
    lat = {}
    for mult in (0.5, 1.0, 2.0):
        qps = mult * plain_ups
        arr = arrivals / qps
        fin = []   # plain path, measured: arrival to labels on the host
        t0 = time.perf_counter()
        for q, a_ in zip(reqs, arr):
            while time.perf_counter() - t0 < a_:
                pass
            plain_one(q)
            fin.append(time.perf_counter() - t0 - a_)
        t0 = time.perf_counter()
        tk = []
        for q, a_ in zip(reqs, arr):
            while time.perf_counter() - t0 < a_:
                pass
            tk.append(submit(q)[0])
        rs = [srv.wait(t) for t in tk]
        ls = [(r["t_done_ns"] - r["t_submit_ns"]) * 1e-6 for r in rs]
        lat[f"{mult}x"] = {"qps": qps,
                           "serving_ms": {"p50": percentile(ls, 50), "p99": percentile(ls, 99)},
                           "plain_ms": {"p50": percentile(fin, 50) * 1e3, "p99": percentile(fin, 99) * 1e3}}
    stats = srv.stats()
    srv.close()
    for o in objs:
        o.close()
    return {
        "workload": (f"{len(reqs)} updates of {len(maps)} maps: D in {{2048,4096,8192}}, 1-16 tiles, "
                     f"grid sides {min(m.side for m in maps)}-{max(m.side for m in maps)} at 0.05 m, "
                     f"{min(q.xy.shape[0] for q in reqs)}-{max(q.xy.shape[0] for q in reqs)} points"),
        "slots": slots,
        "precision": precision,
        "updates_per_s": served_ups,
        "plain_fp32_updates_per_s": plain_ups,
        "speedup": served_ups / plain_ups,
        "label_agreement_min": agree,
        "peak_budget_bytes": stats["peak_bytes"],
        "latency": lat,
    }


def heldout_accuracy(w, precision):
    """AUC / NLL of the held-out 20 % of the points under a map of the other 80 % (untimed)."""
    import torch
    from paper_2408_09066_amd import metrics, native
    tr, te = metrics.split_points(w.n, 0.8, np.random.default_rng(np.random.SeedSequence([2408, 2, 6])))
    m = native.Map(w.theta, w.layout, w.tiles)
    m.encode(torch.from_numpy(np.ascontiguousarray(w.xy[tr])).cuda(),
             torch.from_numpy(np.ascontiguousarray(w.label[tr])).cuda())
    heat, hmax = m.decode(w.grid, w.nx, w.ny, precision)
    ogm, _ = native.classify(heat, hmax, w.r_occ, w.r_emp, w.rho)
    r = metrics.evaluate(ogm.cpu().numpy(), w.grid, w.xy[te], w.label[te])
    m.close()
    r["split"] = "80/20 of the labelled points"
    return r


def volume_benchmark(steps: int = 10, warmup: int = 2, precision: str = "bf16x3"):
    """The 3-D extension at its benchmark size: one step = reset (memories zeroed), encode every
    point, decode every voxel, classify with the ball mask."""
    import torch
    from paper_2408_09066_amd import native, synth
    v = synth.volume("hall3d")
    dev = torch.device("cuda", 0)
    xyz = torch.from_numpy(v.xyz).to(dev)
    lab = torch.from_numpy(v.label).to(dev)
    heat = torch.empty((2, v.nz, v.ny, v.nx), dtype=torch.float32, device=dev)
    hmax = torch.empty(2, dtype=torch.float32, device=dev)
    ogm = torch.empty((v.nz, v.ny, v.nx), dtype=torch.float32, device=dev)
    out = torch.empty((v.nz, v.ny, v.nx), dtype=torch.uint8, device=dev)
    vol = native.Volume(v.theta, v.layout, v.tiles)
    E = torch.cuda.Event
    ev = {s_: [(E(enable_timing=True), E(enable_timing=True)) for _ in range(steps)] for s_ in native.STAGES}
    for evs in ev.values():
        for a, b in evs:
            a.record()
            b.record()

    def step():
        vol.reset()
        vol.encode(xyz, lab)
        vol.decode(v.grid, v.nx, v.ny, v.nz, precision, heat=heat, hmax=hmax)
        native.classify3(heat, hmax, v.r_occ, v.r_emp, v.rho, ogm=ogm, label=out)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    for i in range(steps):   # stage timings on steps of their own, as for the plane workload
        for s_ in native.STAGES:
            native.profile_events(s_, *ev[s_][i])
        step()
    torch.cuda.synchronize()
    for s_ in native.STAGES:
        native.profile_events(s_, None, None)
    vol.close()
    ms = {s_: float(np.mean([a.elapsed_time(b) for a, b in ev[s_]])) for s_ in native.STAGES}
    nvox = v.nx * v.ny * v.nz
    return {
        "workload": (f"{v.name}: {v.n} points, D={v.D}, l={v.ell} m, {v.tiles[0]}x{v.tiles[1]}x{v.tiles[2]} tiles, "
                     f"{v.nx}x{v.ny}x{v.nz} voxels at {v.grid[3]} m, ball r={v.r_occ}, {precision}"),
        "ms_per_step": el / steps * 1e3,
        "voxels_per_s": nvox * steps / el,
        "points_per_s": v.n * steps / el,
        "stage_ms": ms,
        "encode_tcexp_per_s": v.n * (v.D // 2 - 1) / (ms["encode"] * 1e-3) / 1e12,
        "encode_tflops": ENCODE3_OPS_PER_BIN * v.n * (v.D // 2 - 1) / (ms["encode"] * 1e-3) / 1e12,
        "encode_frac": ENCODE3_OPS_PER_BIN * v.n * (v.D // 2 - 1) / (ms["encode"] * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
        "encode_issue_bound_frac": v.n * (v.D // 2 - 1) / (ms["encode"] * 1e-3) / 1e12 / ISSUE_CEXP3_TPS,
        "decode_tflops_useful": 4.0 * v.D * nvox / (ms["decode"] * 1e-3) / 1e12,
    }


def stress_generate(n_updates: int, workers: int):
    """The large-map scenario and its first n_updates updates (host arrays), made before any
    GPU use: generation forks worker processes."""
    from paper_2408_09066_amd import synth
    sc = synth.stress_scenario()
    t = time.perf_counter()
    ups = sc.updates(n_updates, workers=workers)
    return sc, ups, time.perf_counter() - t


def stress_benchmark(sc, ups, precision: str = "bf16x3", load: float = 0.8):
    """Large-map stress: one map of 16 x 16 tiles at D = 16384 and a 4000 x 4000 grid, updated
    through the request loop, one request per 10 poses (118 800 points), each returning the
    grid's labels.  Passes, each on a fresh map: (1) every update queued at once with
    localized decoding (only tiles whose memories changed), (2) the same with full decodes,
    (3) Poisson arrivals at `load` x the throughput of (1), for the sustained latency."""
    import torch
    from paper_2408_09066_amd import native

    R = sc.r
    cells = sc.nx * sc.ny

    def run(srv, batch, local, arrivals=None):
        mid = srv.add_map(sc.theta, sc.layout, sc.tiles)
        items = [{"map_id": mid, "xy": xy, "label": lb, "grid": sc.grid, "nx": sc.nx, "ny": sc.ny,
                  "r_occ": R, "r_emp": R, "precision": precision, "local": local} for xy, lb in batch]
        t0 = time.perf_counter()
        if arrivals is None:
            tk = srv.submit_many(items)
        else:
            tk = []
            for it, a_ in zip(items, arrivals):
                while time.perf_counter() - t0 < a_:
                    pass
                tk.extend(srv.submit_many([it]))
        res = [srv.wait(t) for t, _ in tk]
        total_s = time.perf_counter() - t0
        assert all(r["status"] == 0 for r in res)
        lat = [(r["t_done_ns"] - r["t_submit_ns"]) * 1e-6 for r in res]
        svc = [(r["t_done_ns"] - r["t_start_ns"]) * 1e-6 for r in res]
        return total_s, lat, svc, tk[-1][1]["label"]

    # untimed, on a server of its own: kernels loaded
    warm = native.Server(max_inflight=2)
    run(warm, ups[:2], True)
    warm.close()
    torch.cuda.synchronize()
    free0, total = torch.cuda.mem_get_info()
    srv = native.Server(max_inflight=2)
    t_loc, _, svc_loc, lab_loc = run(srv, ups, True)
    free1, _ = torch.cuda.mem_get_info()
    t_full, _, svc_full, lab_full = run(srv, ups, False)
    rate = load * len(ups) / t_loc
    gaps = np.random.default_rng(np.random.SeedSequence([2408, 5, 5])).exponential(1.0 / rate, size=len(ups))
    t_open, lat_open, _, _ = run(srv, ups, True, np.cumsum(gaps))
    stats = srv.stats()
    srv.close()
    npts = sum(len(xy) for xy, _ in ups)
    steady = svc_loc[1:] if len(svc_loc) > 1 else svc_loc
    return {
        "workload": (f"{sc.name}: 200 m x 200 m world, {len(sc.world.rects)} rectangles + "
                     f"{len(sc.world.circles)} circles, {len(ups)} updates of "
                     f"{sc.poses_per_update} poses x {sc.beams} beams x (1 + {sc.empties}) = "
                     f"{sc.points_per_update} points, D={sc.D}, {sc.tiles[0]}x{sc.tiles[1]} tiles, "
                     f"{sc.nx}x{sc.ny} grid at {sc.grid[2]} m, r={R}, {precision} decode, "
                     "labels returned per update"),
        "updates": len(ups),
        "points": npts,
        "updates_per_s": len(ups) / t_loc,
        "points_per_s": npts / t_loc,
        "cells_per_s": cells * len(ups) / t_loc,
        "full_decode_updates_per_s": len(ups) / t_full,
        "label_agreement_full_decode": float(np.mean(lab_loc == lab_full)),
        "service_ms": {"first": svc_loc[0], "p50": percentile(steady, 50), "p99": percentile(steady, 99)},
        "full_decode_service_ms": {"p50": percentile(svc_full[1:], 50), "p99": percentile(svc_full[1:], 99)},
        "open_loop": {"load": load, "qps": rate, "latency_ms": {"p50": percentile(lat_open, 50),
                                                                "p99": percentile(lat_open, 99)}},
        "hbm_bytes_in_use": int(free0 - free1),   # one map, its tables and the server's buffers
        "hbm_total_bytes": int(total),
        "peak_budget_bytes": stats["peak_bytes"],
    }


def stage_rooflines(workload, stage_ms, n_points, D, ncell, precision):
    """Per-stage rooflines of one update: algorithmic work per launch / measured launch time,
    against the published peak of the unit that bounds the stage."""
    half = D // 2
    cexp = n_points * (half - 1)
    enc_ops = ENCODE_OPS_PER_BIN * cexp
    dec_flop = 4.0 * D * ncell            # 2 classes x D reals x (mul + add) per cell
    cls_bytes = 13.0 * ncell              # 2 x 4 B heat in; 4 B ogm + 1 B label out
    st = {
        "encode": {"bound": "alu", "achieved": enc_ops / (stage_ms["encode"] * 1e-3) / 1e12,
                   "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "ms": stage_ms["encode"],
                   "algorithmic": f"{ENCODE_OPS_PER_BIN} ops x {n_points} points x {half - 1} bins",
                   "tcexp_per_s": cexp / (stage_ms["encode"] * 1e-3) / 1e12,
                   "issue_bound_frac": cexp / (stage_ms["encode"] * 1e-3) / 1e12 / ISSUE_CEXP_TPS},
        "decode": {"bound": "mfma", "achieved": dec_flop / (stage_ms["decode"] * 1e-3) / 1e12,
                   "peak": PEAK_MFMA_TFLOPS[precision], "unit": "TFLOP/s", "ms": stage_ms["decode"],
                   "algorithmic": f"4 D flop x {ncell} cells (D = {D}), useful",
                   # MFMA work issued per useful flop (the split form multiplies three products)
                   "issued_per_useful": 3 if precision == "bf16x3" else 1},
        "classify": {"bound": "hbm", "achieved": cls_bytes / (stage_ms["classify"] * 1e-3) / 1e9,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "ms": stage_ms["classify"],
                     "algorithmic": f"13 B x {ncell} cells"},
    }
    for name, v in st.items():
        v["frac"] = v["achieved"] / v["peak"]
        tb = measured_traffic(workload, name)
        v["traffic"] = tb
        v["hbm_gbs"] = tb / (v["ms"] * 1e-3) / 1e9 if tb else None
    st["decode"]["issued_frac"] = st["decode"]["frac"] * st["decode"]["issued_per_useful"]
    return st


def timed_steps(step, steps: int, warmup: int, graph: bool = False):
    """warmup untimed steps; K steps for the throughput; K steps whose stage kernels record HIP
    events (per-kernel durations; per-step latency); optionally K replays of one step captured in
    a HIP graph.  Returns (seconds of the K plain steps, stage ms means, step latencies ms, graph
    ms per step or None)."""
    import torch
    from paper_2408_09066_amd import native
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    E = torch.cuda.Event
    step_ev = [(E(enable_timing=True), E(enable_timing=True)) for _ in range(steps)]
    stage_ev = {s_: [(E(enable_timing=True), E(enable_timing=True)) for _ in range(steps)] for s_ in native.STAGES}
    # torch creates an event on its first record: record each once so that its handle exists
    # before the library's kernels record it
    for evs in stage_ev.values():
        for a, b in evs:
            a.record()
            b.record()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # a timed kernel completion delays the next kernel by a few microseconds, so these are not
    # the steps the throughput is taken from
    for i in range(steps):
        for s_ in native.STAGES:
            native.profile_events(s_, *stage_ev[s_][i])
        step_ev[i][0].record()
        step()
        step_ev[i][1].record()
    torch.cuda.synchronize()
    for s_ in native.STAGES:
        native.profile_events(s_, None, None)
    lat = [a.elapsed_time(b) for a, b in step_ev]
    stage_ms = {s_: float(np.mean([a.elapsed_time(b) for a, b in stage_ev[s_]])) for s_ in native.STAGES}
    graph_ms = None
    if graph:
        try:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                step()
            g.replay()
            torch.cuda.synchronize()
            tg = time.perf_counter()
            for _ in range(steps):
                g.replay()
            torch.cuda.synchronize()
            graph_ms = (time.perf_counter() - tg) / steps * 1e3
            del g
        except RuntimeError as e:   # reported, not fatal: the eager figures stand
            print(f"graph capture failed: {e}", file=sys.stderr)
    return elapsed, stage_ms, lat, graph_ms


def world40_benchmark(precision: str, steps: int, warmup: int):
    """The plain method at real size: one step = reset + encode all 594 000 points + decode the
    800 x 800 grid + classify (inputs resident in HBM)."""
    import torch
    from paper_2408_09066_amd import native, synth
    w = synth.workload("world40")
    dev = torch.device("cuda", 0)
    xy = torch.from_numpy(w.xy).to(dev)
    lab = torch.from_numpy(w.label).to(dev)
    heat = torch.empty((2, w.ny, w.nx), dtype=torch.float32, device=dev)
    hmax = torch.empty(2, dtype=torch.float32, device=dev)
    ogm = torch.empty((w.ny, w.nx), dtype=torch.float32, device=dev)
    out_lab = torch.empty((w.ny, w.nx), dtype=torch.uint8, device=dev)
    m = native.Map(w.theta, w.layout, w.tiles, device=0)

    def step():
        m.reset()
        m.encode(xy, lab)
        m.decode(w.grid, w.nx, w.ny, precision, heat=heat, hmax=hmax)
        native.classify(heat, hmax, w.r_occ, w.r_emp, w.rho, ogm=ogm, label=out_lab)

    elapsed, stage_ms, lat, graph_ms = timed_steps(step, steps, warmup, graph=True)
    m.close()
    ncell = w.nx * w.ny
    st = stage_rooflines("world40", stage_ms, w.n, w.D, ncell, precision)
    return {
        "workload": (f"{w.name}: {w.n} points ({int(w.label.sum())} occupied), D={w.D}, l={w.ell} m, "
                     f"{w.tiles[0]}x{w.tiles[1]} tiles, {w.nx}x{w.ny} grid at {w.grid[2]} m, disk r={w.r_occ}; "
                     "step = reset + encode all points + decode + classify"),
        "precision": precision,
        "ms_per_step": elapsed / steps * 1e3,
        "cells_per_s": ncell * steps / elapsed,
        "points_per_s": w.n * steps / elapsed,
        "gemm_cells_per_s": ncell / (stage_ms["decode"] * 1e-3),
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
        "graph_ms_per_step": graph_ms,
        "stages": st,
    }


def headline(args, sc, ups, gen_s, n_head):
    """The large-map update step, timed: the bench line's headline fields."""
    import torch
    from paper_2408_09066_amd import native
    dev = torch.device("cuda", 0)
    # ---- headline: incremental updates of the large map, inputs resident in HBM
    dev_ups = [(torch.from_numpy(xy).to(dev), torch.from_numpy(lb).to(dev)) for xy, lb in ups[:n_head]]
    heat = torch.empty((2, sc.ny, sc.nx), dtype=torch.float32, device=dev)
    hmax = torch.empty(2, dtype=torch.float32, device=dev)
    ogm = torch.empty((sc.ny, sc.nx), dtype=torch.float32, device=dev)
    out_lab = torch.empty((sc.ny, sc.nx), dtype=torch.uint8, device=dev)
    m = native.Map(sc.theta, sc.layout, sc.tiles, device=0)
    nxt = [0]

    def step():
        xy, lb = dev_ups[nxt[0] % len(dev_ups)]
        nxt[0] += 1
        m.encode(xy, lb)
        m.decode(sc.grid, sc.nx, sc.ny, args.precision, heat=heat, hmax=hmax)
        native.classify(heat, hmax, sc.r, sc.r, 0.0, ogm=ogm, label=out_lab)

    free0, total = torch.cuda.mem_get_info()
    elapsed, stage_ms, lat, _ = timed_steps(step, args.steps, args.warmup)
    free1, _ = torch.cuda.mem_get_info()
    m.close()
    del dev_ups
    K = args.steps
    ncell = sc.nx * sc.ny
    npts = sc.points_per_update
    stages = stage_rooflines(sc.name, stage_ms, npts, sc.D, ncell, args.precision)
    dom = max(stages, key=lambda s_: stages[s_]["ms"])
    d = stages[dom]
    roof = {"bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"], "unit": d["unit"],
            "frac": d["frac"], "traffic": d["traffic"], "kernel": dom,
            "traffic_source": (f"rocprofv3 FETCH_SIZE / WRITE_SIZE of an earlier profiled run on these kernel "
                               f"sources ({os.path.relpath(traffic_file(sc.name), ROOT)}), copy-calibrated"
                               if d["traffic"] else "no counter run on these kernel sources")}
    if dom == "decode":
        roof["issued_frac"] = d["issued_frac"]

    result = {
        "metric": "heatmap cells decoded/sec + points encoded/sec; p50/p99 map-update latency",
        "value": ncell * K / elapsed,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": elapsed / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else f"f32 ({args.precision} similarity operands)",
        "data": "synthetic",
        "config": {
            "workload": (f"{sc.name}: 200 m x 200 m world, {len(sc.world.rects)} rectangles + "
                         f"{len(sc.world.circles)} circles; one step = one incremental map update of "
                         f"{sc.poses_per_update} poses x {sc.beams} beams x (1 + {sc.empties}) = {npts} points "
                         f"(resident in HBM), D={sc.D}, l={sc.ell} m, {sc.tiles[0]}x{sc.tiles[1]} tiles, "
                         f"{sc.nx}x{sc.ny} grid at {sc.grid[2]} m decoded in full, disk r={sc.r}"),
            "precision": args.precision,
        },
        "points_per_s": npts * K / elapsed,
        # cells/s of the similarity GEMM alone and of decode + classification, from the same
        # launches' timings
        "gemm_cells_per_s": ncell / (stage_ms["decode"] * 1e-3),
        "decode_classify_cells_per_s": ncell / ((stage_ms["decode"] + stage_ms["classify"]) * 1e-3),
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99),
                       "what": "device time of one update (encode + decode + classify), HIP events"},
        "hbm_bytes_map_and_buffers": int(free0 - free1),
        "input_sha256": {"theta": hashlib.sha256(np.ascontiguousarray(sc.theta).tobytes()).hexdigest(),
                         "update0_xy": hashlib.sha256(np.ascontiguousarray(ups[0][0]).tobytes()).hexdigest()},
        "generation_s": gen_s,
        "stages": stages,
        "roofline": roof,
    }
    return result


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16", "fp16", "bf16x3"],
                    help="operands of the headline's similarity contraction; bf16x3 (hi+lo split) meets "
                         "the fp32 accuracy bar")
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of oracle work for the CPU baseline (0 disables it)")
    ap.add_argument("--headline", type=int, default=1,
                    help="run the headline (0: only the other sections, for profiling them)")
    ap.add_argument("--world40", type=int, default=1, help="also run the 40 m world (fp32 and bf16 hi+lo)")
    ap.add_argument("--serving", type=int, default=1,
                    help="also run the request-loop benchmark (256 updates of 16 maps)")
    ap.add_argument("--stress", type=int, default=200,
                    help="updates of the large map served through the request loop (0 disables it)")
    ap.add_argument("--volume", type=int, default=1, help="also run the 3-D benchmark")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="processes that generate the scans")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 512 MiB device to device three times (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        n = 512 << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 3}), flush=True)
        return 0

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the hot path here is the single-GPU kernel set)", file=sys.stderr)
        return 2

    # scans are generated before any GPU use (generation forks worker processes)
    n_head = args.warmup + 2 * args.steps
    sc, ups, gen_s = stress_generate(max(n_head, args.stress), args.workers)

    import torch
    from paper_2408_09066_amd import native

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    native.load()
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)

    K = args.steps
    t_start = time.perf_counter()

    def done(section):
        # one line per finished section on stderr (the JSON line alone goes to stdout)
        print(f"[bench] {section} done at {time.perf_counter() - t_start:.1f} s", file=sys.stderr, flush=True)

    if args.headline:
        result = headline(args, sc, ups, gen_s, n_head)
        done("headline")
    else:
        # a run of the other sections alone (for profiling them): no headline figure
        result = {"metric": "heatmap cells decoded/sec + points encoded/sec; p50/p99 map-update latency",
                  "value": None, "unit": "cells/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
                  "note": "headline not run (--headline 0)"}
    result["measured_peaks"] = {"hbm_copy_gbs": measured_hbm_copy_gbs(), "datasheet_hbm_gbs": PEAK_HBM_GBS}
    if args.world40:
        result["world40"] = {}
        for p_ in ("fp32", "bf16x3"):
            result["world40"][p_] = world40_benchmark(p_, K, args.warmup)
            done(f"world40 {p_}")
        from paper_2408_09066_amd import synth
        result["world40"]["accuracy"] = heldout_accuracy(synth.workload("world40"), "bf16x3")
        done("world40 accuracy")
    if args.volume:
        result["volume"] = volume_benchmark()
        done("volume")
    if args.serving:
        result["serving"] = serving_benchmark()
        done("serving")
    if args.stress > 0:
        result["stress_serving"] = stress_benchmark(sc, ups[:args.stress])
        done("stress serving")
    if args.cpu_budget > 0:
        result["cpu_baseline"] = cpu_baseline(sc, ups[0][0], ups[0][1], args.cpu_budget)
        done("cpu baseline")
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
