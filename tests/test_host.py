"""Host-side contract, on the CPU: the C ABI validates its arguments before it touches a device
and reports every failure as a status with a message (no GPU is needed for that); the benchmark
refuses more than one GPU; the synthetic workloads have the sizes the benchmark and the parity
tests are quoted on, and are reproducible."""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2408_09066_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2408_09066_amd", "libvsaogm.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2408_09066_amd import native
    return native, native.load()


def map_desc(native, theta, layout=(-1.0, -1.0, 1.0, 1.0), tiles=(2, 2), dim=None):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    return native.MapDesc(th.shape[0] if dim is None else dim, th.ctypes.data, *layout, *tiles, 0), th


def test_map_descriptors_are_validated_before_the_device(lib):
    native, L = lib
    th = synth.make_theta(64, 0.3, np.random.default_rng(1))
    h = ctypes.c_void_p()
    cases = {
        "odd dim": dict(dim=63),
        "dim too small": dict(dim=2),
        "no tiles": dict(tiles=(0, 2)),
        "too many tiles": dict(tiles=(65, 1)),
        "empty layout": dict(layout=(1.0, -1.0, 1.0, 1.0)),
        "non-finite layout": dict(layout=(-1.0, -1.0, float("inf"), 1.0)),
    }
    for name, kw in cases.items():
        d, keep = map_desc(native, th, **kw)
        assert L.vsaogm_map_create(ctypes.byref(d), ctypes.byref(h)) == native.EINVAL, name
        assert L.vsaogm_last_error(), name
    bad = th.copy()
    bad[5, 1] += 0.5                         # breaks theta[D-k] = -theta[k]
    d, keep = map_desc(native, bad)
    assert L.vsaogm_map_create(ctypes.byref(d), ctypes.byref(h)) == native.EINVAL
    assert b"conjugate-symmetric" in L.vsaogm_last_error()
    bad = th.copy()
    bad[0, 0] = 0.1                          # bin 0 must carry no phase
    d, keep = map_desc(native, bad)
    assert L.vsaogm_map_create(ctypes.byref(d), ctypes.byref(h)) == native.EINVAL
    bad = th.copy()
    bad[3, 0] = np.nan
    d, keep = map_desc(native, bad)
    assert L.vsaogm_map_create(ctypes.byref(d), ctypes.byref(h)) == native.EINVAL
    assert L.vsaogm_map_create(None, ctypes.byref(h)) == native.EINVAL


def test_volume_and_server_descriptors_are_validated(lib):
    native, L = lib
    th = synth.make_theta3(64, 0.3, np.random.default_rng(2))
    h = ctypes.c_void_p()

    def vdesc(theta, box=(-1, -1, 0, 1, 1, 1), tiles=(2, 2, 1)):
        t = np.ascontiguousarray(theta, dtype=np.float64)
        return native.VolumeDesc(t.shape[0], t.ctypes.data, *[float(b) for b in box], *tiles, 0), t

    for kw in (dict(tiles=(1, 0, 1)), dict(box=(-1, -1, 1, 1, 1, 1)), dict(tiles=(64, 64, 2))):
        d, keep = vdesc(th, **kw)
        assert L.vsaogm_volume_create(ctypes.byref(d), ctypes.byref(h)) == native.EINVAL, kw
    bad = th.copy()
    bad[7, 2] += 1.0
    d, keep = vdesc(bad)
    assert L.vsaogm_volume_create(ctypes.byref(d), ctypes.byref(h)) == native.EINVAL
    for inflight, queue in ((0, 16), (33, 16), (4, 0)):
        sd = native.ServerDesc(0, inflight, queue, 0)
        assert L.vsaogm_server_create(ctypes.byref(sd), ctypes.byref(h)) == native.EINVAL


def test_calls_on_null_handles_return_einval(lib):
    native, L = lib
    assert L.vsaogm_encode(None, None, None, 5, None) == native.EINVAL
    assert L.vsaogm_decode(None, None, 0, None, None, None) == native.EINVAL
    assert L.vsaogm_map_reset(None, None) == native.EINVAL
    assert L.vsaogm_volume_encode(None, None, None, 5, None) == native.EINVAL
    assert L.vsaogm_volume_reset(None, None) == native.EINVAL
    assert L.vsaogm_fuse(None, None, None) == native.EINVAL
    assert L.vsaogm_fuse_many(None, None, 0, None) == native.EINVAL
    srcs = (ctypes.c_void_p * 2)(None, None)
    # a non-null handle is never dereferenced before its arguments are checked: n < 0, a missing
    # source array and a null source are refused first
    fake = ctypes.c_void_p(1)
    assert L.vsaogm_fuse_many(fake, None, -1, None) == native.EINVAL
    assert L.vsaogm_fuse_many(fake, None, 2, None) == native.EINVAL
    assert L.vsaogm_fuse_many(fake, srcs, 2, None) == native.EINVAL
    assert L.vsaogm_classify(None, None, None, 1, 1, 0.0, None, None, 0, None) == native.EINVAL
    assert L.vsaogm_classify3(None, None, None, 1, 1, 0.0, None, None, 0, None) == native.EINVAL
    assert L.vsaogm_last_error()


def test_valid_map_without_a_device_is_a_device_error(lib):
    native, L = lib
    if os.path.exists("/dev/kfd"):
        pytest.skip("a GPU may be present")
    th = synth.make_theta(64, 0.3, np.random.default_rng(1))
    d, keep = map_desc(native, th)
    h = ctypes.c_void_p()
    rc = L.vsaogm_map_create(ctypes.byref(d), ctypes.byref(h))
    assert rc in (native.EDEVICE, native.EINVAL) and not h.value
    assert L.vsaogm_last_error()


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_workload_sizes_and_reproducibility():
    w = synth.workload("world40")
    assert (w.n, int(w.label.sum()), w.D, tuple(w.tiles), w.nx, w.ny) == (594000, 54000, 8192, (4, 4), 800, 800)
    assert (w.r_occ, w.r_emp, w.grid[2]) == (3, 3, 0.05)
    w2 = synth.workload("world40")
    assert np.array_equal(w.xy, w2.xy) and np.array_equal(w.label, w2.label) and np.array_equal(w.theta, w2.theta)
    t = synth.workload("toy_room")
    assert (t.n, t.D, t.nx, t.ny) == (2160, 1024, 128, 128)
    v = synth.volume("room3d")
    assert (v.n, v.D, (v.nx, v.ny, v.nz)) == (7200, 512, (32, 32, 16))
    assert np.array_equal(v.xyz, synth.volume("room3d").xyz)
    th = w.theta
    assert np.all(th[0] == 0) and np.all(th[w.D // 2] == 0)
    assert np.array_equal(th[w.D // 2 + 1:], -th[1:w.D // 2][::-1])


def test_stress_updates_are_independent_of_generation_order():
    sc = synth.stress_scenario(n_poses=30)
    ups = sc.updates(limit=3, workers=1)
    assert len(ups) == 3 and all(len(xy) == 11880 * 10 for xy, _ in ups)
    # each update draws from its own sub-stream: update 2 alone equals update 2 in sequence
    xy2, lb2 = sc.update(2)
    assert np.array_equal(xy2, ups[2][0]) and np.array_equal(lb2, ups[2][1])


def test_binding_rejects_wrong_tensors_before_the_library():
    """The binding checks device, dtype, shape and layout of every tensor it passes on."""
    torch = pytest.importorskip("torch")
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_2408_09066_amd import native
    heat = torch.zeros((2, 4, 5), dtype=torch.float32)
    hmax = torch.zeros(2, dtype=torch.float32)
    with pytest.raises(ValueError, match="device tensor"):
        native.classify(heat, hmax, 1, 1)                        # host memory
    with pytest.raises(ValueError):
        native.classify3(heat.reshape(2, 1, 4, 5).double(), hmax, 1, 1)   # wrong dtype (and host)
    t = native._tensor
    fake = type("T", (), {"is_cuda": True, "dtype": "torch.float64", "shape": (2, 4, 5),
                          "is_contiguous": lambda self: True})()
    with pytest.raises(ValueError, match="float32"):
        t(fake, "float32", (2, 4, 5), "heat")
    fake.dtype = "torch.float32"
    with pytest.raises(ValueError, match="shape"):
        t(fake, "float32", (2, 5, 4), "heat")
    fake.is_contiguous = lambda: False
    with pytest.raises(ValueError, match="contiguous"):
        t(fake, "float32", (2, 4, 5), "heat")


def test_rejected_labels_contract(lib):
    """A label outside {0, 1} names no memory of Algorithm 1: the encode skips and counts such
    points on the device (asynchronously) and vsaogm_map_take_rejected reports the count; the
    header states it, and the count query validates its arguments before any device work."""
    native, L = lib
    with open(os.path.join(ROOT, "include", "vsaogm.h")) as fh:
        hdr = fh.read()
    assert "vsaogm_map_take_rejected reports the count" in hdr
    v = ctypes.c_int64(-1)
    assert L.vsaogm_map_take_rejected(None, None, ctypes.byref(v)) == native.EINVAL
    assert L.vsaogm_volume_take_rejected(None, None, ctypes.byref(v)) == native.EINVAL
    assert L.vsaogm_last_error()


def test_noalloc_classify3_rejects_volumes_beyond_its_scratch(lib):
    """The allocation-free volume classification refuses, before any device work, a volume whose
    entropy terms would not fit its fixed scratch (radii above 4 need 2 floats per voxel, at most
    2^21 voxels), and accepts the argument checks of vsaogm_classify3 otherwise."""
    native, L = lib
    g = native.Grid3Desc(0.0, 0.0, 0.0, 1.0, 256, 128, 65)        # 2 129 920 voxels
    fake = ctypes.c_void_p(4096)                                  # never dereferenced: refused first
    rc = L.vsaogm_classify3_noalloc(ctypes.byref(g), fake, fake, 5, 3, 0.0, None, fake, 0, None)
    assert rc == native.EINVAL
    assert b"2097152" in L.vsaogm_last_error()
    assert L.vsaogm_classify3_noalloc(None, fake, fake, 5, 3, 0.0, None, fake, 0, None) == native.EINVAL
    assert L.vsaogm_classify3_noalloc(ctypes.byref(g), fake, fake, 25, 3, 0.0, None, fake, 0, None) == native.EINVAL
