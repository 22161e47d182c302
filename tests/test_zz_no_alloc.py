"""vsaogm_classify3_noalloc (the volume classification for callers that cannot allocate device
memory: its entropy scratch is a fixed per-device array) against vsaogm_classify3 through the C
ABI: two calls in a row, the second on a smaller volume, both with radii that need the scratch,
then one with radii that need none.  Same kernels on the same inputs: outputs must be identical.
"""
import sys

import numpy as np
import pytest

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


def volume_heat(seed, nx, ny, nz):
    rng = np.random.default_rng(np.random.SeedSequence([2408, 90, seed]))
    heat = rng.uniform(-0.3, 1.0, size=(2, nz, ny, nx)).astype(np.float32)
    hmax = heat.reshape(2, -1).max(axis=1).astype(np.float32)
    return heat, hmax


def test_noalloc_classify3_matches_classify3(torch_cuda):
    from paper_2408_09066_amd import native
    torch = torch_cuda
    cases = [((48, 40, 28), (6, 5), 1), ((19, 23, 9), (7, 3), 2), ((30, 20, 10), (2, 4), 3)]
    got = []
    for (nx, ny, nz), (r_occ, r_emp), seed in cases:
        say(f"[gpu] classify3_noalloc {nx}x{ny}x{nz} radii ({r_occ}, {r_emp})")
        heat, hmax = volume_heat(seed, nx, ny, nz)
        h, m = torch.from_numpy(heat).cuda(), torch.from_numpy(hmax).cuda()
        ogm, lab = native.classify3(h, m, r_occ, r_emp, 0.0, noalloc=True)
        torch.cuda.synchronize()
        got.append((ogm.cpu().numpy(), lab.cpu().numpy()))
    for ((nx, ny, nz), (r_occ, r_emp), seed), (ogm_n, lab_n) in zip(cases, got):
        heat, hmax = volume_heat(seed, nx, ny, nz)
        h, m = torch.from_numpy(heat).cuda(), torch.from_numpy(hmax).cuda()
        ogm, lab = native.classify3(h, m, r_occ, r_emp, 0.0)
        torch.cuda.synchronize()
        ogm, lab = ogm.cpu().numpy(), lab.cpu().numpy()
        say(f"  {nx}x{ny}x{nz}: ogm max-abs {np.max(np.abs(ogm - ogm_n)):.3e}, "
            f"{int(np.sum(lab != lab_n))} label differences")
        assert np.array_equal(ogm, ogm_n)
        assert np.array_equal(lab, lab_n)
