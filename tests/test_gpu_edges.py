"""Edge cases of the field path: the largest lateral sizes (4096-point
transforms), the largest layer count, and rejected batch sizes."""
import ctypes

import numpy as np
import pytest

import oracle
from hfd_testlib import plan_for, rel_err, run_field
from paper_1910_07054_amd import hfd
from paper_1910_07054_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hfd.load()


# (nx, ny, nz): nx = 2048 -> Lx = 4096 (x passes at their largest length),
# ny = 2048 -> Ly = 4096 (five-pass y transforms at their largest length),
# nz = 64 (largest layer count; 16 target groups in the five-pass mixing)
EDGE = [(2048, 3, 1), (3, 2048, 2), (7, 5, 64)]


@pytest.mark.parametrize("fp64", [False, True], ids=["fp32", "fp64"])
@pytest.mark.parametrize("case", EDGE, ids=lambda c: "x".join(map(str, c)))
def test_largest_sizes_match_bruteforce(case, fp64):
    nx, ny, nz = case
    wl = W.small_case(nx, ny, nz, seed=1200 + nz, batch=1)
    plan = plan_for(wl, flags=hfd.HFD_FP64 if fp64 else hfd.HFD_FP32)
    h, mused = run_field(plan, wl.m)
    ref = oracle.field(nx, ny, wl.dx, wl.dy, wl.z_bottom[0], wl.thickness[0], mused[0])
    assert rel_err(h[0], ref) < (1e-10 if fp64 else 1e-5)
    plan.destroy()


def test_equidistant_largest_layer_count():
    nx, ny, nz, t = 6, 5, 64, 0.5
    rng = np.random.default_rng(1264)
    m = W.random_unit(rng, (nz, ny, nx))[None]
    zb = np.arange(nz) * t
    plan = hfd.Plan(nx, ny, 2.0, 1.5, np.full(nz, t), zb, batch_max=1, flags=hfd.HFD_EQUIDISTANT)
    assert plan.info().Lz == 128
    h, mused = run_field(plan, m)
    ref = oracle.field(nx, ny, 2.0, 1.5, zb, np.full(nz, t), mused[0])
    assert rel_err(h[0], ref) < 1e-5
    plan.destroy()


def test_rejected_batch_sizes():
    import torch
    wl = W.small_case(8, 6, 2, seed=1300, batch=2)
    plan = plan_for(wl)
    m = torch.zeros((2, 3, 2, 6, 8), device="cuda")
    h = torch.empty_like(m)
    lib = hfd.load()
    assert lib.hfd_demag_field(plan.handle, m.data_ptr(), h.data_ptr(), 0, None) == hfd.HFD_EINVAL
    assert lib.hfd_demag_field(plan.handle, m.data_ptr(), h.data_ptr(), -1, None) == hfd.HFD_EINVAL
    assert lib.hfd_demag_field(plan.handle, m.data_ptr(), h.data_ptr(), 3, None) == hfd.HFD_EBATCH
    # aliasing input and output is rejected
    assert lib.hfd_demag_field(plan.handle, m.data_ptr(), m.data_ptr(), 1, None) == hfd.HFD_EINVAL
    assert lib.hfd_demag_field(plan.handle, m.data_ptr(), h.data_ptr(), 2, None) == hfd.HFD_OK
    torch.cuda.synchronize()
    plan.destroy()
