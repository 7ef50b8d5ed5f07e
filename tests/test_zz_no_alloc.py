"""hfd_demag_field_noalloc (the x-pass spectra in the library's per-GPU
device scratch) against hfd_demag_field, called through the C ABI: two calls
in a row on one plan, the second with a smaller batch, plus the host-side
rejection of a batch whose spectra exceed the scratch."""
import ctypes

import numpy as np
import pytest

from paper_1910_07054_amd import hfd
from paper_1910_07054_amd import workloads as W

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 32 << 20


def _plan(nx, ny, nz, batch_max, seed):
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.5, 2.5, nz)
    z = np.concatenate([[0.0], np.cumsum(t[:-1] + rng.uniform(0.2, 1.0, nz - 1))])
    return hfd.Plan(nx, ny, 2.0, 2.5, t, z, batch_max=batch_max)


def _m(B, nz, ny, nx, seed):
    import torch
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((B, 3, nz, ny, nx))
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    return torch.from_numpy(m.astype(np.float32)).cuda()


def _noalloc(plan, m, h):
    import torch
    st = hfd.load().hfd_demag_field_noalloc(plan.handle, ctypes.c_void_p(m.data_ptr()),
                                           ctypes.c_void_p(h.data_ptr()), int(m.shape[0]),
                                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def test_noalloc_matches_field_twice_second_smaller():
    import torch
    nx, ny, nz = 200, 136, 5          # Lx = 512, Ly = 512: the exact-layer fused kernel
    plan = _plan(nx, ny, nz, batch_max=3, seed=11)
    try:
        for B, seed in ((3, 21), (1, 22)):
            m = _m(B, nz, ny, nx, seed)
            ref = plan.field(m)
            got = torch.full_like(m, float("nan"))
            assert _noalloc(plan, m, got) == hfd.HFD_OK, hfd.load().hfd_last_error()
            torch.cuda.synchronize()
            r, g = ref.cpu().numpy(), got.cpu().numpy()
            assert np.isfinite(g).all()
            err = np.abs(g - r).max() / np.abs(r).max()
            assert err <= 1e-6, (B, err)
    finally:
        plan.destroy()


def test_noalloc_generic_fused_kernel_and_second_plan():
    import torch
    # 48 x 40 cells (Ly = 128: the generic fused kernel), then a second plan on
    # the same GPU sharing the scratch
    plans = [_plan(48, 40, 3, batch_max=2, seed=31), _plan(20, 12, 2, batch_max=2, seed=32)]
    try:
        for plan, B in zip(plans, (2, 1)):
            m = _m(B, plan.nz, plan.ny, plan.nx, 40 + B)
            ref = plan.field(m)
            got = torch.full_like(m, float("nan"))
            assert _noalloc(plan, m, got) == hfd.HFD_OK, hfd.load().hfd_last_error()
            torch.cuda.synchronize()
            err = np.abs(got.cpu().numpy() - ref.cpu().numpy()).max() / np.abs(ref.cpu().numpy()).max()
            assert err <= 1e-6, err
    finally:
        for p in plans:
            p.destroy()


def test_noalloc_rejects_batch_beyond_scratch():
    import torch
    nx, ny, nz = 256, 256, 8            # 12.6 MB of spectra per state: 3 states exceed 32 MiB
    plan = _plan(nx, ny, nz, batch_max=3, seed=51)
    try:
        per_state = 3 * nz * 256 * ny * 8
        assert 2 * per_state <= SCRATCH_BYTES < 3 * per_state
        m = torch.zeros((3, 3, nz, ny, nx), dtype=torch.float32, device="cuda")
        h = torch.empty_like(m)
        assert _noalloc(plan, m, h) == hfd.HFD_EINVAL
        assert b"scratch" in hfd.load().hfd_last_error()
        wl = W.small_case(nx, ny, nz, seed=5)
        m2 = torch.from_numpy(np.ascontiguousarray(wl.m[:1]).astype(np.float32)).cuda()
        m2 = m2.expand(2, -1, -1, -1, -1).contiguous()
        h2 = torch.empty_like(m2)
        assert _noalloc(plan, m2, h2) == hfd.HFD_OK
        ref = plan.field(m2)
        torch.cuda.synchronize()
        assert np.abs(h2.cpu().numpy() - ref.cpu().numpy()).max() <= 1e-6 * np.abs(ref.cpu().numpy()).max()
    finally:
        plan.destroy()


def test_noalloc_split_pass_plan_is_not_supported():
    import torch
    rng = np.random.default_rng(3)
    plan = hfd.Plan(16, 16, 1.0, 1.0, rng.uniform(0.5, 1.5, 2), None, batch_max=1,
                    flags=hfd.HFD_SPLIT_PASSES)
    try:
        m = torch.zeros((1, 3, 2, 16, 16), dtype=torch.float32, device="cuda")
        h = torch.empty_like(m)
        assert _noalloc(plan, m, h) == hfd.HFD_ENOTSUP
    finally:
        plan.destroy()
