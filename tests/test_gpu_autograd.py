"""The differentiable field demag_field(m, thickness, plan): backward through
torch.autograd against the plan's VJP and against the oracle's transposed
field and thickness gradient (the thickness optimisation of Sec. 4 needs
d<h>/dt), with several stacks per plan so that the per-stack sum of the
thickness gradients runs, and with the thickness on the host and on the GPU."""
import numpy as np
import pytest

import oracle
from paper_1910_07054_amd import hfd
from paper_1910_07054_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hfd.load()


def _stacks():
    """Two 3-layer stacks that differ in the middle thickness, shared gaps."""
    t = np.array([[1.0, 0.7, 2.3], [1.0, 1.1, 2.3]])
    gaps = np.array([0.5, 0.4])
    zb = np.zeros_like(t)
    for g in range(2):
        for l in range(1, 3):
            zb[g, l] = zb[g, l - 1] + t[g, l - 1] + gaps[l - 1]
    return t, zb


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("thickness_on_gpu", [False, True])
def test_demag_field_backward_matches_vjp_and_oracle(fp64, thickness_on_gpu):
    import torch
    nx, ny, dx, dy = 12, 9, 2.0, 2.5
    t, zb = _stacks()
    G, nz = t.shape
    bpg = 2
    B = G * bpg
    rng = np.random.default_rng(2024)
    m_np = W.random_unit(rng, (B, nz, ny, nx)).transpose(1, 0, 2, 3, 4).copy()  # [B][3][nz][ny][nx]
    g_np = rng.standard_normal((B, 3, nz, ny, nx))
    dt = torch.float64 if fp64 else torch.float32
    flags = hfd.HFD_FP64 if fp64 else hfd.HFD_FP32
    plan = hfd.Plan(nx, ny, dx, dy, t, zb, batch_max=B, flags=flags)
    dev = "cuda" if thickness_on_gpu else "cpu"
    m = torch.tensor(m_np, dtype=dt, device="cuda", requires_grad=True)
    th = torch.tensor(t, dtype=torch.float64, device=dev, requires_grad=True)
    gh = torch.tensor(g_np, dtype=dt, device="cuda")
    h = hfd.demag_field(m, th, plan)
    assert h.shape == m.shape and h.dtype == dt
    gm, gth = torch.autograd.grad(h, (m, th), grad_outputs=gh)
    assert gth.device == th.device and gth.dtype == th.dtype and gth.shape == th.shape

    # the same products through the plan directly
    vm, vt = plan.vjp(m.detach(), gh)
    assert torch.equal(gm, vm)
    vt_sum = vt.reshape(G, bpg, nz).sum(1).cpu()
    assert torch.allclose(gth.detach().cpu(), vt_sum, rtol=1e-12, atol=0)

    # and against the oracle: transposed field and thickness gradient per state
    mused = m.detach().double().cpu().numpy()
    gused = gh.double().cpu().numpy()
    tol_m = 1e-10 if fp64 else 1e-5
    tol_t = 1e-10 if fp64 else 2e-5
    ref_t = np.zeros((G, nz))
    for b in range(B):
        s = b // bpg
        ref_m = oracle.field(nx, ny, dx, dy, zb[s], t[s], gused[b], transpose=True)
        got_m = gm[b].double().cpu().numpy()
        assert np.abs(got_m - ref_m).max() < tol_m * np.abs(ref_m).max()
        ref_t[s] += oracle.thickness_grad(nx, ny, dx, dy, zb[s], t[s], mused[b], gused[b])
    got_t = gth.detach().cpu().numpy()
    assert np.abs(got_t - ref_t).max() < tol_t * np.abs(ref_t).max(), (got_t, ref_t)
    plan.destroy()


def test_demag_field_rejects_mismatched_thickness_and_inputs():
    import torch
    t, zb = _stacks()
    plan = hfd.Plan(8, 6, 2.0, 2.0, t[:1], zb[:1], batch_max=1)
    m = torch.zeros((1, 3, 3, 6, 8), device="cuda", requires_grad=True)
    with pytest.raises(ValueError):
        hfd.demag_field(m, torch.tensor(t[1]), plan)        # not the plan's geometry
    with pytest.raises(ValueError):
        plan.field(m.detach().double())                      # wrong dtype for an FP32 plan
    with pytest.raises(ValueError):
        plan.field(m.detach().cpu())                         # host tensor
    with pytest.raises(ValueError):
        plan.field(m.detach().transpose(3, 4))               # wrong shape / not contiguous
    with pytest.raises(ValueError):
        plan.field(m.detach().expand(2, 3, 3, 6, 8))         # batch above batch_max
    plan.destroy()
