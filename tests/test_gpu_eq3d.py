"""Equidistant stacks (eq. FFT_3D of Sec. 3.1): the layer sum by a transform
along z, against the oracle's direct sum and 3-D transform."""
import numpy as np
import pytest

import oracle
from hfd_testlib import rel_err, run_field
from paper_1910_07054_amd import hfd
from paper_1910_07054_amd import workloads as W

pytestmark = pytest.mark.gpu

# (nx, ny, nz, thickness, pitch): touching and spaced layers; Lz from 2 to 128
CASES = [(20, 12, 1, 0.9, 0.9), (17, 9, 2, 0.7, 1.2), (24, 20, 5, 1.0, 1.0), (13, 30, 8, 0.6, 1.1),
         (9, 7, 13, 0.8, 0.8), (10, 6, 33, 0.5, 0.5)]
DX, DY = 2.0, 1.5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hfd.load()


def _plan(nx, ny, nz, t, pitch, fp64, B):
    zb = np.arange(nz) * pitch
    flags = hfd.HFD_EQUIDISTANT | (hfd.HFD_FP64 if fp64 else hfd.HFD_FP32)
    return hfd.Plan(nx, ny, DX, DY, np.full(nz, t), zb, batch_max=B, flags=flags), zb


@pytest.mark.parametrize("fp64", [False, True], ids=["fp32", "fp64"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:3])))
def test_equidistant_field_matches_bruteforce(case, fp64):
    nx, ny, nz, t, pitch = case
    rng = np.random.default_rng(900 + nz)
    B = 2
    m = np.stack([W.random_unit(rng, (nz, ny, nx)) for _ in range(B)])
    plan, zb = _plan(nx, ny, nz, t, pitch, fp64, B)
    inf = plan.info()
    assert inf.equidistant == 1 and inf.Lz >= 2 * nz
    h, mused = run_field(plan, m)
    for b in range(B):
        ref = oracle.field(nx, ny, DX, DY, zb, np.full(nz, t), mused[b])
        assert rel_err(h[b], ref) < (1e-10 if fp64 else 1e-5), b
    plan.destroy()


def test_equidistant_tensor_matches_oracle_transform():
    nx, ny, nz, t, pitch = 11, 7, 6, 0.9, 1.3
    plan, _ = _plan(nx, ny, nz, t, pitch, True, 1)
    inf = plan.info()
    got = plan.export_fourier_tensor()                      # [kx][kz][c][ky]
    T = oracle.fourier_tensor3(nx, ny, DX, DY, nz, t, pitch, Lx=inf.Lx, Ly=inf.Ly, Lz=inf.Lz)
    ref = -T.real / (inf.Lx * inf.Ly * inf.Lz)              # [c][kz][ky][kx]
    QX, QZ, QY = inf.Lx // 2 + 1, inf.Lz // 2 + 1, inf.Ly // 2 + 1
    ref = np.transpose(ref[:, :QZ, :QY, :QX], (3, 1, 0, 2))
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
    plan.destroy()


def test_equidistant_agrees_with_hybrid_path():
    """Same equidistant stack through the explicit layer sum (fused y-pass)
    and through the z transform."""
    nx, ny, nz, t, pitch = 30, 22, 6, 0.8, 1.0
    rng = np.random.default_rng(77)
    m = W.random_unit(rng, (nz, ny, nx))[None]
    p3, zb = _plan(nx, ny, nz, t, pitch, False, 1)
    p2 = hfd.Plan(nx, ny, DX, DY, np.full(nz, t), zb, batch_max=1, flags=hfd.HFD_FP32)
    h3, mused = run_field(p3, m)
    h2, _ = run_field(p2, m)
    ref = oracle.field(nx, ny, DX, DY, zb, np.full(nz, t), mused[0])
    assert rel_err(h3[0], ref) < 1e-5 and rel_err(h2[0], ref) < 1e-5
    assert rel_err(h3[0], h2[0]) < 2e-6
    p3.destroy()
    p2.destroy()


def test_equidistant_adjoint_and_unsupported_thickness_gradient():
    import torch
    nx, ny, nz, t, pitch = 14, 10, 4, 0.7, 0.9
    rng = np.random.default_rng(78)
    g = rng.standard_normal((1, 3, nz, ny, nx))
    plan, zb = _plan(nx, ny, nz, t, pitch, True, 1)
    gm, _ = plan.vjp(None, torch.from_numpy(g).cuda(), want_m=True, want_t=False)
    ref = oracle.field(nx, ny, DX, DY, zb, np.full(nz, t), g[0], transpose=True)
    assert rel_err(gm.cpu().numpy()[0], ref) < 1e-10
    with pytest.raises(hfd.HFDError) as ei:
        plan.vjp(torch.from_numpy(g).cuda(), torch.from_numpy(g).cuda(), want_m=False, want_t=True)
    assert ei.value.status == hfd.HFD_ENOTSUP
    plan.destroy()
