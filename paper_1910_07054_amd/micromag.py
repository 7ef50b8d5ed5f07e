"""Hysteresis of the MRAM free layer (Sec. 4 of the paper).

After the SAFM thickness has been optimised, the paper pins the magnetization
of the two SAFM layers, applies a field along z to the 3 nm free layer
(CoFe: J_s = 1.75 T, A_ex = 1.5e-11 J/m, K_u = 2.09e6 J/m^3 along +z) and
relaxes the free-layer magnetization with L-BFGS energy minimization at each
of 2000 field steps; the loop switches at 1.51 T.

Here the energy and its gradient come from the library (include/hfd_mm.h:
exchange, anisotropy, applied field and the fixed stray field of the pinned
layers in HIP kernels, the free layer's own demagnetizing field through
hfd_demag_field on an FP64 one-layer plan); the stray field of the pinned
layers is one hfd_demag_field evaluation of the whole stack with the free
layer empty.  L-BFGS (scipy's L-BFGS-B, unconstrained) runs on the host over
the unnormalized vectors u, m = u / |u|.

Readings where the paper is silent (listed in the design doc): finite-difference
exchange with free surfaces at the disk edge, one cell through the free-layer
thickness, the pinned layers of the same J_s, an L-BFGS tolerance of 1e-6 on
the largest torque component, the loop +B_max -> -B_max -> +B_max in 2000
equal steps with B_max = 2.5 T, the switching field where the mean m_z of the
free layer changes sign (linear interpolation between steps), and the field
tilted by FIELD_TILT = 1e-4 rad from z: with the field exactly along the easy
axis the symmetric state remains a stationary point (a saddle) past the
instability and a minimizer does not leave it; at this tilt the
Stoner-Wohlfarth switching field of a macrospin is lowered by 0.3 %.
"""
from __future__ import annotations

import ctypes
import math
import sys
import time
from dataclasses import dataclass, field

import numpy as np

from . import hfd
from . import workloads as W

MU0 = 4e-7 * math.pi
FIELD_TILT = 1.0e-4      # rad from z, in the xz plane (see the module docstring)


@dataclass
class Material:
    """CoFe constants of Sec. 4."""
    Js: float = 1.75        # mu0 Ms, T
    A: float = 1.5e-11      # J/m
    Ku: float = 2.09e6      # J/m^3, easy axis +z

    def lex2(self) -> float:
        """2 A / (mu0 Ms^2) in m^2."""
        return 2.0 * self.A * MU0 / self.Js ** 2

    def hk(self) -> float:
        """Anisotropy field over Ms, 2 K_u / (mu0 Ms^2)."""
        return 2.0 * self.Ku * MU0 / self.Js ** 2


class Energy:
    """hfd_mm object: reduced energy e = E / (mu0 Ms^2 V_cell) and d e / d u of
    one layer on the grid of an FP64 one-layer plan."""

    def __init__(self, plan: "hfd.Plan", mask: np.ndarray, cex_x: float, cex_y: float, hk: float):
        import torch
        self.plan = plan
        self.ny, self.nx = mask.shape
        mk = np.ascontiguousarray(mask.astype(np.uint8))
        h = ctypes.c_void_p()
        hfd._check(hfd.load().hfd_mm_create(ctypes.byref(h), plan.handle, mk.ctypes.data,
                                            float(cex_x), float(cex_y), float(hk),
                                            hfd._stream_handle(None)))
        self.handle = h
        dev = torch.device("cuda")
        self._u = torch.zeros((3, self.ny, self.nx), dtype=torch.float64, device=dev)
        self._g = torch.zeros_like(self._u)
        self._m = torch.zeros_like(self._u)
        self.evaluations = 0

    def set_bias(self, h_bias):
        """Field of the fixed sources, torch [3, ny, nx] float64 on the GPU."""
        hb = h_bias.contiguous()
        hfd._check(hfd.load().hfd_mm_set_bias(self.handle, hfd._dptr(hb), hfd._stream_handle(None)))

    def __call__(self, u: np.ndarray, h_ext) -> tuple[float, np.ndarray]:
        """(e, de/du) for u [3, ny, nx] (host float64) and h_ext (3,) / Ms."""
        import torch
        self._u.copy_(torch.from_numpy(np.ascontiguousarray(u).reshape(3, self.ny, self.nx)))
        he = np.ascontiguousarray(np.asarray(h_ext, dtype=np.float64))
        e = ctypes.c_double()
        hfd._check(hfd.load().hfd_mm_energy_grad(self.handle, hfd._dptr(self._u), he.ctypes.data,
                                                 hfd._dptr(self._g), None, hfd._dptr(self._m),
                                                 ctypes.byref(e), hfd._stream_handle(None)))
        self.evaluations += 1
        return e.value, self._g.cpu().numpy()

    def effective_field(self, u: np.ndarray, h_ext):
        """(e, grad, h_eff, m) as host arrays, for checks."""
        import torch
        self._u.copy_(torch.from_numpy(np.ascontiguousarray(u).reshape(3, self.ny, self.nx)))
        he = np.ascontiguousarray(np.asarray(h_ext, dtype=np.float64))
        heff = torch.zeros_like(self._u)
        e = ctypes.c_double()
        hfd._check(hfd.load().hfd_mm_energy_grad(self.handle, hfd._dptr(self._u), he.ctypes.data,
                                                 hfd._dptr(self._g), hfd._dptr(heff),
                                                 hfd._dptr(self._m), ctypes.byref(e),
                                                 hfd._stream_handle(None)))
        return e.value, self._g.cpu().numpy(), heff.cpu().numpy(), self._m.cpu().numpy()

    def destroy(self):
        if self.handle:
            hfd._check(hfd.load().hfd_mm_destroy(self.handle))
            self.handle = None


# The energy depends on u only through m = u / |u|.  L-BFGS-B's first step
# has unit length in its variables; on unit vectors that is a rotation large
# enough to carry a metastable state over the small barrier left just before
# switching.  Each relaxation therefore starts from START_SCALE * m, so the
# first step rotates by at most 1 / START_SCALE (the gradient and the
# tolerance scale by 1 / START_SCALE).
START_SCALE = 1.0e3


def relax(energy: Energy, u0: np.ndarray, h_ext, gtol: float = 1e-6, max_iter: int = 20000):
    """L-BFGS minimization of e(u) from the state u0; returns (u normalized on
    the mask, e, iterations, evaluations).  gtol bounds the largest component
    of d e / d u at |u| = 1 (the torque per cell)."""
    from scipy.optimize import minimize
    shape = u0.shape
    before = energy.evaluations
    r0 = np.sqrt((u0 * u0).sum(0))
    x0 = START_SCALE * np.where(r0 > 0, u0 / np.where(r0 > 0, r0, 1.0), 0.0)
    res = minimize(lambda x: energy(x.reshape(shape), h_ext), x0.ravel(), jac=True,
                   method="L-BFGS-B",
                   options={"maxiter": max_iter, "maxfun": 4 * max_iter, "gtol": gtol / START_SCALE,
                            "ftol": 1e-15, "maxcor": 10})
    u = res.x.reshape(shape)
    r = np.sqrt((u * u).sum(0))
    u = np.where(r > 0, u / np.where(r > 0, r, 1.0), 0.0)
    return u, float(res.fun), int(res.nit), energy.evaluations - before


@dataclass
class LayerProblem:
    """One magnetic layer of thickness t on an n x n grid, cells of d x d,
    disk mask, material, bias field of fixed sources (units of Ms)."""
    n: int
    d_nm: float
    t_nm: float
    mask: np.ndarray
    material: Material
    h_bias: np.ndarray
    plan: "hfd.Plan" = None
    energy: Energy = None
    info: dict = field(default_factory=dict)

    def build(self):
        import torch
        mat = self.material
        self.plan = hfd.Plan(self.n, self.n, self.d_nm, self.d_nm, [self.t_nm], None, batch_max=1,
                             flags=hfd.HFD_FP64)
        cex = mat.lex2() / (self.d_nm * 1e-9) ** 2
        self.energy = Energy(self.plan, self.mask, cex, cex, mat.hk())
        self.energy.set_bias(torch.from_numpy(np.ascontiguousarray(self.h_bias)).cuda())
        return self

    def destroy(self):
        if self.energy is not None:
            self.energy.destroy()
        if self.plan is not None:
            self.plan.destroy()

    def mean_mz(self, u: np.ndarray) -> float:
        return float(u[2][self.mask].mean())


def mram_free_layer(t_mid: float, n: int = 64, material: Material | None = None) -> LayerProblem:
    """Free layer of the Sec. 4 MRAM disk on n x n cells, with the stray field
    of the two pinned SAFM layers (5 nm +z, t_mid nm -z, spacers 1 nm) at the
    free layer computed by the library on the whole stack."""
    import torch
    wl = W.mram_disk(t_mid, n)
    mask = wl.notes["disk"]
    stack = hfd.Plan(wl.nx, wl.ny, wl.dx, wl.dy, wl.thickness, wl.z_bottom, batch_max=1,
                     flags=hfd.HFD_FP64)
    h = stack.field(torch.from_numpy(wl.m).cuda())
    torch.cuda.synchronize()
    hb = h[0, :, wl.notes["free_layer"]].cpu().numpy().copy()
    stack.destroy()
    return LayerProblem(n, wl.dx, float(wl.thickness[0][wl.notes["free_layer"]]), mask,
                        material or Material(), hb).build()


def sweep(prob: LayerProblem, b_max: float = 2.5, steps: int = 2000, gtol: float = 1e-6,
          direction=(0.0, 0.0, 1.0), progress=None):
    """Hysteresis loop +b_max -> -b_max -> +b_max in `steps` equal steps of the
    applied field (tesla) along `direction`, starting from m = +z; each step
    relaxes from the previous state.  Returns dict of arrays (b, mean m_z,
    iterations, evaluations) and the wall time."""
    Js = prob.material.Js
    dirv = np.asarray(direction, dtype=np.float64)
    dirv = dirv / np.linalg.norm(dirv)
    half = steps // 2
    down = np.linspace(b_max, -b_max, half + 1)
    up = np.linspace(-b_max, b_max, steps - half + 1)[1:]
    bs = np.concatenate([down, up])
    u = np.zeros((3, prob.n, prob.n))
    u[2][prob.mask] = 1.0
    out = {"b": [], "mz": [], "iterations": [], "evaluations": []}
    t0 = time.perf_counter()
    for k, b in enumerate(bs):
        u, _, nit, nev = relax(prob.energy, u, (b / Js) * dirv, gtol=gtol)
        out["b"].append(float(b))
        out["mz"].append(prob.mean_mz(u))
        out["iterations"].append(nit)
        out["evaluations"].append(nev)
        if progress and (k % progress == 0):
            print(f"  step {k}/{len(bs)} B = {b:+.4f} T  <m_z> = {out['mz'][-1]:+.5f}  "
                  f"({nit} iterations)", file=sys.stderr, flush=True)
    out = {k: np.array(v) for k, v in out.items()}
    out["seconds"] = time.perf_counter() - t0
    out["final_u"] = u
    return out


def switching_fields(b: np.ndarray, mz: np.ndarray):
    """Fields (T) where the mean m_z changes sign on the descending and on the
    ascending branch (linear interpolation between steps); None if absent."""
    k_min = int(np.argmin(b))
    res = []
    for lo, hi in ((0, k_min + 1), (k_min, len(b))):
        bb, mm = b[lo:hi], mz[lo:hi]
        s = np.nonzero(np.sign(mm[1:]) != np.sign(mm[:-1]))[0]
        if len(s) == 0:
            res.append(None)
            continue
        i = s[0]
        res.append(float(bb[i] + (bb[i + 1] - bb[i]) * mm[i] / (mm[i] - mm[i + 1])))
    return tuple(res)


def effective_anisotropy(prob: LayerProblem):
    """Macrospin estimate of the loop: the demagnetizing factors of the
    discretized layer (mean self field of the uniform +z and +x states over
    the mask, from the library) and hk_eff = hk - (N_zz - N_xx), with the
    mean bias field; the Stoner-Wohlfarth switching field is Js hk_eff at
    zero tilt."""
    import torch
    mk = torch.from_numpy(prob.mask).cuda()

    def mean_self_field(k):
        m = torch.zeros((1, 3, 1, prob.n, prob.n), dtype=torch.float64, device="cuda")
        m[0, k, 0][mk] = 1.0
        h = prob.plan.field(m)[0, :, 0]
        return [float(h[c][mk].mean()) for c in range(3)]

    nzz = -mean_self_field(2)[2]
    nxx = -mean_self_field(0)[0]
    hk_eff = prob.material.hk() - (nzz - nxx)
    return {"Nzz": nzz, "Nxx": nxx, "hk_eff": hk_eff, "B_K_eff_T": prob.material.Js * hk_eff,
            "mean_bias_T": [prob.material.Js * float(prob.h_bias[c][prob.mask].mean()) for c in range(3)]}


def mram_hysteresis(steps: int = 2000, b_max: float = 2.5, n: int = 64, t_mid: float = 3.4389,
                    tilt: float = FIELD_TILT, progress=None):
    """The Sec. 4 loop: free layer of the optimised MRAM disk (SAFM middle
    layer t_mid nm), `steps` field steps, field tilted by `tilt` rad.  Returns
    the sweep record with the switching fields, H_sw (mean magnitude of the two
    branches) and the macrospin estimate."""
    prob = mram_free_layer(t_mid, n=n)
    try:
        est = effective_anisotropy(prob)
        res = sweep(prob, b_max=b_max, steps=steps, direction=(math.sin(tilt), 0.0, math.cos(tilt)),
                    progress=progress)
    finally:
        prob.destroy()
    down, up = switching_fields(res["b"], res["mz"])
    res["switching_T"] = (down, up)
    res["H_sw_T"] = None if down is None or up is None else 0.5 * (abs(down) + abs(up))
    res["estimate"] = est
    return res
