"""Layer-thickness optimization by Newton iteration (Sec. 4 of the paper).

One layer thickness t_k of a stack is varied until a scalar field objective
L(t) vanishes; here L is the mean of h_z over a target layer (the free layer),
the quantity the paper drives to zero for an MRAM cell.  Each step evaluates
the field and its thickness derivative with the library (hfd_demag_field and
hfd_demag_vjp); the gaps between layers stay fixed, so thickening layer k lifts
every layer above it.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import hfd


@dataclass
class NewtonResult:
    thickness: float
    objective: float
    iterations: int
    history: list = field(default_factory=list)   # (t_k, L, dL/dt_k) per step


def mean_hz_objective(plan: "hfd.Plan", m, target_layer: int):
    """L = mean over the target layer of h_z and dL/dt (all layers), FP64."""
    import torch
    h = plan.field(m)
    gh = torch.zeros_like(m)
    gh[:, 2, target_layer] = 1.0 / (plan.nx * plan.ny)
    _, gt = plan.vjp(m, gh, want_m=False, want_t=True)
    L = float(h[0, 2, target_layer].double().mean().item())
    return L, gt[0].cpu().numpy()


def optimize_thickness(plan: "hfd.Plan", m, layer: int, target_layer: int, tol: float = 1e-5,
                       max_iter: int = 20, t_min: float = 1e-3) -> NewtonResult:
    """Newton iteration t_k <- t_k - L / (dL/dt_k) on a one-stack plan until
    |L| < tol.  ``m`` is the device magnetization [1, 3, nz, ny, nx]."""
    if plan.n_geom != 1:
        raise ValueError("Newton optimization runs on a single stack")
    t = plan.thickness[0].copy()
    z = plan.z_bottom[0].copy() if plan.z_bottom is not None else np.concatenate(
        [[0.0], np.cumsum(t[:-1])])
    gaps = z[1:] - (z[:-1] + t[:-1])
    hist = []
    L, g = mean_hz_objective(plan, m, target_layer)
    it = 0
    while abs(L) >= tol and it < max_iter:
        dL = g[layer]
        if dL == 0.0:
            raise RuntimeError("zero derivative; Newton step undefined")
        hist.append((t[layer], L, dL))
        t[layer] = max(t[layer] - L / dL, t_min)
        z = np.concatenate([[z[0]], z[0] + np.cumsum(t[:-1] + gaps)])
        plan.set_thickness(t, z)
        L, g = mean_hz_objective(plan, m, target_layer)
        it += 1
    hist.append((t[layer], L, g[layer]))
    return NewtonResult(thickness=float(t[layer]), objective=L, iterations=it, history=hist)
