"""Oracle for the micromagnetic energy of the hysteresis simulation (Sec. 4).

TEST INFRASTRUCTURE ONLY (see the package docstring): plain CPU code, FP64,
sharing nothing with the HIP library.

The paper names the energy terms of the free-layer simulation (exchange,
uniaxial anisotropy along +z, applied field, demagnetization; the two SAFM
layers pinned) and the CoFe constants, and relaxes the magnetization with an
L-BFGS energy minimization at every field step.  It gives no discretization;
the reading here is the usual finite-difference micromagnetic energy of one
layer of cells, in units of mu0 Ms^2 V_cell, term by term:

    e_ex   = sum over neighbour pairs (c, n) inside the mask of cex (1 - m_c . m_n)
             cex = 2 A / (mu0 Ms^2 d^2) along the pair's axis (free surfaces:
             no coupling across the mask edge)
    e_an   = - hk/2 sum_c m_z(c)^2,             hk = 2 K_u / (mu0 Ms^2)
    e_ext  = - sum_c m_c . h_ext
    e_bias = - sum_c m_c . h_bias(c)            (fixed sources: pinned layers)
    e_d    = - 1/2 sum_c m_c . h_d(c),          h_d = - N * m (brute-force sum)

and the effective field h_eff = - d e / d m (per cell, units of Ms).  The
minimizer's variables are unnormalized vectors u with m = u / |u|.
"""
from __future__ import annotations

import math

import numpy as np

from . import field as _demag_field
from . import tensor_cuboids as _tensor_cuboids

MU0 = 4e-7 * math.pi
NEIGHBOURS = ((0, -1, "x"), (0, 1, "x"), (-1, 0, "y"), (1, 0, "y"))


def normalize(u, mask):
    """m = u / |u| on the mask, 0 elsewhere."""
    r = np.sqrt((u * u).sum(0))
    m = np.zeros_like(u)
    for y in range(mask.shape[0]):
        for x in range(mask.shape[1]):
            if mask[y, x]:
                m[:, y, x] = u[:, y, x] / r[y, x]
    return m


def exchange_energy(m, mask, cex_x, cex_y):
    """Sum over unordered neighbour pairs inside the mask of cex (1 - m_c . m_n)."""
    ny, nx = mask.shape
    e = 0.0
    for y in range(ny):
        for x in range(nx):
            if not mask[y, x]:
                continue
            if x + 1 < nx and mask[y, x + 1]:
                e += cex_x * (1.0 - m[:, y, x] @ m[:, y, x + 1])
            if y + 1 < ny and mask[y + 1, x]:
                e += cex_y * (1.0 - m[:, y, x] @ m[:, y + 1, x])
    return e


def exchange_field(m, mask, cex_x, cex_y):
    """- d e_ex / d m: sum over the neighbours inside the mask of cex m_n (the
    pair energy cex (1 - m_c . m_n)); written here as cex (m_n - m_c), which
    differs only along m_c (no torque, no change of the tangential gradient)
    and is the form the effective field conventionally takes."""
    ny, nx = mask.shape
    h = np.zeros_like(m)
    for y in range(ny):
        for x in range(nx):
            if not mask[y, x]:
                continue
            for dy, dx, ax in NEIGHBOURS:
                yy, xx = y + dy, x + dx
                if 0 <= yy < ny and 0 <= xx < nx and mask[yy, xx]:
                    c = cex_x if ax == "x" else cex_y
                    h[:, y, x] += c * (m[:, yy, xx] - m[:, y, x])
    return h


def demag_field(m, mask, dx, dy, t):
    """Self field of the layer, brute-force sum over all cell pairs (the
    oracle's field of Sec. 3 with one layer)."""
    ny, nx = mask.shape
    mm = (m * mask[None]).reshape(3, 1, ny, nx)
    return _demag_field(nx, ny, dx, dy, np.array([0.0]), np.array([float(t)]), mm)[:, 0]


def energy_terms(u, mask, dx, dy, t, cex_x, cex_y, hk, h_ext, h_bias):
    """Dict of the reduced energy terms, the total, h_eff and the gradient
    with respect to u, for u [3][ny][nx]."""
    m = normalize(u, mask)
    hd = demag_field(m, mask, dx, dy, t)
    hex_ = exchange_field(m, mask, cex_x, cex_y)
    han = np.zeros_like(m)
    han[2] = hk * m[2]
    hext = np.asarray(h_ext, dtype=np.float64)[:, None, None] * np.ones_like(m)
    mk = mask[None].astype(np.float64)
    terms = {
        "exchange": exchange_energy(m, mask, cex_x, cex_y),
        "anisotropy": float(-0.5 * hk * (m[2] ** 2 * mask).sum()),
        "external": float(-(m * hext * mk).sum()),
        "bias": float(-(m * h_bias * mk).sum()),
        "demag": float(-0.5 * (m * hd * mk).sum()),
    }
    terms["total"] = sum(terms.values())
    heff = (hex_ + han + hd + hext + h_bias) * mk
    mh = (m * heff).sum(0)
    r = np.sqrt((u * u).sum(0))
    grad = np.zeros_like(u)
    for y in range(mask.shape[0]):
        for x in range(mask.shape[1]):
            if mask[y, x]:
                grad[:, y, x] = -(heff[:, y, x] - mh[y, x] * m[:, y, x]) / r[y, x]
    terms["h_eff"] = heff
    terms["grad"] = grad
    terms["m"] = m
    return terms


# e depends on u only through u / |u|, so the minimizer may start from a
# scaled copy: L-BFGS-B's first step has unit length in its variables, which
# on unit vectors is a rotation of tens of degrees and can carry a metastable
# state over a small barrier; started from SCALE * m it rotates by 1 / SCALE
# at most (the gradient scales by 1 / SCALE, the tolerance with it)
SCALE = 1.0e3


def relax(u0, mask, dx, dy, t, cex_x, cex_y, hk, h_ext, h_bias, gtol=1e-6):
    """L-BFGS (scipy's L-BFGS-B as the library step) on e(u) from u0 (the
    previous state); returns the normalized state.  gtol bounds the largest
    component of d e / d u at |u| = 1."""
    from scipy.optimize import minimize
    shape = u0.shape

    def fun(x):
        tm = energy_terms(x.reshape(shape), mask, dx, dy, t, cex_x, cex_y, hk, h_ext, h_bias)
        return tm["total"], tm["grad"].ravel()

    x0 = SCALE * normalize(u0, mask)
    res = minimize(fun, x0.ravel(), jac=True, method="L-BFGS-B",
                   options={"maxiter": 20000, "maxfun": 80000, "gtol": gtol / SCALE,
                            "ftol": 1e-15})
    return normalize(res.x.reshape(shape), mask)


def hysteresis(mask, dx, dy, t, cex_x, cex_y, hk, Js, h_bias, b_max, steps, direction=(0, 0, 1),
               gtol=1e-6):
    """Loop +b_max -> -b_max -> +b_max (tesla) in `steps` equal field steps
    along `direction`, from m = +z; returns (b, mean m_z over the mask)."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    half = steps // 2
    bs = np.concatenate([np.linspace(b_max, -b_max, half + 1),
                         np.linspace(-b_max, b_max, steps - half + 1)[1:]])
    u = np.zeros((3,) + mask.shape)
    u[2][mask] = 1.0
    mz = []
    for b in bs:
        u = relax(u, mask, dx, dy, t, cex_x, cex_y, hk, (b / Js) * d, h_bias, gtol)
        mz.append(float(u[2][mask].mean()))
    return bs, np.array(mz)


def sign_changes(b, mz):
    """Fields where the mean m_z changes sign on the descending and the
    ascending branch (linear interpolation), None where it does not."""
    k = int(np.argmin(b))
    out = []
    for lo, hi in ((0, k + 1), (k, len(b))):
        bb, mm = b[lo:hi], mz[lo:hi]
        idx = [i for i in range(len(mm) - 1) if np.sign(mm[i]) != np.sign(mm[i + 1])]
        if not idx:
            out.append(None)
            continue
        i = idx[0]
        out.append(float(bb[i] + (bb[i + 1] - bb[i]) * mm[i] / (mm[i] - mm[i + 1])))
    return tuple(out)


def stoner_wohlfarth_switching(hk_eff, psi):
    """Switching field (in units of the anisotropy field's unit) of a single
    domain particle with uniaxial effective anisotropy hk_eff when the field
    makes the angle psi with the easy axis (Stoner and Wohlfarth, 1948):
    hk_eff / (cos^(2/3) psi + sin^(2/3) psi)^(3/2)."""
    c, s = abs(math.cos(psi)), abs(math.sin(psi))
    return hk_eff / (c ** (2.0 / 3.0) + s ** (2.0 / 3.0)) ** 1.5


def cell_shape_anisotropy(d, t):
    """N_zz - N_xx of a single d x d x t cuboid (its self tensor)."""
    n = _tensor_cuboids(0.0, 0.0, 0.0, (d, d, t), (d, d, t))
    return float(n[2] - n[0])
