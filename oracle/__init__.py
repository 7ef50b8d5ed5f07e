"""Reference oracle for the hybrid-FFT demagnetization field (arXiv:1910.07054).

TEST INFRASTRUCTURE ONLY.  Plain, slow CPU code that states what the GPU
library must compute.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product path never does, and
nothing here is shared with the HIP library.

Parts:
  * ``newell_oracle.c`` (loaded through ctypes): the Newell kernels f and g in
    extended precision, the generalized tensor of a cuboid pair (Sec. 2 and
    appendices A/B), layer-pair tables on the lateral lattice (entries beyond
    50 cell sizes by quadrature of the dipole kernel, where the closed form
    has lost its digits), the brute-force field over all cell pairs (Sec. 3),
    its transpose, and the thickness gradient.
  * ``fft_field``: the hybrid algorithm of Sec. 3.1 (2D discrete Fourier
    transform in x and y, explicit sum over layers in z), written with
    numpy's FFT as the library step, in FP64.
  * ``fft3_field`` / ``fourier_tensor3``: the equidistant case of Sec. 3.1
    (eq. FFT_3D, three-dimensional transform), same library step.
  * ``quad_tensor``: Gauss-Legendre quadrature of the cell-averaged dipole
    kernel, an independent route to the tensor of two disjoint cuboids.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "newell_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")
_SYM = np.array([[0, 3, 4], [3, 1, 5], [4, 5, 2]])


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    d, i, p = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
    for name in ("hfdo_f", "hfdo_g"):
        getattr(lib, name).restype = d
        getattr(lib, name).argtypes = [d, d, d]
    for name in ("hfdo_df", "hfdo_dg", "hfdo_phi"):
        getattr(lib, name).restype = d
        getattr(lib, name).argtypes = [i, d, d, d]
    lib.hfdo_tensor_cuboids.restype = None
    lib.hfdo_tensor_cuboids.argtypes = [d] * 9 + [p]
    lib.hfdo_dtensor_dZ_cuboids.restype = None
    lib.hfdo_dtensor_dZ_cuboids.argtypes = [d] * 9 + [p]
    lib.hfdo_tensor_far.restype = None
    lib.hfdo_tensor_far.argtypes = [d] * 9 + [p]
    lib.hfdo_pair_table.restype = i
    lib.hfdo_pair_table.argtypes = [i, i, d, d, d, d, d, d, p]
    lib.hfdo_pair_dtable.restype = i
    lib.hfdo_pair_dtable.argtypes = [i, i, d, d, d, d, d, d, p]
    lib.hfdo_field.restype = i
    lib.hfdo_field.argtypes = [i, i, i, d, d, p, p, p, i, p, p, i]
    lib.hfdo_thickness_grad.restype = i
    lib.hfdo_thickness_grad.argtypes = [i, i, i, d, d, p, p, p, p, i, p, p]
    lib.hfdo_num_threads.restype = i
    lib.hfdo_num_threads.argtypes = []
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().hfdo_num_threads())


# --------------------------------------------------------------------------
# Kernels and tensors
# --------------------------------------------------------------------------
def f(x, y, z) -> float:
    """Newell's f (Sec. 2.1), extended precision, returned as float64."""
    return _load().hfdo_f(float(x), float(y), float(z))


def g(x, y, z) -> float:
    """Newell's g (Sec. 2.2), extended precision, returned as float64."""
    return _load().hfdo_g(float(x), float(y), float(z))


def df(arg: int, x, y, z) -> float:
    return _load().hfdo_df(int(arg), float(x), float(y), float(z))


def dg(arg: int, x, y, z) -> float:
    return _load().hfdo_dg(int(arg), float(x), float(y), float(z))


def tensor_cuboids(X, Y, Z, target, source) -> np.ndarray:
    """Six components (xx, yy, zz, xy, xz, yz) of N for a target cuboid of
    dimensions ``target`` whose origin is offset by (X, Y, Z) from a source
    cuboid of dimensions ``source`` (Sec. 2, direct 64-term form)."""
    out = np.zeros(6)
    _load().hfdo_tensor_cuboids(float(X), float(Y), float(Z), *map(float, target),
                                *map(float, source), _ptr(out))
    return out


def tensor_far(X, Y, Z, target, source) -> np.ndarray:
    """The far-field rule the pair tables use beyond 50 cell sizes: the
    cell-averaged dipole kernel integrated over both cuboids with 3
    Gauss-Legendre points per axis, extended precision (same conventions as
    tensor_cuboids)."""
    out = np.zeros(6)
    _load().hfdo_tensor_far(float(X), float(Y), float(Z), *map(float, target), *map(float, source),
                            _ptr(out))
    return out


def dtensor_dZ_cuboids(X, Y, Z, target, source) -> np.ndarray:
    out = np.zeros(6)
    _load().hfdo_dtensor_dZ_cuboids(float(X), float(Y), float(Z), *map(float, target),
                                    *map(float, source), _ptr(out))
    return out


def full3x3(t6: np.ndarray) -> np.ndarray:
    """Expand the six stored components (last axis) into the symmetric 3x3."""
    return np.asarray(t6)[..., _SYM]


def pair_table(nx, ny, dx, dy, tbot, ttop, sbot, stop) -> np.ndarray:
    """N^{ij}(p, q) for p in [-(nx-1), nx-1], q in [-(ny-1), ny-1]:
    array [6][2ny-1][2nx-1], offset (p, q) at [:, q+ny-1, p+nx-1]."""
    out = np.zeros((6, 2 * ny - 1, 2 * nx - 1))
    rc = _load().hfdo_pair_table(int(nx), int(ny), float(dx), float(dy), float(tbot), float(ttop),
                                 float(sbot), float(stop), _ptr(out))
    if rc:
        raise ValueError(f"hfdo_pair_table failed ({rc})")
    return out


def pair_dtable(nx, ny, dx, dy, tbot, ttop, sbot, stop) -> np.ndarray:
    """Derivatives of the pair table with respect to (target top, target
    bottom, source top, source bottom): array [4][6][2ny-1][2nx-1]."""
    out = np.zeros((4, 6, 2 * ny - 1, 2 * nx - 1))
    rc = _load().hfdo_pair_dtable(int(nx), int(ny), float(dx), float(dy), float(tbot), float(ttop),
                                  float(sbot), float(stop), _ptr(out))
    if rc:
        raise ValueError(f"hfdo_pair_dtable failed ({rc})")
    return out


# --------------------------------------------------------------------------
# Field by direct summation over all cell pairs
# --------------------------------------------------------------------------
def _geom(nx, ny, zbot, thick):
    zb = np.ascontiguousarray(zbot, dtype=np.float64)
    tk = np.ascontiguousarray(thick, dtype=np.float64)
    return zb, tk


def field(nx, ny, dx, dy, zbot, thick, m, samples=None, transpose=False) -> np.ndarray:
    """Brute-force field h = -sum_j N^{ij} * m_j (Sec. 3), FP64.

    m: [3][nz][ny][nx].  samples: optional int array [S][3] of (layer, iy, ix);
    returns [S][3] for samples, else [3][nz][ny][nx].  ``transpose`` applies
    the transposed operator (gradient with respect to m of <g, h>)."""
    zb, tk = _geom(nx, ny, zbot, thick)
    nz = zb.shape[0]
    mm = np.ascontiguousarray(m, dtype=np.float64).reshape(3, nz, ny, nx)
    if samples is None:
        out = np.zeros((3, nz, ny, nx))
        ns, sp = 0, None
    else:
        s = np.ascontiguousarray(samples, dtype=np.int32).reshape(-1, 3)
        out = np.zeros((s.shape[0], 3))
        ns, sp = s.shape[0], _ptr(s)
    rc = _load().hfdo_field(int(nx), int(ny), int(nz), float(dx), float(dy), _ptr(zb), _ptr(tk),
                            _ptr(mm), ns, sp, _ptr(out), int(bool(transpose)))
    if rc:
        raise ValueError(f"hfdo_field failed ({rc})")
    return out


def thickness_grad(nx, ny, dx, dy, zbot, thick, m, g, uniform=False, with_interfaces=False):
    """Gradient of L = <g, h(m)> with respect to the layer thicknesses, for a
    stack whose gaps stay fixed (raising t_k lifts every layer above k).

    ``g`` is a full field [3][nz][ny][nx], or with ``uniform=True`` one vector
    per layer [nz][3] (the same upstream gradient in every cell of a layer)."""
    zb, tk = _geom(nx, ny, zbot, thick)
    nz = zb.shape[0]
    mm = np.ascontiguousarray(m, dtype=np.float64).reshape(3, nz, ny, nx)
    if uniform:
        gg = np.ascontiguousarray(g, dtype=np.float64).reshape(nz, 3)
    else:
        gg = np.ascontiguousarray(g, dtype=np.float64).reshape(3, nz, ny, nx)
    gt = np.zeros(nz)
    gi = np.zeros(2 * nz)
    rc = _load().hfdo_thickness_grad(int(nx), int(ny), int(nz), float(dx), float(dy), _ptr(zb),
                                     _ptr(tk), _ptr(mm), _ptr(gg), int(bool(uniform)), _ptr(gt),
                                     _ptr(gi))
    if rc:
        raise ValueError(f"hfdo_thickness_grad failed ({rc})")
    return (gt, gi.reshape(nz, 2)) if with_interfaces else gt


# --------------------------------------------------------------------------
# Hybrid FFT (Sec. 3.1): 2D transform along x and y, explicit sum along z
# --------------------------------------------------------------------------
def fourier_tensor(nx, ny, dx, dy, zbot, thick, Lx=None, Ly=None):
    """2D DFT (numpy) of every layer-pair table placed on an Lx x Ly periodic
    grid (zero padding; Lx >= 2nx-1): complex array [nz][nz][6][Ly][Lx]."""
    zb, tk = _geom(nx, ny, zbot, thick)
    nz = zb.shape[0]
    Lx = Lx or 2 * nx
    Ly = Ly or 2 * ny
    if Lx < 2 * nx - 1 or Ly < 2 * ny - 1:
        raise ValueError("padded length too short for an aperiodic convolution")
    out = np.zeros((nz, nz, 6, Ly, Lx), dtype=np.complex128)
    py = np.arange(-(ny - 1), ny) % Ly
    px = np.arange(-(nx - 1), nx) % Lx
    for i in range(nz):
        for j in range(nz):
            tab = pair_table(nx, ny, dx, dy, zb[i], zb[i] + tk[i], zb[j], zb[j] + tk[j])
            grid = np.zeros((6, Ly, Lx))
            grid[:, py[:, None], px[None, :]] = tab
            out[i, j] = np.fft.fft2(grid)
    return out


def fft_field(nx, ny, dx, dy, zbot, thick, m, Ntil=None, transpose=False) -> np.ndarray:
    """h_k,i = -sum_l F2^-1 F1^-1 sum_j [F1F2(N_kl)_{ij} F1F2(m_l)_j]   (FP64).

    m: [3][nz][ny][nx] (or [B][3][nz][ny][nx]); returns the same shape."""
    zb, tk = _geom(nx, ny, zbot, thick)
    nz = zb.shape[0]
    if Ntil is None:
        Ntil = fourier_tensor(nx, ny, dx, dy, zb, tk)
    Ly, Lx = Ntil.shape[-2:]
    mm = np.asarray(m, dtype=np.float64)
    batched = mm.ndim == 5
    if not batched:
        mm = mm[None]
    out = np.empty_like(mm)
    N33 = full3x3(np.moveaxis(Ntil, 2, -1))          # [i][j][Ly][Lx][3][3]
    for b in range(mm.shape[0]):
        mh = np.fft.fft2(mm[b], s=(Ly, Lx))           # [3][nz][Ly][Lx]
        hh = np.zeros_like(mh)
        for i in range(nz):
            for j in range(nz):
                if transpose:
                    # (A^T g)_j = -sum_i N^{ij}(p - q) g_i(p): correlation, conj spectrum
                    T = np.conj(N33[i, j])
                    hh[:, j] -= np.einsum("yxkl,kyx->lyx", T, mh[:, i])
                else:
                    hh[:, i] -= np.einsum("yxkl,lyx->kyx", N33[i, j], mh[:, j])
        out[b] = np.real(np.fft.ifft2(hh))[:, :, :ny, :nx]
    return out if batched else out[0]


# --------------------------------------------------------------------------
# Equidistant case (eq. FFT_3D of Sec. 3.1): transform along z as well
# --------------------------------------------------------------------------
def _pow2_at_least(n: int) -> int:
    L = 1
    while L < n:
        L *= 2
    return L


def fourier_tensor3(nx, ny, dx, dy, nz, thick, pitch, Lx=None, Ly=None, Lz=None):
    """3-D DFT (numpy) of the tensor of equal cells of thickness `thick` on a
    regular z grid of `pitch`: the layer-offset tables N(p, q, d), d in
    [-(nz-1), nz-1] (target minus source, Z = d * pitch), placed on an
    Lx x Ly x Lz periodic grid; complex array [6][Lz][Ly][Lx]."""
    Lx = Lx or 2 * nx
    Ly = Ly or 2 * ny
    Lz = Lz or max(2, _pow2_at_least(2 * nz))
    if Lx < 2 * nx - 1 or Ly < 2 * ny - 1 or Lz < 2 * nz - 1:
        raise ValueError("padded length too short for an aperiodic convolution")
    grid = np.zeros((6, Lz, Ly, Lx))
    py = np.arange(-(ny - 1), ny) % Ly
    px = np.arange(-(nx - 1), nx) % Lx
    for d in range(-(nz - 1), nz):
        zt = d * pitch
        tab = pair_table(nx, ny, dx, dy, zt, zt + thick, 0.0, thick)
        grid[:, d % Lz, py[:, None], px[None, :]] = tab
    return np.fft.fftn(grid, axes=(1, 2, 3))


def fft3_field(nx, ny, dx, dy, thick, pitch, m, Ntil3=None) -> np.ndarray:
    """h_k = -sum_l F^-1[F(N_kl) F(m_l)] with F the 3-D DFT (eq. FFT_3D), for
    nz equal layers of thickness `thick` at bottoms z_i = i * pitch, FP64.
    m: [3][nz][ny][nx] (or [B][3][nz][ny][nx]); returns the same shape."""
    mm = np.asarray(m, dtype=np.float64)
    batched = mm.ndim == 5
    if not batched:
        mm = mm[None]
    nz = mm.shape[2]
    if Ntil3 is None:
        Ntil3 = fourier_tensor3(nx, ny, dx, dy, nz, thick, pitch)
    Lz, Ly, Lx = Ntil3.shape[1:]
    N33 = full3x3(np.moveaxis(Ntil3, 0, -1))          # [Lz][Ly][Lx][3][3]
    out = np.empty_like(mm)
    for b in range(mm.shape[0]):
        mh = np.fft.fftn(mm[b], s=(Lz, Ly, Lx), axes=(1, 2, 3))   # [3][Lz][Ly][Lx]
        hh = -np.einsum("zyxkl,lzyx->kzyx", N33, mh)
        out[b] = np.real(np.fft.ifftn(hh, axes=(1, 2, 3)))[:, :nz, :ny, :nx]
    return out if batched else out[0]


# --------------------------------------------------------------------------
# Independent route: Gauss-Legendre quadrature of the dipole kernel
# --------------------------------------------------------------------------
def quad_tensor(X, Y, Z, target, source, n=12) -> np.ndarray:
    """N_kl = -(1/(4 pi |tau|)) int_tau int_tau' (3 r_k r_l - r^2 d_kl)/r^5
    with r = r_target - r_source, for DISJOINT cuboids, by n-point
    Gauss-Legendre quadrature per axis (n^6 points)."""
    xg, wg = np.polynomial.legendre.leggauss(n)

    def nodes(lo, width):
        return lo + 0.5 * width * (xg + 1.0), 0.5 * width * wg

    tx, twx = nodes(X, target[0])
    ty, twy = nodes(Y, target[1])
    tz, twz = nodes(Z, target[2])
    sx, swx = nodes(0.0, source[0])
    sy, swy = nodes(0.0, source[1])
    sz, swz = nodes(0.0, source[2])
    T = np.stack(np.meshgrid(tx, ty, tz, indexing="ij"), -1).reshape(-1, 3)
    TW = np.einsum("a,b,c->abc", twx, twy, twz).reshape(-1)
    S = np.stack(np.meshgrid(sx, sy, sz, indexing="ij"), -1).reshape(-1, 3)
    SW = np.einsum("a,b,c->abc", swx, swy, swz).reshape(-1)
    acc = np.zeros(6)
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for k0 in range(0, T.shape[0], 256):
        r = T[k0:k0 + 256, None, :] - S[None, :, :]
        r2 = np.einsum("abk,abk->ab", r, r)
        inv5 = r2 ** -2.5
        w = TW[k0:k0 + 256, None] * SW[None, :]
        for c, (a, b) in enumerate(pairs):
            ker = 3.0 * r[..., a] * r[..., b] - (r2 if a == b else 0.0)
            acc[c] += np.sum(w * ker * inv5)
    vol = target[0] * target[1] * target[2]
    return -acc / (4.0 * np.pi * vol)
