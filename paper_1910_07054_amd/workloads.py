"""Seeded synthetic workloads for the demagnetization-field library.

This module only draws geometry and magnetization; it holds none of the
field computation.  Tests, the benchmark and the reference oracle all take
their inputs from here so that every side sees the same bytes.

Random streams: ``numpy.random.Generator(PCG64(seed))``; a random unit vector
is three standard-normal draws normalised to length one.  Arrays use the
layout ``[B][3][nz][ny][nx]`` (x fastest), float64.

Geometry recipes follow the stacks the paper works with (Sec. 3: layers that
share the lateral cell size and have individual thicknesses; Sec. 4: a
cylindrical MRAM stack of 64 x 64 x 5 cells).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    dx: float
    dy: float
    thickness: np.ndarray          # [G][nz] float64 (G geometries)
    z_bottom: np.ndarray           # [G][nz] float64
    m: np.ndarray                  # [B][3][nz][ny][nx] float64
    seed: int
    precision: str = "fp32"        # "fp32" or "fp64"
    notes: dict = field(default_factory=dict)

    @property
    def nz(self) -> int:
        return int(self.thickness.shape[1])

    @property
    def batch(self) -> int:
        return int(self.m.shape[0])

    @property
    def n_geom(self) -> int:
        return int(self.thickness.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def stack_bottoms(thickness: np.ndarray, gaps: np.ndarray, z0: float = 0.0) -> np.ndarray:
    """Layer bottoms of a stack with the given thicknesses and gaps (gaps[l]
    separates layer l from layer l+1)."""
    t = np.asarray(thickness, dtype=np.float64)
    g = np.asarray(gaps, dtype=np.float64)
    z = np.empty_like(t)
    acc = z0
    for l in range(t.shape[0]):
        z[l] = acc
        acc = acc + t[l] + (g[l] if l < g.shape[0] else 0.0)
    return z


def random_unit(rng: np.random.Generator, shape) -> np.ndarray:
    """Random unit vectors along axis 0 of the result ([3] + shape)."""
    v = rng.standard_normal((3,) + tuple(shape))
    return v / np.linalg.norm(v, axis=0, keepdims=True)


def tilted_alternating(rng: np.random.Generator, nz: int, ny: int, nx: int) -> np.ndarray:
    """m_j = normalize(s_j z + (u_x, u_y, 0)), u ~ U[-0.1, 0.1] per cell, s_j = (-1)^j."""
    u = rng.uniform(-0.1, 0.1, size=(2, nz, ny, nx))
    m = np.zeros((3, nz, ny, nx))
    m[0] = u[0]
    m[1] = u[1]
    for j in range(nz):
        m[2, j] = (-1.0) ** j
    return m / np.linalg.norm(m, axis=0, keepdims=True)


def mram_like_stack(rng: np.random.Generator, nz: int):
    """Thicknesses U[0.4, 3.0] nm (drawn first), gaps U[0.3, 1.5] nm."""
    t = rng.uniform(0.4, 3.0, size=nz)
    gaps = rng.uniform(0.3, 1.5, size=max(nz - 1, 0))
    return t, stack_bottoms(t, gaps)


def c1() -> Workload:
    """16 x 16 cells of 2.0 x 2.0 nm, 3 layers {1.0, 0.7, 2.3} nm, 0.5 nm gaps, FP64."""
    rng = _rng(1001)
    t = np.array([1.0, 0.7, 2.3])
    zb = stack_bottoms(t, [0.5, 0.5])
    m = random_unit(rng, (3, 16, 16))[None]
    return Workload("C1", 16, 16, 2.0, 2.0, t[None], zb[None], m, 1001, "fp64")


def _mram_state(name: str, n: int, seed: int) -> Workload:
    rng = _rng(seed)
    t, zb = mram_like_stack(rng, 8)
    m = tilted_alternating(rng, 8, n, n)[None]
    return Workload(name, n, n, 2.5, 2.5, t[None], zb[None], m, seed)


def c2() -> Workload:
    """128 x 128 cells of 2.5 nm, 8-layer MRAM-like stack."""
    return _mram_state("C2", 128, 1002)


def m0() -> Workload:
    """256 x 256 cells of 2.5 nm, 8-layer MRAM-like stack (throughput headline)."""
    return _mram_state("M0", 256, 1000)


def c3(batch: int = 64) -> Workload:
    """512 x 512 cells of 2 nm, 4 layers {1.2, 0.8, 0.9, 2.0} nm, no gaps;
    ``batch`` magnetization states of a hysteresis-like sweep:
    state s: m = normalize(a_s z + 0.5 xi), a_s = 1 - 2 s / (B - 1), xi ~ N(0, I)."""
    rng = _rng(1003)
    t = np.array([1.2, 0.8, 0.9, 2.0])
    zb = stack_bottoms(t, np.zeros(3))
    n = 512
    m = np.empty((batch, 3, 4, n, n))
    for s in range(batch):
        a = 1.0 - 2.0 * s / max(batch - 1, 1)
        v = 0.5 * rng.standard_normal((3, 4, n, n))
        v[2] += a
        m[s] = v / np.linalg.norm(v, axis=0, keepdims=True)
    return Workload("C3", n, n, 2.0, 2.0, t[None], zb[None], m, 1003)


def c4() -> Workload:
    """256 x 256 cells of 3 nm, 32 layers log-uniform in [0.3, 5] nm, no gaps."""
    rng = _rng(1004)
    t = np.exp(rng.uniform(np.log(0.3), np.log(5.0), size=32))
    zb = stack_bottoms(t, np.zeros(31))
    m = random_unit(rng, (32, 256, 256))[None]
    return Workload("C4", 256, 256, 3.0, 3.0, t[None], zb[None], m, 1004)


def c5(candidates: int = 16) -> Workload:
    """256 x 256 cells of 2.5 nm, 10 layers, no gaps.  Layers 0-8 are pinned
    (t ~ U[0.5, 3.0] nm, m along +-z with a small tilt, alternating), layer 9 is
    the free layer (random unit m); the batch holds ``candidates`` stacks whose
    free-layer thickness runs over linspace(1.0, 2.0)."""
    rng = _rng(1005)
    t_pinned = rng.uniform(0.5, 3.0, size=9)
    m = tilted_alternating(rng, 10, 256, 256)
    m[:, 9] = random_unit(rng, (256, 256))
    tf = np.linspace(1.0, 2.0, candidates)
    T = np.empty((candidates, 10))
    Z = np.empty((candidates, 10))
    for c in range(candidates):
        T[c, :9] = t_pinned
        T[c, 9] = tf[c]
        Z[c] = stack_bottoms(T[c], np.zeros(9))
    mm = np.broadcast_to(m[None], (candidates,) + m.shape).copy()
    return Workload("C5", 256, 256, 2.5, 2.5, T, Z, mm, 1005, notes={"free_layer": 9})


def mram_disk(t_mid: float = 5.0, n: int = 64) -> Workload:
    """Cylindrical SAFM stack of Sec. 4: 60 nm disk on n x n cells of 60/n nm;
    5 nm pinned (+z) / 1 nm spacer / t_mid pinned (-z) / 1 nm spacer / 3 nm free.
    The spacers are carried as gaps; the free layer has m = 0 (its own field is
    not part of the stray field of the two pinned layers).  Cells belong to the
    disk when their centre lies within 30 nm of the axis."""
    d = 60.0 / n
    t = np.array([5.0, t_mid, 3.0])
    zb = stack_bottoms(t, [1.0, 1.0])
    c = (np.arange(n) + 0.5) * d - 30.0
    X, Y = np.meshgrid(c, c, indexing="xy")
    disk = (X * X + Y * Y) <= 30.0 * 30.0
    m = np.zeros((1, 3, 3, n, n))
    m[0, 2, 0][disk] = 1.0
    m[0, 2, 1][disk] = -1.0
    return Workload("MRAM", n, n, d, d, t[None], zb[None], m, 0, "fp64",
                    notes={"free_layer": 2, "disk": disk})


def small_case(nx: int, ny: int, nz: int, seed: int, batch: int = 1, dx: float = 2.0,
               dy: float = 1.5) -> Workload:
    """Small random stack for element-by-element parity: thicknesses
    U[0.4, 3.0], gaps U[0, 1.0] (some layers touch), random unit m."""
    rng = _rng(seed)
    t = rng.uniform(0.4, 3.0, size=nz)
    gaps = rng.uniform(0.0, 1.0, size=max(nz - 1, 0))
    gaps[rng.uniform(size=gaps.shape) < 0.3] = 0.0
    zb = stack_bottoms(t, gaps)
    m = np.stack([random_unit(rng, (nz, ny, nx)) for _ in range(batch)])
    return Workload(f"small{nx}x{ny}x{nz}", nx, ny, dx, dy, t[None], zb[None], m, seed)


CONFIGS = {"C1": c1, "C2": c2, "M0": m0, "C3": c3, "C4": c4, "C5": c5}
