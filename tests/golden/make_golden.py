"""Write the stored expected values for the full-size parity tests.

Calls only the reference oracle (brute-force sum over all source cells with
extended-precision tensor tables) and the seeded workload generators.  For each
configuration it stores sampled target cells (state, layer, iy, ix) and the
FP64 field there, for the magnetization rounded to FP32 (the GPU input).

    python tests/golden/make_golden.py [C2 M0 C3 C4 C5]

Output: tests/golden/<name>_samples.npz with
  state [S], samples [S][3] (layer, iy, ix), h [S][3], hnorm_max (largest |h|_2
  over the sampled cells; the tests divide errors by it).

    python tests/golden/make_golden.py C2full M0full

writes tests/golden/<name>_full.npz: the whole FP64 brute-force field of
state 0, [3][nz][ny][nx], stored rounded to FP32 (a relative change of at
most 2^-24 per value, far below the 1e-5 tolerance it is compared at), and
hnorm_max (largest |h|_2 over all cells, from the FP64 field).  M0 takes
about ten minutes on 8 cores.

    python tests/golden/make_golden.py C5grad

writes the thickness gradients of all 16 C5 candidate stacks.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1910_07054_amd import workloads as W  # noqa: E402

# (states to sample, target layers to sample, samples per (state, layer))
PLAN = {
    "C2": dict(states=[0], layers=None, per=32),
    "M0": dict(states=[0], layers=None, per=32),
    "C3": dict(states=[0, 21, 42, 63], layers=None, per=16),
    "C4": dict(states=[0], layers=[0, 7, 19, 31], per=48),
    "C5": dict(states=[0, 7, 15], layers=[0, 4, 9], per=24),
}


def make(name: str):
    wl = W.CONFIGS[name]()
    cfg = PLAN[name]
    rng = np.random.default_rng(4242)
    layers = cfg["layers"] if cfg["layers"] is not None else list(range(wl.nz))
    bpg = wl.batch // wl.n_geom
    st_all, smp_all, h_all = [], [], []
    t0 = time.time()
    for b in cfg["states"]:
        g = b // bpg
        s = []
        for l in layers:
            ys = rng.integers(0, wl.ny, cfg["per"])
            xs = rng.integers(0, wl.nx, cfg["per"])
            s += [[l, y, x] for y, x in zip(ys, xs)]
        s = np.array(s, dtype=np.int32)
        m = wl.m[b].astype(np.float32).astype(np.float64)
        h = oracle.field(wl.nx, wl.ny, wl.dx, wl.dy, wl.z_bottom[g], wl.thickness[g], m, samples=s)
        st_all.append(np.full(len(s), b, dtype=np.int32))
        smp_all.append(s)
        h_all.append(h)
        print(f"{name}: state {b} ({len(s)} cells) done at {time.time() - t0:.0f} s", flush=True)
    h = np.concatenate(h_all)
    out = os.path.join(HERE, f"{name}_samples.npz")
    np.savez_compressed(out, state=np.concatenate(st_all), samples=np.concatenate(smp_all), h=h,
                        hnorm_max=np.sqrt((h ** 2).sum(1)).max())
    print(f"wrote {out}", flush=True)


def make_full(name: str):
    """Every cell of state 0 by brute force (FP32-rounded m, as on the GPU)."""
    wl = W.CONFIGS[name]()
    m = wl.m[0].astype(np.float32).astype(np.float64)
    t0 = time.time()
    h = oracle.field(wl.nx, wl.ny, wl.dx, wl.dy, wl.z_bottom[0], wl.thickness[0], m)
    print(f"{name}: full field in {time.time() - t0:.0f} s on {oracle.num_threads()} threads",
          flush=True)
    out = os.path.join(HERE, f"{name}_full.npz")
    np.savez_compressed(out, h=h.astype(np.float32), hnorm_max=np.sqrt((h ** 2).sum(0)).max())
    print(f"wrote {out}", flush=True)


def make_c5_grad(candidates=tuple(range(16))):
    """Thickness gradient of L = mean over the free layer of h_z for the C5
    stacks (all ten thicknesses; gaps fixed), FP32-rounded m."""
    wl = W.c5()
    free = wl.notes["free_layer"]
    gv = np.zeros((wl.nz, 3))
    gv[free, 2] = 1.0 / (wl.nx * wl.ny)
    res = []
    t0 = time.time()
    for c in candidates:
        m = wl.m[c].astype(np.float32).astype(np.float64)
        gt = oracle.thickness_grad(wl.nx, wl.ny, wl.dx, wl.dy, wl.z_bottom[c], wl.thickness[c], m,
                                   gv, uniform=True)
        res.append(gt)
        print(f"C5grad: candidate {c} done at {time.time() - t0:.0f} s: {gt}", flush=True)
    out = os.path.join(HERE, "C5_thickness_grad.npz")
    np.savez_compressed(out, candidates=np.array(candidates), grad=np.array(res))
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(PLAN) + ["C5grad"]
    for n in names:
        if n == "C5grad":
            make_c5_grad()
        elif n.endswith("full"):
            make_full(n[:-4])
        else:
            make(n)
