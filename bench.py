"""Throughput benchmark of the hybrid-FFT demagnetization field on one MI355X.

One step = one full field evaluation h = -N * m (x-pass R2C, y-pass with the
explicit z-mixing, inverse x-pass) of the 256 x 256 x 8 MRAM-like stack
(2.5 nm cells, FP32 field, tensor set up in FP64 beforehand), inputs resident
in HBM.  Steps are replayed from a HIP graph that holds G complete evaluations
(G: the largest divisor of K up to 50, or --graph-evals), so K steps are K / G
replays.  Prints one JSON line.

The line carries the roofline of the dominant kernel against the method's
algorithmic bytes (m in, h out, the unique FP32 Fourier tensor once), the
end-to-end fraction, per-evaluation median / p10 / p90 over many replays,
a table of the other workloads (128^2 x 8, 512^2 x 4 with 64 states,
256^2 x 32, 256^2 x 10 with 16 thickness candidates and its VJP), and the
oracle timed on the host: the hybrid FFT of eq. FFT_v2 in numpy and the
brute-force sum.

  python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--no-configs] [--no-graph]
                  [--graph-evals G]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, public spec
FP32_VALU_PEAK_TFLOPS = 157.3   # MI355X FP32 vector, public spec (packed FMA)
FP32_VALU_NONPACKED_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (one FMA per lane)
STATS_REPLAYS = 200             # replays behind the median / p10 / p90


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="M0")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the table of the other workloads (C2, C3, C4, C5 and the C5 VJP)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--graph-evals", type=int, default=0,
                    help="evaluations captured per HIP graph (0: the largest divisor of --steps "
                         "up to 50); each replay runs that many complete evaluations")
    ap.add_argument("--split", action="store_true", help="force the five-pass path")
    ap.add_argument("--compare", action="store_true",
                    help="also time every mixing path (and 64 single-state calls) on the workload, "
                         "each with its error against the stored oracle values")
    ap.add_argument("--nz-sweep", action="store_true",
                    help="also time the explicit layer sum and the equidistant z-FFT path on "
                         "256x256 x nz equal-thickness stacks, nz = 1 .. 64 (Sec. 3.2 scaling)")
    ap.add_argument("--vjp", action="store_true",
                    help="also time hfd_demag_vjp (grad m and grad thickness) on the workload, with the "
                         "derivative tensors recomputed per call and stored")
    ap.add_argument("--hysteresis", type=int, default=0, metavar="STEPS",
                    help="also run the free-layer hysteresis loop of Sec. 4 with STEPS field steps "
                         "(the paper uses 2000; L-BFGS relaxation per step on the library's energy "
                         "and gradient) and report the switching field")
    ap.add_argument("--cpu-hybrid-child", nargs=3, metavar=("WORKLOAD", "WORKERS", "SECONDS"),
                    help=argparse.SUPPRESS)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def graph_evals(steps: int, requested: int = 0) -> int:
    """Evaluations captured per HIP graph: `requested`, or the largest divisor
    of `steps` up to 50, so that `steps` evaluations are a whole number of
    replays (a time-stepping code captures its inner loop the same way; each
    replay boundary costs about 1 us per evaluation at 10 per graph)."""
    if steps < 1:
        raise SystemExit("--steps must be >= 1")
    G = requested or max(d for d in range(1, 51) if steps % d == 0)
    if G < 1 or steps % G:
        raise SystemExit(f"--steps {steps} is not a multiple of --graph-evals {G}")
    return G


def algorithmic_bytes(nx, ny, nz, B, G=1):
    """Bytes the method must move per launch: m in and h out in FP32
    (24 nx ny nz per state) plus the unique-pair Fourier tensor, six FP32
    components on the (nx+1) x (ny+1) quadrant, read once per stack."""
    P = nz * (nz + 1) // 2
    return B * 24 * nx * ny * nz + G * 24 * (nx + 1) * (ny + 1) * P


def with_distinct_tensor(roof, nx, ny, nz, B, slots):
    """Add to a roofline record the bytes with the tensor counted once per
    distinct pair geometry of all stacks (`slots`: stacks that differ in one
    layer share the other pairs, and the plan stores and reads them once) and
    the dominant kernel's fraction of HBM peak on those bytes."""
    b = B * 24 * nx * ny * nz + 24 * (nx + 1) * (ny + 1) * slots
    roof["tensor_slots"] = slots
    roof["alg_bytes_distinct"] = b
    roof["frac_distinct"] = b / (roof["kernel_ms"] * 1e-3) / (HBM_PEAK_GBPS * 1e9)
    return roof


def algorithmic_flops(nx, ny, nz, B):
    """FP32 flops per launch: the pruned 2D FFTs (5 N log2 N convention) of
    the 3 nz input and output signals and the explicit layer sum, 36 nz^2
    per frequency of the (nx+1) x 2ny half spectrum."""
    Lx, Ly = 2 * nx, 2 * ny
    fft = 3 * nz * 2 * (ny * 2.5 * Lx * np.log2(Lx) + (nx + 1) * 5 * Ly * np.log2(Ly))
    mix = 36 * nz * nz * (nx + 1) * Ly
    return B * (fft + mix)


def fused_kernel_bytes(nx, ny, nz, B, Lx, Ly):
    """Bytes the fused y-pass kernel itself moves: the x-pass spectra in and
    out (complex64, Lx/2 columns of ny) plus the stored tensor quadrant (five
    FP32 components; zz follows from the trace)."""
    P = nz * (nz + 1) // 2
    return 2 * B * 3 * nz * (Lx // 2) * ny * 8 + P * 5 * (Lx // 2 + 1) * (Ly // 2 + 1) * 4


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "M0_fused_traffic.txt")
FUSED_SOURCES = ["hfd_device.hpp", "field_kernels.hpp", "fused.hip", "fused_exact.hpp",
                 "fused_exact_1.hip", "fused_exact_2.hip", "fused_exact_3.hip", "fused_exact_4.hip",
                 "fused_exact_5.hip"]


def measured_traffic(workload):
    """HBM bytes per dispatch of the fused kernel from the stored counter runs
    (copy-calibrated FETCH_SIZE + WRITE_SIZE), or None if they were taken on
    other kernel sources or another workload."""
    import hashlib
    if workload != "M0" or not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        line = line.strip()
        if line and not line.startswith("#") and "=" in line:
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in FUSED_SOURCES:
        with open(os.path.join(ROOT, "paper_1910_07054_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != kv.get("source_sha256"):
        return None
    return 1024.0 * (float(kv["fetch_kb"]) * float(kv["fetch_factor"]) +
                     float(kv["write_kb"]) * float(kv["write_factor"]))


def cpu_baseline_bruteforce(wl, target_s=12.0):
    """The oracle's brute-force sum timed on a bounded sample of target cells of
    layer 0 (all sources of all layers), extrapolated to one full evaluation.
    Pair-table construction (the oracle's tensor setup) is timed apart and not
    counted, as the GPU figure excludes the tensor setup."""
    import oracle
    zb, t = wl.z_bottom[0], wl.thickness[0]
    m = wl.m[0].astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(7)

    def samples(n):
        ys = rng.integers(0, wl.ny, n)
        xs = rng.integers(0, wl.nx, n)
        return np.stack([np.zeros(n, dtype=np.int64), ys, xs], 1)

    t0 = time.perf_counter()
    oracle.field(wl.nx, wl.ny, wl.dx, wl.dy, zb, t, m, samples=samples(1))
    t_tab = time.perf_counter() - t0
    n = 64
    t0 = time.perf_counter()
    oracle.field(wl.nx, wl.ny, wl.dx, wl.dy, zb, t, m, samples=samples(n))
    t_n = time.perf_counter() - t0
    per = max((t_n - t_tab) / n, 1e-9)
    n2 = int(min(131072, max(n, target_s / per)))
    t0 = time.perf_counter()
    oracle.field(wl.nx, wl.ny, wl.dx, wl.dy, zb, t, m, samples=samples(n2))
    t_n2 = time.perf_counter() - t0
    per = max((t_n2 - t_tab) / n2, 1e-12)
    cells = wl.nx * wl.ny * wl.nz
    t_eval = per * cells
    return {
        "value": 1.0 / t_eval,
        "unit": "evals/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"brute-force FP64 sum (extended-precision tensor tables, quadrature beyond 50 cell "
                   f"sizes) for {n2} random target "
                   f"cells of layer 0 against all {cells} source cells, {t_n2:.1f} s incl. "
                   f"{t_tab:.1f} s of pair tables for that layer; extrapolated to {cells} targets "
                   f"= {t_eval:.0f} s per evaluation (tables excluded)"),
    }


CPU_WORKERS = 16   # host cores of the measurement box's share per GPU

_HYBRID = {}       # the child's workload and Fourier tensor, inherited by its forked workers


def _hybrid_worker(deadline):
    """Evaluations of the oracle's hybrid FFT until `deadline` (time.monotonic)."""
    import oracle
    wl, Ntil = _HYBRID["wl"], _HYBRID["Ntil"]
    zb, t = wl.z_bottom[0], wl.thickness[0]
    n = 0
    while True:
        oracle.fft_field(wl.nx, wl.ny, wl.dx, wl.dy, zb, t, _HYBRID["m"], Ntil=Ntil)
        n += 1
        if time.monotonic() >= deadline:
            return n


def cpu_hybrid_child(name, workers, target_s):
    """The all-core oracle baseline, run in a child process that never touches
    the GPU: the oracle's Fourier tensor of the workload is built once, then
    `workers` forked processes each evaluate the oracle's hybrid FFT (one
    thread each) for target_s seconds; prints one JSON object."""
    import multiprocessing as mp
    import oracle
    from paper_1910_07054_amd import workloads as W
    wl = W.CONFIGS[name]()
    zb, t = wl.z_bottom[0], wl.thickness[0]
    t0 = time.perf_counter()
    Ntil = oracle.fourier_tensor(wl.nx, wl.ny, wl.dx, wl.dy, zb, t)
    t_setup = time.perf_counter() - t0
    _HYBRID.update(wl=wl, Ntil=Ntil, m=wl.m[0].astype(np.float32).astype(np.float64))
    start = time.monotonic()
    with mp.get_context("fork").Pool(workers) as pool:
        counts = pool.map(_hybrid_worker, [start + target_s] * workers)
    wall = time.monotonic() - start
    print(json.dumps({"evals": int(sum(counts)), "wall_s": wall, "workers": workers,
                      "setup_s": t_setup, "pair_threads": oracle.num_threads()}), flush=True)


def cpu_baseline_hybrid(wl, target_s=10.0):
    """The oracle's hybrid FFT (eq. FFT_v2: numpy 2D FFTs per layer, explicit
    layer sum per frequency, inverse FFT, crop) on the full workload, the same
    algorithm as the GPU path in FP64, as throughput over the host cores:
    independent evaluations in CPU_WORKERS single-threaded processes (the
    oracle itself is unchanged).  Its Fourier tensor (the oracle's pair tables
    and their DFTs) is built first and timed apart, like the GPU's tensor
    setup."""
    import subprocess
    workers = max(1, min(CPU_WORKERS, os.cpu_count() or 1))
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-hybrid-child", wl.name, str(workers),
           str(target_s)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"CPU baseline child failed ({r.returncode}): {r.stderr[-2000:]}")
    d = json.loads([ln for ln in r.stdout.splitlines() if ln.startswith("{")][-1])
    rate = d["evals"] / d["wall_s"]
    return {
        "value": rate,
        "unit": "evals/s",
        "cores": d["workers"],
        "kind": "oracle",
        "sample": (f"hybrid FFT of eq. FFT_v2 in FP64 (numpy FFT and einsum) on the whole "
                   f"{wl.nx}x{wl.ny}x{wl.nz} workload: {d['evals']} evaluations by {d['workers']} "
                   f"single-threaded processes in {d['wall_s']:.1f} s "
                   f"({d['workers'] / rate:.2f} s per evaluation and process); its Fourier tensor "
                   f"(pair tables on {d['pair_threads']} threads + DFTs) took {d['setup_s']:.1f} s "
                   f"and is not counted"),
        "tensor_setup_s": d["setup_s"],
    }


def golden_error(wl, h):
    """max |h - h_oracle| / max |h_oracle| over the stored oracle samples of
    this workload (None if there are none)."""
    gpath = os.path.join(ROOT, "tests", "golden", f"{wl.name}_samples.npz")
    if not os.path.exists(gpath):
        return None
    g = np.load(gpath)
    import torch
    idx = [torch.as_tensor(a, device=h.device) for a in (g["state"], *g["samples"].T)]
    got = h[idx[0], :, idx[1], idx[2], idx[3]].double().cpu().numpy()
    return float(np.abs(got.astype(np.float64) - g["h"]).max() / g["hnorm_max"])


def replay_ms(fn, steps, warmup, stream):
    """Capture fn() into a HIP graph and time `steps` replays; ms per replay."""
    import torch
    with torch.cuda.stream(stream):
        for _ in range(max(warmup, 1)):
            fn()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        fn()
    for _ in range(3):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def compare_paths(wl, m, steps, warmup, stream, only=None):
    """Every field path (or the ones named in `only`) on the same states: one
    plan per path, B states per call, plus the plain single-state form (B calls
    of one state)."""
    import torch
    from paper_1910_07054_amd import hfd
    B = wl.batch
    res = {}
    h = torch.empty_like(m)
    plan1 = hfd.Plan(wl.nx, wl.ny, wl.dx, wl.dy, wl.thickness, wl.z_bottom, batch_max=1, flags=hfd.HFD_FP32)
    tune1 = plan1.autotune(1)

    def single():
        for b in range(B):
            plan1.field(m[b:b + 1], out=h[b:b + 1], stream=stream)
    ms = replay_ms(single, max(steps // 4, 5), warmup, stream)
    res["single_state_fp32_fused"] = {"ms_per_batch": ms, "evals_per_s": B / (ms * 1e-3),
                                      "err_vs_fp64_oracle": golden_error(wl, h), "autotune": tune1}
    plan1.destroy()
    variants = [("fused_fp32", hfd.HFD_FP32), ("five_pass_fp32", hfd.HFD_SPLIT_PASSES),
                ("five_pass_batched_fp32", hfd.HFD_MIX_BATCHED_FP32),
                ("five_pass_split_bf16_mfma", hfd.HFD_MIX_SPLIT_BF16)]
    for name, fl in variants:
        if only is not None and name not in only:
            continue
        plan = hfd.Plan(wl.nx, wl.ny, wl.dx, wl.dy, wl.thickness, wl.z_bottom, batch_max=B, flags=fl)
        # each variant with its own tuned x tile (and, on the fused path, state
        # runs and kernel); the path itself stays the one the flags select
        tune = plan.autotune(B)
        path = {hfd.HFD_FP32: 0, hfd.HFD_SPLIT_PASSES: 1, hfd.HFD_MIX_BATCHED_FP32: 2,
                hfd.HFD_MIX_SPLIT_BF16: 3}[fl]
        if f"-> {('fused', 'five_pass', 'five_pass_batched_fp32', 'five_pass_bf16_mfma')[path]} " not in tune + " ":
            plan.set_path(B, path, int(tune.rsplit(" x", 1)[1].split()[0]))
        h.zero_()
        ms = replay_ms(lambda: plan.field(m, out=h, stream=stream), steps, warmup, stream)
        res[name] = {"ms_per_batch": ms, "evals_per_s": B / (ms * 1e-3),
                     "err_vs_fp64_oracle": golden_error(wl, h), "autotune": tune,
                     "stage_ms": plan.time_stages(m, h, reps=max(steps // 4, 5), stream=stream)}
        plan.destroy()
    base = res["single_state_fp32_fused"]["ms_per_batch"]
    for v in res.values():
        v["speedup_vs_single_state"] = base / v["ms_per_batch"]
    return res


def run_hysteresis(steps):
    """Sec. 4: hysteresis of the free layer of the optimised MRAM disk (64 x 64
    cells, SAFM middle layer 3.4389 nm), field along z (tilted 1e-4 rad), loop
    +2.5 T -> -2.5 T -> +2.5 T in `steps` steps, L-BFGS per step.  The paper
    reports 1.51 T for 2000 steps."""
    from paper_1910_07054_amd import micromag as mm
    res = mm.mram_hysteresis(steps=steps, progress=max(steps // 8, 1))
    ev = int(res["evaluations"].sum())
    return {"steps": steps, "seconds": res["seconds"], "energy_evaluations": ev,
            "ms_per_evaluation": res["seconds"] * 1e3 / max(ev, 1),
            "lbfgs_iterations": int(res["iterations"].sum()),
            "switching_T": res["switching_T"], "H_sw_T": res["H_sw_T"], "paper_H_sw_T": 1.51,
            "macrospin_estimate": res["estimate"], "field_tilt_rad": mm.FIELD_TILT}


def nz_sweep(steps, warmup, stream, nzs=(1, 2, 4, 8, 16, 32, 64)):
    """Field evaluation time of the explicit layer sum (fastest path after
    autotuning) and of the equidistant z-FFT path on the same 256 x 256 x nz
    stack of equal 1 nm layers (2.5 nm cells, no gaps, alternating +-z
    magnetization with a small tilt), with the least-squares fits of Sec. 3.2:
    a nz^2 + b nz + c and a nz log nz + b."""
    import torch
    from paper_1910_07054_amd import hfd
    from paper_1910_07054_amd import workloads as W
    rows = []
    for nz in nzs:
        rng = np.random.default_rng(1100 + nz)
        t = np.ones(nz)
        zb = np.arange(nz, dtype=np.float64)
        m = torch.from_numpy(W.tilted_alternating(rng, nz, 256, 256)[None].astype(np.float32)).cuda()
        row = {"nz": nz}
        outs = {}
        for name, fl in (("layer_sum", hfd.HFD_FP32), ("equidistant", hfd.HFD_EQUIDISTANT)):
            t0 = time.perf_counter()
            plan = hfd.Plan(256, 256, 2.5, 2.5, t, zb, batch_max=1, flags=fl)
            setup = time.perf_counter() - t0
            rep = plan.autotune(1)
            h = torch.empty_like(m)
            ms = replay_ms(lambda: plan.field(m, out=h, stream=stream), steps, warmup, stream)
            outs[name] = h.double()
            row[name + "_ms"] = ms
            row[name + "_setup_s"] = setup
            row[name + "_path"] = rep.split("-> ")[-1]
            plan.destroy()
        d = (outs["layer_sum"] - outs["equidistant"]).abs().max().item()
        row["max_diff_rel"] = d / outs["layer_sum"].norm(dim=1).max().item()
        print(f"nz_sweep nz={nz}: " + json.dumps(row), file=sys.stderr, flush=True)
        rows.append(row)
        del m, outs
        torch.cuda.empty_cache()
    x = np.array([r["nz"] for r in rows], dtype=np.float64)
    y1 = np.array([r["layer_sum_ms"] for r in rows])
    y2 = np.array([r["equidistant_ms"] for r in rows])
    a1 = np.linalg.lstsq(np.stack([x * x, x, np.ones_like(x)], 1), y1, rcond=None)[0]
    a2 = np.linalg.lstsq(np.stack([x * np.log(x), np.ones_like(x)], 1), y2, rcond=None)[0]
    return {"rows": rows, "fit_layer_sum_ms": {"a_nz2": a1[0], "b_nz": a1[1], "c": a1[2]},
            "fit_equidistant_ms": {"a_nzlognz": a2[0], "b": a2[1]}}


def time_vjp(wl, m, steps, warmup, stream):
    """hfd_demag_vjp for L = mean of h_z over the last layer (the free layer of
    C5) of every state: grad_m and grad_thickness, derivative tensors
    recomputed per call or stored in the plan; graph replay."""
    import torch
    from paper_1910_07054_amd import hfd
    res = {}
    gh = torch.zeros_like(m)
    gh[:, 2, -1] = 1.0 / (wl.nx * wl.ny)
    for name, fl in (("recomputed", hfd.HFD_FP32), ("stored", hfd.HFD_FP32 | hfd.HFD_STORE_DTENSOR)):
        t0 = time.perf_counter()
        plan = hfd.Plan(wl.nx, wl.ny, wl.dx, wl.dy, wl.thickness, wl.z_bottom, batch_max=wl.batch, flags=fl)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        out = {}

        def run():
            gm, gt = plan.vjp(m, gh, want_m=True, want_t=True, stream=stream)
            out["gm"], out["gt"] = gm, gt
        ms = replay_ms(run, steps, warmup, stream)
        res[name] = {"ms_per_call": ms, "ms_per_state": ms / wl.batch, "setup_s": setup_s}
        plan.destroy()
    return res


def percentiles(x):
    x = np.asarray(x, dtype=np.float64)
    return {"median": float(np.median(x)), "p10": float(np.percentile(x, 10)),
            "p90": float(np.percentile(x, 90)), "n": int(x.size)}


def replay_stats(graph, stream, per_replay, n):
    """Per-evaluation times of n replays of `graph` (each holds `per_replay`
    evaluations), measured with HIP events on the launch stream."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(n)]
    with torch.cuda.stream(stream):
        for e0, e1 in evs:
            e0.record(stream)
            graph.replay()
            e1.record(stream)
    torch.cuda.synchronize()
    return percentiles([e0.elapsed_time(e1) / per_replay for e0, e1 in evs])


def roofline_of(stages, alg_bytes, alg_flops, ms_per_eval, kernel_bytes=None):
    """Roofline of the dominant stage: the method's algorithmic bytes per
    launch against HBM and its algorithmic FP32 flops against the FP32
    vector peak, both over the stage's duration; `bound` names the resource
    with the larger fraction ("hbm" or "alu", the vector ALUs: the field path
    uses no MFMA).  End-to-end fractions over the whole evaluation beside it."""
    dom = max(stages, key=stages.get)
    dom_ms = stages[dom]
    gbps = alg_bytes / (dom_ms * 1e-3) / 1e9
    tflops = alg_flops / (dom_ms * 1e-3) / 1e12
    e2e = alg_bytes / (ms_per_eval * 1e-3) / 1e9
    tf = alg_flops / (ms_per_eval * 1e-3) / 1e12
    if tflops / FP32_VALU_PEAK_TFLOPS > gbps / HBM_PEAK_GBPS:
        head = {"bound": "alu", "achieved": tflops, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tflops / FP32_VALU_PEAK_TFLOPS, "hbm_frac": gbps / HBM_PEAK_GBPS}
    else:
        head = {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": gbps / HBM_PEAK_GBPS, "alu_frac": tflops / FP32_VALU_PEAK_TFLOPS}
    r = dict(head, kernel=dom, kernel_ms=dom_ms, alg_bytes_per_launch=alg_bytes,
             alg_flops_per_launch=alg_flops,
             end_to_end_GBps=e2e, end_to_end_frac=e2e / HBM_PEAK_GBPS,
             valu_TFLOPs=tf, valu_frac=tf / FP32_VALU_PEAK_TFLOPS,
             valu_frac_nonpacked=tf / FP32_VALU_NONPACKED_TFLOPS)
    if kernel_bytes is not None:
        kb = kernel_bytes / (dom_ms * 1e-3) / 1e9
        r["kernel_own_bytes"] = kernel_bytes
        r["kernel_frac"] = kb / HBM_PEAK_GBPS
    return r


def measure_config(name, steps, warmup, stream):
    """One workload: autotuned field path, graph of 10 evaluations, per
    evaluation median / p10 / p90 over 40 replays, stage durations, roofline
    and error against the stored oracle samples."""
    import torch
    from paper_1910_07054_amd import hfd
    from paper_1910_07054_amd import workloads as W
    wl = W.CONFIGS[name]()
    B, G = wl.batch, wl.n_geom
    t0 = time.perf_counter()
    plan = hfd.Plan(wl.nx, wl.ny, wl.dx, wl.dy, wl.thickness, wl.z_bottom, batch_max=B)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    tune = plan.autotune(B)
    m = torch.from_numpy(wl.m.astype(np.float32)).cuda()
    h = torch.empty_like(m)
    with torch.cuda.stream(stream):
        for _ in range(max(warmup, 1)):
            plan.field(m, out=h, stream=stream)
    torch.cuda.synchronize()
    ge = 10
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        for _ in range(ge):
            plan.field(m, out=h, stream=stream)
    graph.replay()
    torch.cuda.synchronize()
    st = replay_stats(graph, stream, ge, 40)
    stages = plan.time_stages(m, h, reps=20, stream=stream)
    plan.field(m, out=h, stream=stream)
    torch.cuda.synchronize()
    err = golden_error(wl, h)
    ms = st["median"]
    inf = plan.info()
    res = {"workload": f"{wl.nx}x{wl.ny}x{wl.nz}, {B} state(s), {G} stack(s)",
           "evals_per_s": B / (ms * 1e-3), "ms_per_launch": st,
           "cell_updates_per_s": B * wl.nx * wl.ny * wl.nz / (ms * 1e-3),
           "path": tune.split("-> ")[-1], "stage_ms": stages, "setup_s": setup_s,
           "err_vs_fp64_oracle": err,
           "roofline": with_distinct_tensor(
               roofline_of(stages, algorithmic_bytes(wl.nx, wl.ny, wl.nz, B, G),
                           algorithmic_flops(wl.nx, wl.ny, wl.nz, B), ms),
               wl.nx, wl.ny, wl.nz, B, inf.tensor_slots)}
    if name == "C5":
        res["vjp"] = time_vjp(wl, m, 10, 2, stream)
    if name == "C3":
        # the batched launch against the plain single-state form, and the
        # split-BF16 matrix-core mixing beside it, on the same 64 states
        forms = compare_paths(wl, m, 20, warmup, stream, only=("five_pass_split_bf16_mfma",))
        forms["batched_fused_fp32"] = {"ms_per_batch": ms, "evals_per_s": B / (ms * 1e-3),
                                       "err_vs_fp64_oracle": err,
                                       "speedup_vs_single_state":
                                           forms["single_state_fp32_fused"]["ms_per_batch"] / ms}
        res["forms"] = forms
    del graph
    plan.destroy()
    del m, h
    torch.cuda.empty_cache()
    print(f"config {name}: {res['evals_per_s']:.0f} evals/s, err {err}", file=sys.stderr, flush=True)
    return res


def main():
    args = parse()
    if args.cpu_hybrid_child:
        name, workers, secs = args.cpu_hybrid_child
        cpu_hybrid_child(name, int(workers), float(secs))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build measures one GPU only (the method needs no inter-GPU "
              "exchange for a single field evaluation at this size); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1910_07054_amd import hfd
    from paper_1910_07054_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    hfd.load()
    wl = W.CONFIGS[args.workload]()
    dev = torch.device("cuda:0")
    B = wl.batch
    flags = hfd.HFD_FP32 | (hfd.HFD_SPLIT_PASSES if args.split else 0)
    t0 = time.perf_counter()
    plan = hfd.Plan(wl.nx, wl.ny, wl.dx, wl.dy, wl.thickness, wl.z_bottom, batch_max=B, flags=flags)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    inf = plan.info()
    tune = plan.autotune(B)
    m = torch.from_numpy(wl.m.astype(np.float32)).to(dev)
    h = torch.empty_like(m)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    with torch.cuda.stream(stream):
        for _ in range(max(args.warmup, 1)):
            plan.field(m, out=h, stream=stream)
    torch.cuda.synchronize()

    # G evaluations per graph (a time-stepping code captures its inner loop the
    # same way); K steps = K / G replays, every step a complete evaluation
    graph = None
    G = 1
    if not args.no_graph:
        G = graph_evals(args.steps, args.graph_evals)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            for _ in range(G):
                plan.field(m, out=h, stream=stream)
        for _ in range(3):
            graph.replay()
        torch.cuda.synchronize()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        if graph is not None:
            for _ in range(args.steps // G):
                graph.replay()
        else:
            for _ in range(args.steps):
                plan.field(m, out=h, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    evals_per_s = B / (elapsed / args.steps)

    # distribution: STATS_REPLAYS replays of the same graph, HIP events on
    # the launch stream, per evaluation
    stats = replay_stats(graph, stream, G, STATS_REPLAYS) if graph is not None else None

    # per-stage kernel durations with HIP events on the launch stream (each
    # stage launched back to back; this leaves h overwritten, so the field is
    # evaluated once more for the accuracy check)
    stages = plan.time_stages(m, h, reps=max(args.steps, 10), stream=stream)
    plan.field(m, out=h, stream=stream)
    torch.cuda.synchronize()
    alg_bytes = algorithmic_bytes(wl.nx, wl.ny, wl.nz, B, wl.n_geom)
    alg_flops = algorithmic_flops(wl.nx, wl.ny, wl.nz, B)
    err = golden_error(wl, h)

    dom = max(stages, key=stages.get)
    kbytes = fused_kernel_bytes(wl.nx, wl.ny, wl.nz, B, inf.Lx, inf.Ly) if dom == "ymix_fused" else None
    roof = roofline_of(stages, alg_bytes, alg_flops, stats["median"] if stats else ms_per_step / B,
                       kbytes)
    with_distinct_tensor(roof, wl.nx, wl.ny, wl.nz, B, inf.tensor_slots)
    roof["traffic"] = measured_traffic(args.workload) if dom == "ymix_fused" else None
    roof["traffic_unit"] = "bytes per launch of the dominant kernel (copy-calibrated FETCH_SIZE + WRITE_SIZE)"

    out = {
        "metric": "demag field evals/s at 256^2 x 8 layers",
        "value": evals_per_s,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.nx}x{wl.ny} cells of {wl.dx} nm, {wl.nz} layers "
                               f"(MRAM-like stack, seed {wl.seed}), batch {B}, FP32 field / FP64 tensor",
                   "nx": wl.nx, "ny": wl.ny, "nz": wl.nz, "batch": B, "Lx": inf.Lx, "Ly": inf.Ly,
                   "path": "fused" if inf.fused else "split", "graph": graph is not None,
                   "evals_per_graph": G if graph is not None else 0},
        "cell_updates_per_s": evals_per_s * wl.nx * wl.ny * wl.nz,
        "alg_GBps": alg_bytes / (elapsed / args.steps) / 1e9,
        "alg_bytes_per_eval": alg_bytes,
        "ms_per_eval_stats": stats,
        "err_vs_fp64_oracle": err,
        "stage_ms": stages,
        "setup_ms": setup_ms,
        "autotune": tune,
        "roofline": roof,
    }
    del graph
    plan.destroy()
    if not args.no_configs:
        out["configs"] = {}
        for name in ("C2", "C3", "C4", "C5"):
            out["configs"][name] = measure_config(name, args.steps, args.warmup, stream)
    if args.compare:
        out["path_comparison"] = compare_paths(wl, m, args.steps, args.warmup, stream)
    if args.nz_sweep:
        out["nz_sweep"] = nz_sweep(max(args.steps // 4, 20), args.warmup, stream)
    if args.vjp:
        out["vjp"] = time_vjp(wl, m, max(args.steps // 4, 10), args.warmup, stream)
    if args.hysteresis:
        out["hysteresis"] = run_hysteresis(args.hysteresis)
    if not args.no_cpu_baseline:
        cb = cpu_baseline_hybrid(wl)
        cb["bruteforce"] = cpu_baseline_bruteforce(wl)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
