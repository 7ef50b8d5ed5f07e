"""HIP-graph capture of the field and VJP calls: every replay, with eager work
and synchronizations between replays, must reproduce the eager result."""
import numpy as np
import pytest

from paper_1910_07054_amd import hfd
from paper_1910_07054_amd import workloads as W

pytestmark = pytest.mark.gpu


def _replay_check(plan, run, make_inputs, n_replays=4):
    """run(inputs, stream) -> tuple of output tensors, captured once; inputs are
    overwritten in place before each replay."""
    import torch
    s = torch.cuda.Stream()
    inputs = make_inputs(0)
    with torch.cuda.stream(s):
        run(inputs, s)                      # warm-up (eager)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        outs = run(inputs, s)
    torch.cuda.synchronize()
    for r in range(1, n_replays + 1):
        new = make_inputs(r)
        for dst, src in zip(inputs, new):
            dst.copy_(src)                   # eager work on the default stream
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [o.clone() for o in outs]
        with torch.cuda.stream(s):
            ref = run(new, s)                # eager evaluation of the same inputs
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b), f"replay {r} differs from the eager call"


@pytest.mark.parametrize("flags", [hfd.HFD_FP32, hfd.HFD_SPLIT_PASSES, hfd.HFD_MIX_SPLIT_BF16,
                                   hfd.HFD_FP64],
                         ids=["fused", "five_pass", "bf16_mfma", "fp64"])
def test_field_graph_replays_match_eager(flags):
    import torch
    wl = W.small_case(40, 28, 3, seed=71, batch=16)
    plan = hfd.Plan(wl.nx, wl.ny, wl.dx, wl.dy, wl.thickness, wl.z_bottom, batch_max=16, flags=flags)
    dt = torch.float64 if flags & hfd.HFD_FP64 else torch.float32
    rng = np.random.default_rng(5)

    def make(r):
        return [torch.from_numpy(rng.standard_normal(wl.m.shape)).to(dtype=dt, device="cuda")]

    def run(inp, s):
        return (plan.field(inp[0], stream=s),)

    _replay_check(plan, run, make)
    plan.destroy()


@pytest.mark.parametrize("store", [False, True], ids=["recompute", "stored"])
def test_vjp_graph_replays_match_eager(store):
    import torch
    wl = W.small_case(24, 20, 3, seed=72, batch=2)
    flags = hfd.HFD_FP32 | (hfd.HFD_STORE_DTENSOR if store else 0)
    plan = hfd.Plan(wl.nx, wl.ny, wl.dx, wl.dy, wl.thickness, wl.z_bottom, batch_max=2, flags=flags)
    rng = np.random.default_rng(6)

    def make(r):
        return [torch.from_numpy(rng.standard_normal(wl.m.shape)).float().cuda(),
                torch.from_numpy(rng.standard_normal(wl.m.shape)).float().cuda()]

    def run(inp, s):
        return plan.vjp(inp[0], inp[1], want_m=True, want_t=True, stream=s)

    _replay_check(plan, run, make)
    plan.destroy()
