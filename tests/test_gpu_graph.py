"""The evaluation and the Heun step captured into a HIP graph (torch.cuda.CUDAGraph
on the library's stream).  After one warm-up call with the same sizes the
library enqueues kernels only (no allocation, copy, memset or host
synchronisation when check_domain and timing are off), so a captured graph
replays the same work.  Each replay follows eager work that changes the
inputs and a synchronisation, and is checked bit for bit against an eager
call on the same inputs.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

L = 2 * math.pi


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1110_2921_amd as vm
    return vm.FMM(0)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float64).T)).cuda()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_captured_evaluation_replays_exactly(ctx, precision):
    import torch
    w = W.WORKLOADS["rand32_periodic"]
    x0, a0 = W.make(w)
    x, a = dev(x0), dev(a0)
    n = w.n
    u = torch.empty((3, n), dtype=torch.float64, device="cuda")
    da = torch.empty_like(u)
    J = torch.empty((9, n), dtype=torch.float64, device="cuda")
    kw = dict(periodic=w.periodic, box_len=w.box_len, precision=precision, want_grad=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx.eval(x, a, w.sigma, w.p, w.level, out=(u, da, J), **kw)      # warm-up: workspace, operators
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ctx.eval(x, a, w.sigma, w.p, w.level, out=(u, da, J), **kw)
    torch.cuda.synchronize()
    rng = np.random.default_rng(71)
    for rep in range(4):
        # eager work between replays: new strengths and a small displacement
        x.copy_(dev(x0 + 0.05 * w.h * rng.standard_normal(x0.shape)))
        a.copy_(dev(a0 * (1.0 + 0.1 * rep)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ue, dae, Je = ctx.eval(x, a, w.sigma, w.p, w.level, **kw)
        torch.cuda.synchronize()
        assert torch.equal(u, ue) and torch.equal(da, dae) and torch.equal(J, Je), rep


def test_captured_heun_steps_replay_exactly(ctx):
    import torch
    w = W.WORKLOADS["rand32_periodic"]
    x0, a0 = W.make(w)
    kw = dict(periodic=w.periodic, box_len=w.box_len, precision="mixed")
    x, a = dev(x0), dev(a0)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx.rk2_step(x, a, w.sigma, w.p, w.level, 0.005, **kw)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(2):
            ctx.rk2_step(x, a, w.sigma, w.p, w.level, 0.005, **kw)
    for rep in range(3):
        start_x, start_a = x.clone(), a.clone()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        xe, ae = start_x.clone(), start_a.clone()
        for _ in range(2):
            ctx.rk2_step(xe, ae, w.sigma, w.p, w.level, 0.005, **kw)
        torch.cuda.synchronize()
        assert torch.equal(x, xe) and torch.equal(a, ae), rep
