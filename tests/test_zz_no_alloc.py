"""The allocation-free diagnostics entry point (vm_diagnostics_noalloc) against
vm_diagnostics, through the C ABI: two calls in a row on one context, the
second on a smaller input, each compared bit for bit with the allocating entry
point on the same arrays (same kernels, same grid, same reduction order), and
with the FP64 sums computed on the host."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_1110_2921_amd as vm

pytestmark = pytest.mark.gpu


def _host_sums(u, J, a, h3):
    u = u.cpu().numpy()
    J = J.cpu().numpy()
    a = a.cpu().numpy()
    w = np.stack([J[5] - J[7], J[6] - J[2], J[1] - J[3]])
    return np.array([0.5 * h3 * np.sum(u * u), 0.5 * h3 * np.sum(w * w), 0.5 * np.sum(a * a) / h3])


@pytest.fixture(scope="module")
def ctx():
    c = vm.FMM(0)
    yield c
    c.close()


def test_noalloc_diagnostics_matches_allocating_entry_point(ctx):
    g = torch.Generator(device="cpu").manual_seed(11)
    h3 = 0.37 ** 3
    # 300 000 particles use the full 1024-block grid; 1000 use 4 blocks, so the
    # second call reads fewer slots than the first call wrote
    for n in (300_000, 1000):
        u = torch.randn(3, n, generator=g, dtype=torch.float64).cuda()
        J = torch.randn(9, n, generator=g, dtype=torch.float64).cuda()
        a = torch.randn(3, n, generator=g, dtype=torch.float64).cuda()
        out = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.diagnostics_noalloc(u, J, a, h3, out)
        ref = ctx.diagnostics(u, J, a, h3)
        torch.cuda.synchronize()
        got, want = out.cpu().numpy(), ref.cpu().numpy()
        print(f"[no-alloc] n={n} got {got} want {want}", flush=True)
        assert np.array_equal(got, want), (n, got, want)
        host = _host_sums(u, J, a, h3)
        assert np.allclose(got, host, rtol=1e-12, atol=0.0), (n, got, host)
        # optional inputs absent: zeros in their slots, as vm_diagnostics
        out2 = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.diagnostics_noalloc(u, None, None, h3, out2)
        ref2 = ctx.diagnostics(u, None, None, h3)
        torch.cuda.synchronize()
        assert np.array_equal(out2.cpu().numpy(), ref2.cpu().numpy())
        assert out2[1].item() == 0.0 and out2[2].item() == 0.0


def test_noalloc_diagnostics_rejects_bad_arguments(ctx):
    u = torch.zeros(3, 4, dtype=torch.float64, device="cuda")
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(vm._lib.VmError):
        ctx.diagnostics_noalloc(u, None, None, 0.0, out)
