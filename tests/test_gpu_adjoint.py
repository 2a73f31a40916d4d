"""GPU checks of the adjoint FMM, the Heun step and the diagnostics.

Tolerances:
* dot-product test <u_bar, B alpha> = <B^T u_bar, alpha> (u is linear in alpha): 1e-12 relative;
* central finite differences (FP64, 32 particles, random directions) of
  L = h^3/2 sum |u|^2, per directional derivative: 1e-6 relative plus a noise floor.
  Moving one particle re-rounds every particle's far field (~1e-15 each), so the
  difference quotient carries ~sqrt(N) 1e-15 h^3 / eps of noise: ~4e-9 at eps = 1e-6
  (floor 1e-8 max|grad|), ~4e-10 at eps = 1e-5 (floor 2e-9 max|grad|); the FD
  truncation (eps^2) stays below both;
* direct-sum reference gradient (exact kernel, images S_1) at N = 4096:
    dL/dalpha_k = h^3 v_k,  dL/dx_k = h^3 (J_k u_k + J^v_k alpha_k)
  with v, J^v the field and gradient of strengths u: 1e-4 (FMM truncation at p = 10);
* FP32 adjoint vs FP64 adjoint: 1e-4;
* the 64^3 backward case at its full size: central differences (eps = 1e-6) on 32
  particles and 8 strengths, floor 2e-7 max|grad| (the noise grows like sqrt(N));
* Heun step against the same step built from the oracle FMM: 1e-10.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import direct as D
from oracle import fmm as OF
from oracle import tree as T

pytestmark = pytest.mark.gpu

L = 2 * math.pi


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1110_2921_amd as vm
    return vm.FMM(0)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float64).T)).cuda()


def _host(t):
    return t.cpu().numpy().T


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASE = dict(ng=16, k0=4.0, seed=31, p=8, level=2, K=3)


def _case():
    x, a = W.random_field(CASE["ng"], CASE["k0"], CASE["seed"])
    h = L / CASE["ng"]
    return x, a, h


def _loss(ctx, x, a, h, precision="fp64", K=None):
    import torch
    u, _, _ = ctx.eval(_dev(x), _dev(a), h, CASE["p"], CASE["level"], periodic=CASE["K"] if K is None else K,
                       precision=precision, want_dalpha=False)
    torch.cuda.synchronize()
    u = _host(u)
    return 0.5 * h ** 3 * np.sum(u * u), u


def test_dot_product_identity(ctx):
    x, a, h = _case()
    rng = np.random.default_rng(1)
    ubar = rng.standard_normal(x.shape)
    _, u = _loss(ctx, x, a, h)
    _, ab = ctx.adjoint(_dev(x), _dev(a), _dev(ubar), h, CASE["p"], CASE["level"], periodic=CASE["K"],
                        want_x=False)
    lhs = np.sum(ubar * u)
    rhs = np.sum(_host(ab) * a)
    assert abs(lhs - rhs) < 1e-12 * np.sum(np.abs(ubar * u))


def _fd(ctx, x, a, h, xp, xm, ap, am, eps):
    """Central difference of L = h^3/2 sum |u|^2, formed as h^3/2 sum (u+ - u-).(u+ + u-)
    (the same number as L+ - L-, without cancelling the ~10^2-sized L)."""
    _, up = _loss(ctx, xp, ap, h)
    _, um = _loss(ctx, xm, am, h)
    return 0.5 * h ** 3 * np.sum((up - um) * (up + um)) / (2 * eps)


@pytest.mark.parametrize("eps,floor", [(1e-6, 1e-8), (1e-5, 2e-9)])
def test_finite_differences(ctx, eps, floor):
    x, a, h = _case()
    _, u = _loss(ctx, x, a, h)
    xb, ab = ctx.adjoint(_dev(x), _dev(a), _dev(h ** 3 * u), h, CASE["p"], CASE["level"], periodic=CASE["K"])
    xb, ab = _host(xb), _host(ab)
    rng = np.random.default_rng(2)
    for k in rng.choice(len(x), 32, replace=False):
        e = rng.standard_normal(3)
        e /= np.linalg.norm(e)
        xp, xm = x.copy(), x.copy()
        xp[k] += eps * e
        xm[k] -= eps * e
        fd = _fd(ctx, x, a, h, xp, xm, a, a, eps)
        an = float(xb[k] @ e)
        assert abs(fd - an) < 1e-6 * abs(an) + floor * np.abs(xb).max(), (k, fd, an)
    for k in rng.choice(len(x), 8, replace=False):
        e = rng.standard_normal(3)
        ap, am = a.copy(), a.copy()
        ap[k] += eps * e
        am[k] -= eps * e
        fd = _fd(ctx, x, a, h, x, x, ap, am, eps)
        an = float(ab[k] @ e)
        assert abs(fd - an) < 1e-6 * abs(an) + floor * np.abs(ab).max(), (k, fd, an)


def test_direct_sum_reference_gradient(ctx):
    x, a = W.random_field(16, 4.0, 37)
    h = L / 16
    K, p, level = 1, 10, 2
    tr = T.build(x, (0, 0, 0), L, level, 1)
    xw = tr["xw"]
    u, J = D.direct(xw, xw, a, h, L, K=K)
    v, Jv = D.direct(xw, xw, h ** 3 * u, h, L, K=K)
    ab_ref = v
    xb_ref = h ** 3 * (np.einsum("iab,ib->ia", J, u) + np.einsum("iab,ib->ia", Jv / h ** 3, a))
    import torch
    ug, _, _ = ctx.eval(_dev(x), _dev(a), h, p, level, periodic=K, want_dalpha=False)
    torch.cuda.synchronize()
    xb, ab = ctx.adjoint(_dev(x), _dev(a), h ** 3 * ug, h, p, level, periodic=K)
    assert rel(_host(ab), ab_ref) < 1e-4
    assert rel(_host(xb), xb_ref) < 1e-4


def test_mixed_adjoint_matches_fp64(ctx):
    x, a, h = _case()
    _, u = _loss(ctx, x, a, h)
    ub = _dev(h ** 3 * u)
    args = (h, CASE["p"], CASE["level"])
    xb, ab = ctx.adjoint(_dev(x), _dev(a), ub, *args, periodic=CASE["K"])
    xm, am = ctx.adjoint(_dev(x), _dev(a), ub, *args, periodic=CASE["K"], precision="mixed")
    assert rel(_host(am), _host(ab)) < 1e-4
    assert rel(_host(xm), _host(xb)) < 1e-4


def test_autograd_function(ctx):
    import torch
    import paper_1110_2921_amd as vm
    x, a, h = _case()
    xt = _dev(x).requires_grad_(True)
    at = _dev(a).requires_grad_(True)
    u = vm.velocity(xt, at, ctx, h, CASE["p"], CASE["level"], periodic=CASE["K"])
    loss = 0.5 * h ** 3 * (u * u).sum()
    gx, ga = torch.autograd.grad(loss, (xt, at))
    xb, ab = ctx.adjoint(_dev(x), _dev(a), (h ** 3 * u).detach(), h, CASE["p"], CASE["level"],
                         periodic=CASE["K"])
    assert torch.equal(gx, xb) and torch.equal(ga, ab)


def test_heun_step_matches_oracle(ctx):
    import torch
    x, a = W.random_field(8, 2.0, 41)
    h = L / 8
    p, level, K, dt = 6, 1, 3, 0.05
    xt, at = _dev(x), _dev(a)
    ctx.rk2_step(xt, at, h, p, level, dt, periodic=K)
    torch.cuda.synchronize()

    def rates(xx, aa):
        u, J = OF.fmm(xx, aa, h, p, level, periodic=K)
        return u, D.stretching(J, aa)

    u1, s1 = rates(x, a)
    u2, s2 = rates(x + dt * u1, a + dt * s1)
    x1 = T.wrap(x + 0.5 * dt * u1 + 0.5 * dt * u2, (0, 0, 0), L)
    a1 = a + 0.5 * dt * s1 + 0.5 * dt * s2
    assert rel(_host(xt), x1) < 1e-10
    assert rel(_host(at), a1) < 1e-10


def test_diagnostics(ctx):
    import torch
    x, a, h = _case()
    u, _, J = ctx.eval(_dev(x), _dev(a), h, 6, 2, periodic=3, want_grad=True)
    d = ctx.diagnostics(u, J, _dev(a), h ** 3).cpu().numpy()
    un, Jn = _host(u), _host(J).reshape(-1, 3, 3)
    w = np.stack([Jn[:, 1, 2] - Jn[:, 2, 1], Jn[:, 2, 0] - Jn[:, 0, 2], Jn[:, 0, 1] - Jn[:, 1, 0]], 1)
    ref = [0.5 * h ** 3 * np.sum(un * un), 0.5 * h ** 3 * np.sum(w * w), 0.5 * np.sum(a * a) / h ** 3]
    assert np.allclose(d, ref, rtol=1e-13, atol=0)
    d2 = ctx.diagnostics(u, J, _dev(a), h ** 3).cpu().numpy()
    assert np.array_equal(d, d2)


@pytest.mark.parametrize("precision", ["fp64"])
def test_backward_case_at_full_size(ctx, precision):
    """The 64^3 backward case (p = 8, level 4, 27^3 images): central differences
    with eps = 1e-6 on 32 random particles (positions, random directions) and on
    8 strengths.  Moving one particle re-rounds all N far fields, so the noise
    floor grows like sqrt(N) against the 16^3 case: 2e-7 max|grad| at eps = 1e-6.
    The FP32 adjoint matches the FP64 one to 1e-4."""
    import torch
    w = W.WORKLOADS["rand64_periodic"]
    x, a = W.make(w)
    h = w.h
    eps, floor = 1e-6, 2e-7
    kw = dict(periodic=w.periodic, box_len=w.box_len)

    def loss_u(xx, aa):
        u, _, _ = ctx.eval(_dev(xx), _dev(aa), w.sigma, w.p, w.level, precision="fp64", want_dalpha=False, **kw)
        torch.cuda.synchronize()
        return _host(u)

    u = loss_u(x, a)
    ub = _dev(h ** 3 * u)
    xb, ab = ctx.adjoint(_dev(x), _dev(a), ub, w.sigma, w.p, w.level, precision="fp64", **kw)
    xb, ab = _host(xb), _host(ab)
    rng = np.random.default_rng(5)

    def fd(xp, xm, ap, am):
        up, um = loss_u(xp, ap), loss_u(xm, am)
        return 0.5 * h ** 3 * np.sum((up - um) * (up + um)) / (2 * eps)

    for k in rng.choice(w.n, 32, replace=False):
        e = rng.standard_normal(3)
        e /= np.linalg.norm(e)
        xp, xm = x.copy(), x.copy()
        xp[k] += eps * e
        xm[k] -= eps * e
        an = float(xb[k] @ e)
        assert abs(fd(xp, xm, a, a) - an) < 1e-6 * abs(an) + floor * np.abs(xb).max(), k
    for k in rng.choice(w.n, 8, replace=False):
        e = rng.standard_normal(3)
        ap, am = a.copy(), a.copy()
        ap[k] += eps * e
        am[k] -= eps * e
        an = float(ab[k] @ e)
        assert abs(fd(x, x, ap, am) - an) < 1e-6 * abs(an) + floor * np.abs(ab).max(), k
    xm32, am32 = ctx.adjoint(_dev(x), _dev(a), ub, w.sigma, w.p, w.level, precision="mixed", **kw)
    assert rel(_host(am32), ab) < 1e-4
    assert rel(_host(xm32), xb) < 1e-4


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adjoint_reuse_matches_recompute(ctx, precision):
    """vm_fmm_adjoint_reuse takes the tree and gradient of the context's last
    evaluation and gives vm_fmm_adjoint's result bit for bit; a stale call is
    rejected before anything runs."""
    import torch
    import paper_1110_2921_amd as vm
    x, a, h = _case()
    xt, at = _dev(x), _dev(a)
    kw = dict(periodic=CASE["K"], precision=precision)
    ub = _dev(np.random.default_rng(91).standard_normal(a.shape))
    u, _, J = ctx.eval(xt, at, h, CASE["p"], CASE["level"], want_grad=True, want_dalpha=False, **kw)
    xr, ar = ctx.adjoint(xt, at, ub, h, CASE["p"], CASE["level"], grad=J, **kw)
    xr2, ar2 = ctx.adjoint(xt, at, ub, h, CASE["p"], CASE["level"], grad=J, **kw)   # again, same evaluation
    xf, af = ctx.adjoint(xt, at, ub, h, CASE["p"], CASE["level"], **kw)
    assert torch.equal(xr, xf) and torch.equal(ar, af)
    assert torch.equal(xr2, xf) and torch.equal(ar2, af)
    # the recomputing call above rebuilt the tree, and another evaluation or tree
    # build in between invalidates the reuse
    ctx.eval(xt, at, h, CASE["p"], CASE["level"], want_grad=True, want_dalpha=False, **kw)
    ctx.gauss_sum(xt, at, h, CASE["level"], periodic=CASE["K"])
    with pytest.raises(vm._lib.VmError):
        ctx.adjoint(xt, at, ub, h, CASE["p"], CASE["level"], grad=J, **kw)
    a2 = at.clone()
    ctx.eval(a2, at, h, CASE["p"], CASE["level"], want_grad=True, want_dalpha=False, **kw)
    with pytest.raises(vm._lib.VmError):
        ctx.adjoint(xt, at, ub, h, CASE["p"], CASE["level"], grad=J, **kw)


def test_autograd_falls_back_when_the_context_moved_on(ctx):
    """The backward pass reuses the forward evaluation when nothing ran in
    between, and recomputes it otherwise: both give the adjoint's gradient."""
    import torch
    import paper_1110_2921_amd as vm
    x, a, h = _case()
    xt = _dev(x).requires_grad_(True)
    at = _dev(a).requires_grad_(True)
    u = vm.velocity(xt, at, ctx, h, CASE["p"], CASE["level"], periodic=CASE["K"])
    ctx.eval(_dev(x + 0.01), _dev(a), h, CASE["p"], CASE["level"], periodic=CASE["K"])   # something else
    loss = 0.5 * h ** 3 * (u * u).sum()
    gx, ga = torch.autograd.grad(loss, (xt, at))
    xb, ab = ctx.adjoint(_dev(x), _dev(a), (h ** 3 * u).detach(), h, CASE["p"], CASE["level"],
                         periodic=CASE["K"])
    assert torch.equal(gx, xb) and torch.equal(ga, ab)


def test_autograd_with_row_major_inputs_and_an_eval_in_between(ctx):
    """(n, 3) inputs are copied into SoA tensors for the library.  The forward
    pass keeps those copies, so the temporaries of a later evaluation of the
    same size cannot take their addresses and pass the library's reuse check:
    the backward pass must recompute and give vm_fmm_adjoint's gradient bit for
    bit, in the (n, 3) layout of the inputs.  Keyword arguments that only the
    evaluation takes (check_domain) do not reach the adjoint."""
    import torch
    import paper_1110_2921_amd as vm
    x, a, h = _case()
    args = (h, CASE["p"], CASE["level"])
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda().requires_grad_(True)
    at = torch.from_numpy(np.ascontiguousarray(a)).cuda().requires_grad_(True)
    u = vm.velocity(xt, at, ctx, *args, periodic=CASE["K"], check_domain=True)
    u2 = vm.velocity(xt.detach(), at.detach(), ctx, *args, periodic=CASE["K"])   # reuses nothing of u
    ctx.eval(torch.from_numpy(np.ascontiguousarray(x + 0.01)).cuda(),
             torch.from_numpy(np.ascontiguousarray(a[::-1])).cuda(), *args, periodic=CASE["K"])
    loss = 0.5 * h ** 3 * (u * u).sum()
    gx, ga = torch.autograd.grad(loss, (xt, at))
    assert gx.shape == xt.shape and ga.shape == at.shape
    xb, ab = ctx.adjoint(_dev(x), _dev(a), (h ** 3 * u).detach(), *args, periodic=CASE["K"])
    assert torch.equal(gx, xb.t()) and torch.equal(ga, ab.t())
    assert torch.equal(u2, u.detach())


def test_velocity_rejects_output_keywords(ctx):
    import paper_1110_2921_amd as vm
    x, a, h = _case()
    with pytest.raises(TypeError):
        vm.velocity(_dev(x), _dev(a), ctx, h, CASE["p"], CASE["level"], want_grad=True)


@pytest.mark.parametrize("precision,K", [("fp64", 3), ("fp64", 0), ("mixed", 3), ("mixed", 0)])
def test_orbit_m2l_adjoint_is_the_transpose(ctx, precision, K):
    """p = 10 at level 4: the forward and the adjoint M2L both run by reflection
    orbits (the adjoint with the transposed operators of the negated offsets),
    so the alpha-adjoint satisfies <u_bar, u(alpha)> = <alpha_bar(u_bar), alpha>
    to round-off (FP64: 1e-12, mixed: 1e-5 of sum |u_bar u|), periodic and free."""
    import torch
    x, a = W.random_field(24, 4.0, 77 + K)
    h = L / 24
    rng = np.random.default_rng(5 + K)
    ubar = rng.standard_normal(x.shape)
    u, _, _ = ctx.eval(_dev(x), _dev(a), h, 10, 4, periodic=K, precision=precision, want_dalpha=False)
    torch.cuda.synchronize()
    u = _host(u)
    _, ab = ctx.adjoint(_dev(x), _dev(a), _dev(ubar), h, 10, 4, periodic=K, precision=precision, want_x=False)
    lhs = np.sum(ubar * u)
    rhs = np.sum(_host(ab) * a)
    tol = 1e-12 if precision == "fp64" else 1e-5
    print(f"[orbit-adjoint] {precision} K={K}: {abs(lhs - rhs) / np.sum(np.abs(ubar * u)):.2e}", flush=True)
    assert abs(lhs - rhs) < tol * np.sum(np.abs(ubar * u))
