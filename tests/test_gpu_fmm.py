"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances (relative L2 over all particles, and the worst particle's error
over the largest reference magnitude, as ``_gates`` defines them):
* tree arrays (keys, sorted order, leaf ranges): bit-exact;
* FP64 FMM vs the oracle FMM of the same definition: 1e-10 in both measures
  (round-off apart: same tree, lists, truncation and lattice construction);
* no far field (one leaf, free space): FP64 vs the direct sum 1e-13;
* mixed (FP32 near field + FP32 MFMA expansions) vs FP64: 1e-5 / 4e-5 for u,
  1e-4 / 4e-4 for dalpha/dt and J;
* compensated near-field sums: same-sign velocity terms summed over 16368
  sources, mixed vs the FP64 direct sum within 1e-6, where plain FP32
  accumulation in the same order (emulated on the CPU) is off by more than 2e-6.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import direct as D
from oracle import fmm as OF
from oracle import tree as T
from _gates import FP64, MIXED_J, MIXED_U, close, rel

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


def _run(ctx, x, a, sigma, p, level, periodic, precision="fp64", scheme="classic", lo=(0, 0, 0)):
    import torch
    u, da, J = ctx.eval(_dev(x), _dev(a), sigma, p, level, periodic=periodic, box_lo=lo,
                        precision=precision, scheme=scheme, want_grad=True)
    torch.cuda.synchronize()
    return u.cpu().numpy().T, da.cpu().numpy().T, J.cpu().numpy().T.reshape(-1, 3, 3)


def _host(t):
    return t.cpu().numpy().T


@pytest.mark.parametrize("periodic", [0, 1])
@pytest.mark.parametrize("level", [1, 2, 3, 5])
def test_tree_is_bit_exact(ctx, periodic, level):
    x, a = W.random_particles(5000, 100 + level)
    if periodic:
        x[:50] += np.array([L, -L, 3 * L])          # outside the box: wrapped
        x[50] = [0.0, L, np.nextafter(0.0, -1.0)]    # faces
    else:
        x[50] = [0.0, np.nextafter(L, 0), L]
    lat = W.lattice(16)                              # particles on cell-centre planes
    x = np.concatenate([x, lat])
    a = np.concatenate([a, np.ones_like(lat)])
    _run(ctx, x, a, 0.1, 2, level, periodic)
    keys, perm, start = ctx.debug_tree(len(x), level)
    ref = T.build(x, (0, 0, 0), L, level, periodic)
    assert np.array_equal(perm, ref["perm"])
    assert np.array_equal(keys, ref["keys"][ref["perm"]])
    assert np.array_equal(start, np.append(ref["start"], len(x)))


def test_level0_free_space_is_direct_sum(ctx):
    x, a = W.random_particles(2048, 7)
    sigma = 0.2
    u, da, J = _run(ctx, x, a, sigma, 4, 0, 0)
    u0, J0 = D.direct(x, x, a, sigma)
    close(u, u0, (1e-13, 1e-13), "u vs u0")
    close(J, J0, (1e-13, 1e-13), "J vs J0")
    close(da, D.stretching(J0, a), (1e-13, 1e-13), "dalpha/dt vs direct")


def test_taylor_green_free_space_matches_oracle(ctx):
    w = W.WORKLOADS["tg16_free"]
    x, a = W.make(w)
    u, da, J = _run(ctx, x, a, w.sigma, w.p, w.level, 0)
    uo, Jo = OF.fmm(x, a, w.sigma, w.p, w.level, periodic=0)
    close(u, uo, FP64, "u vs uo")
    close(J, Jo, FP64, "J vs Jo")
    close(da, D.stretching(Jo, a), FP64, "dalpha/dt vs oracle")
    # and it is close to the exact direct sum (p = 6 truncation)
    ud, Jd = D.direct(x, x, a, w.sigma)
    assert rel(u, ud) < 1e-3


@pytest.mark.parametrize("K", [1, 3])
def test_periodic_fp64_matches_oracle(ctx, K):
    x, a = W.random_field(16, 4.0, 17)
    h = L / 16
    u, da, J = _run(ctx, x, a, h, 8, 2, K)
    uo, Jo = OF.fmm(x, a, h, 8, 2, periodic=K)
    close(u, uo, FP64, "u vs uo")
    close(J, Jo, FP64, "J vs Jo")


def test_rand32_periodic_matches_oracle(ctx):
    w = W.WORKLOADS["rand32_periodic"]
    x, a = W.make(w)
    u, da, J = _run(ctx, x, a, w.sigma, w.p, w.level, w.periodic)
    uo, Jo = OF.fmm(x, a, w.sigma, w.p, w.level, periodic=w.periodic)
    close(u, uo, FP64, "u vs uo")
    close(J, Jo, FP64, "J vs Jo")
    close(da, D.stretching(Jo, a), FP64, "dalpha/dt vs oracle")
    um, dam, Jm = _run(ctx, x, a, w.sigma, w.p, w.level, w.periodic, precision="mixed")
    close(um, u, MIXED_U, "um vs u")
    close(dam, da, MIXED_J, "dam vs da")
    close(Jm, J, MIXED_J, "Jm vs J")


# leaf populations around the kernel's block boundaries: empty, a few (lane groups
# of 1..32), one full block of 64 and partial second blocks of both forms
COUNTS = [0, 1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 31, 32, 33, 47, 63, 64, 65, 66, 80, 95, 96, 97,
          127, 128, 129, 150, 6, 40, 70, 100]


@pytest.mark.parametrize("periodic", [0, 3])
def test_uneven_leaf_populations(ctx, periodic):
    level = 2
    counts = [COUNTS[i % len(COUNTS)] for i in range(8 ** level)]
    x, a = W.particles_with_leaf_counts(counts, level, seed=61)
    sigma, p = 0.15, 6
    u, da, J = _run(ctx, x, a, sigma, p, level, periodic)
    uo, Jo = OF.fmm(x, a, sigma, p, level, periodic=periodic)
    close(u, uo, FP64, "u vs uo")
    close(J, Jo, FP64, "J vs Jo")
    close(da, D.stretching(Jo, a), FP64, "dalpha/dt vs oracle")
    um, dam, Jm = _run(ctx, x, a, sigma, p, level, periodic, precision="mixed")
    close(um, u, MIXED_U, "um vs u")
    close(Jm, J, MIXED_J, "Jm vs J")
    close(dam, da, MIXED_J, "dam vs da")


def test_compensated_near_field_sums(ctx):
    """One leaf (level 0, free space): 16 targets with no strength at x ~ 1 and
    16368 sources with equal strengths along z at x in [2, 5].  Every term of
    u_y at a target has the same sign, so plain FP32 accumulation drifts like
    sqrt(n) ulp of the running sum (emulated on the CPU in the kernel's order:
    more than 2e-6 off at one of the targets); the compensated sums stay within
    1e-6 of the FP64 direct sum."""
    from scipy.special import erf
    rng = np.random.default_rng(71)
    n = 16384
    ns = n - 16
    xs = np.stack([rng.uniform(2.0, 5.0, ns), rng.uniform(2.0, 4.0, ns), rng.uniform(2.0, 4.0, ns)], 1)
    xt = np.stack([rng.uniform(1.0, 1.1, 16), rng.uniform(2.9, 3.1, 16), rng.uniform(2.9, 3.1, 16)], 1)
    x = np.concatenate([xt, xs])
    a = np.zeros((n, 3))
    a[16:, 2] = 1e-3
    sigma = 0.05
    t = np.arange(16)
    um, _, _ = _run(ctx, x, a, sigma, 4, 0, 0, precision="mixed")
    ud, _ = D.direct(x[t], x, a, sigma)
    err = np.abs(um[t, 1] - ud[:, 1]) / np.abs(ud[:, 1])
    assert err.max() < 1e-6, err.max()
    naive = []
    for i in t:
        r = (x[i] - x).astype(np.float32)
        r2 = np.sum(r.astype(np.float64) ** 2, axis=1)
        rr = np.sqrt(r2)
        rho = rr / sigma
        g = erf(rho / math.sqrt(2)) - math.sqrt(2 / math.pi) * rho * np.exp(-0.5 * rho * rho)
        q = np.where(rr > 0, g / np.maximum(r2 * rr, 1e-300), 0.0)
        terms = (q * a[:, 2] * r[:, 0] / (4 * math.pi)).astype(np.float32)   # (alpha x r)_y = alpha_z r_x
        naive.append(np.add.accumulate(terms, dtype=np.float32)[-1])
    nerr = np.abs(np.array(naive, np.float64) - ud[:, 1]) / np.abs(ud[:, 1])
    assert nerr.max() > 2e-6, nerr.max()


@pytest.mark.parametrize("periodic", [0, 2])
def test_largest_degree(ctx, periodic):
    """p = 18, the largest degree (single-buffered translation tiles, 7 P2M
    order ranges, the widest L2P tables): against the direct sum with the
    far-field model (g = 1 beyond adjacent leaves), to which the FMM converges
    as p grows.  FP64 at p = 18 within 3e-7 (u) and 5e-7 (J) of it (measured
    free space u 1.0e-7, periodic K = 2 u 1.6e-7 and J 3.2e-7: what is left of
    the truncation, largest in the lattice ring of S_2 whose images sit
    closest to the root cell) and at least 10x closer than at p = 12; mixed
    within the usual gates of FP64."""
    x, a = W.random_particles(3000, 43)
    sigma, level = 0.15, 2
    tr = T.build(x, (0, 0, 0), L, level, periodic)
    c = tr["coords"]            # input order, as xw
    ud, Jd = D.direct(tr["xw"], tr["xw"], a, sigma, L, K=periodic, cells_t=c, cells_s=c, level=level)
    u12, _, J12 = _run(ctx, x, a, sigma, 12, level, periodic)
    u, _, J = _run(ctx, x, a, sigma, 18, level, periodic)
    print(f"[parity] p=18 vs model: u {rel(u, ud):.2e} J {rel(J, Jd):.2e}; p=12: u {rel(u12, ud):.2e}")
    assert rel(u, ud) < 3e-7 and rel(J, Jd) < 5e-7
    assert rel(u, ud) < rel(u12, ud) / 10 and rel(J, Jd) < rel(J12, Jd) / 10
    um, _, Jm = _run(ctx, x, a, sigma, 18, level, periodic, precision="mixed")
    close(um, u, MIXED_U, "um vs u")
    close(Jm, J, MIXED_J, "Jm vs J")


def test_transpose_scheme_conserves_vorticity(ctx):
    x, a = W.random_field(16, 4.0, 23)
    h = L / 16
    _, da, _ = _run(ctx, x, a, h, 10, 2, 3, scheme="transpose")
    _, dc, J = _run(ctx, x, a, h, 10, 2, 3, scheme="classic")
    tot = np.abs(da.sum(axis=0)).max() / np.abs(da).sum()
    assert tot < 1e-6
    assert np.abs(dc.sum(axis=0)).max() / np.abs(dc).sum() > 10 * tot
    assert rel(da, D.stretching(J, a, "transpose")) < 1e-14


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_runs_are_bitwise_reproducible(ctx, precision):
    x, a = W.random_field(16, 4.0, 29)
    h = L / 16
    r1 = _run(ctx, x, a, h, 6, 2, 3, precision=precision)
    r2 = _run(ctx, x, a, h, 6, 2, 3, precision=precision)
    for p, q in zip(r1, r2):
        assert np.array_equal(p, q)


def test_invalid_arguments_are_rejected(ctx):
    import paper_1110_2921_amd as vm
    x, a = W.random_particles(64, 3)
    for kw in (dict(p=0), dict(p=19), dict(level=11), dict(periodic=5)):
        args = dict(p=4, level=1, periodic=0)
        args.update(kw)
        with pytest.raises(vm._lib.VmError) as e:
            ctx.eval(_dev(x), _dev(a), 0.1, args["p"], args["level"], periodic=args["periodic"])
        assert e.value.status == vm._lib.VM_EINVAL
    with pytest.raises(vm._lib.VmError) as e:
        ctx.eval(_dev(x), _dev(a), -1.0, 4, 1)
    assert e.value.status == vm._lib.VM_EINVAL
    xb = x.copy()
    xb[3, 0] = 2 * L
    with pytest.raises(vm._lib.VmError) as e:
        ctx.eval(_dev(xb), _dev(a), 0.1, 4, 2, check_domain=True)
    assert e.value.status == vm._lib.VM_EDOMAIN


def test_one_particle_and_the_empty_set(ctx):
    """No particles: VM_EINVAL.  One particle: in free space no velocity at
    all (the self pair has r = 0) and the gradient is the self term; with the
    images of S_1, the oracle FMM's velocity and gradient."""
    import paper_1110_2921_amd as vm
    x = np.array([[1.1, 2.3, 4.0]])
    a = np.array([[0.3, -0.2, 0.5]])
    with pytest.raises(vm._lib.VmError) as e:
        ctx.eval(_dev(x[:0]), _dev(a[:0]), 0.2, 6, 2)
    assert e.value.status == vm._lib.VM_EINVAL
    for K in (0, 1):
        uo, Jo = OF.fmm(x, a, 0.2, 6, 2, periodic=K)
        print(f"[fmm] one particle, periodic {K}", flush=True)
        u, _, J = ctx.eval(_dev(x), _dev(a), 0.2, 6, 2, periodic=K, want_grad=True)
        um, _, Jm = ctx.eval(_dev(x), _dev(a), 0.2, 6, 2, periodic=K, want_grad=True, precision="mixed")
        u, J, um, Jm = _host(u), _host(J).reshape(-1, 3, 3), _host(um), _host(Jm).reshape(-1, 3, 3)
        close(J, Jo, FP64, "J vs oracle")
        close(Jm, J, MIXED_J, "J mixed vs fp64")
        if K == 0:
            assert np.all(u == 0.0) and np.all(um == 0.0)
        else:
            assert np.abs(u - uo).max() < 1e-13 * np.abs(Jo).max()


@pytest.mark.parametrize("periodic", [0, 2])
def test_coincident_particles(ctx, periodic):
    """Particles at the same position (40 pairs, different strengths): each
    such pair is a pair at r = 0, summed like the self term (the small-r
    series); FP64 against the oracle FMM, mixed against FP64."""
    x, a = W.random_particles(300, 77)
    x = np.concatenate([x, x[:40]])
    a = np.concatenate([a, a[40:80]])
    uo, Jo = OF.fmm(x, a, 0.2, 8, 2, periodic=periodic)
    print(f"[fmm] coincident particles, periodic {periodic}", flush=True)
    u, _, J = ctx.eval(_dev(x), _dev(a), 0.2, 8, 2, periodic=periodic, want_grad=True)
    um, _, Jm = ctx.eval(_dev(x), _dev(a), 0.2, 8, 2, periodic=periodic, want_grad=True, precision="mixed")
    u, J = _host(u), _host(J).reshape(-1, 3, 3)
    close(u, uo, FP64, "u vs oracle")
    close(J, Jo, FP64, "J vs oracle")
    close(_host(um), u, MIXED_U, "u mixed vs fp64")
    close(_host(Jm).reshape(-1, 3, 3), J, MIXED_J, "J mixed vs fp64")


@pytest.mark.parametrize("p", [6, 8, 10])
def test_triangular_truncation_matches_oracle(ctx, p):
    """M2L truncated to n + n' <= p: FP64 against the oracle with the same
    truncation (1e-10); the mixed form (whose operator-stationary M2L skips
    the zero tiles, three kernel shapes for p = 6, 8, 10) against FP64 within
    the usual 1e-5 / 1e-4."""
    x, a = W.random_field(16, 4.0, 61)
    h = L / 16
    kw = dict(periodic=3, want_grad=True, truncation="triangular")
    u, da, J = ctx.eval(_dev(x), _dev(a), h, p, 2, **kw)
    uo, Jo = OF.fmm(x, a, h, p, 2, periodic=3, truncation="triangular")
    u, J = _host(u), _host(J).reshape(-1, 3, 3)
    close(u, uo, FP64, "u vs uo")
    close(J, Jo, FP64, "J vs Jo")
    um, _, Jm = ctx.eval(_dev(x), _dev(a), h, p, 2, precision="mixed", **kw)
    close(_host(um), u, MIXED_U, "um vs u")
    close(_host(Jm).reshape(-1, 3, 3), J, MIXED_J, "Jm vs J")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_triangular_adjoint_is_the_transpose(ctx, precision):
    """u is linear in alpha, so <u_bar, u(alpha)> = <alpha_bar(u_bar), alpha> for
    the discrete adjoint of the truncated FMM (FP64 to round-off; mixed within
    its 1e-5)."""
    import torch
    x, a = W.random_field(16, 4.0, 62)
    h = L / 16
    ub = np.random.default_rng(63).standard_normal(a.shape)
    u, _, _ = ctx.eval(_dev(x), _dev(a), h, 8, 2, periodic=3, precision=precision, truncation="triangular")
    _, ab = ctx.adjoint(_dev(x), _dev(a), _dev(ub), h, 8, 2, periodic=3, precision=precision,
                        want_x=False, truncation="triangular")
    lhs = float(np.sum(ub * _host(u)))
    rhs = float(np.sum(_host(ab) * a))
    assert abs(lhs - rhs) < (1e-12 if precision == "fp64" else 1e-5) * abs(lhs)


def test_level_tuning(ctx):
    """The tuner tries the finest level with leaves >= 4 sigma (and no more
    leaves than particles) and coarser ones while the time falls, and returns
    the fastest it tried; clustered particles in free space as well."""
    import paper_1110_2921_amd as vm
    w = W.WORKLOADS["rand32_periodic"]
    x, a = W.make(w)
    lv, ms = ctx.tune_level(_dev(x), _dev(a), w.sigma, w.p, periodic=w.periodic, box_len=w.box_len)
    assert max(ms) == 3 and lv in ms and ms[lv] == min(ms.values())
    rng = np.random.default_rng(81)
    xc = 2.0 + rng.uniform(0.0, 1.0, size=(20000, 3))
    ac = rng.standard_normal((20000, 3))
    lv, ms = ctx.tune_level(_dev(xc), _dev(ac), 0.05, 6, periodic=0)
    assert max(ms) == 4 and lv in ms and ms[lv] == min(ms.values())
    for kw in ({"min_leaf_sigmas": 0.0}, {"reps": 0}):
        with pytest.raises(vm._lib.VmError):
            ctx.tune_level(_dev(x), _dev(a), w.sigma, w.p, periodic=w.periodic, **kw)


@pytest.mark.parametrize("K", [2, 4])
@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_low_degrees_and_largest_image_block(ctx, p, K):
    """Degrees below the operator-stationary M2L's shapes (p <= 4 take the
    generic translation kernel in both precisions) and the 81^3 image block:
    FP64 against the oracle 1e-10, mixed against FP64 1e-5 / 1e-4."""
    x, a = W.random_field(8, 2.0, 100 + p)
    h = L / 8
    u, _, J = _run(ctx, x, a, h, p, 1, K)
    uo, Jo = OF.fmm(x, a, h, p, 1, periodic=K)
    close(u, uo, FP64, "u vs uo")
    close(J, Jo, FP64, "J vs Jo")
    um, _, Jm = _run(ctx, x, a, h, p, 1, K, precision="mixed")
    close(um, u, MIXED_U, "um vs u")
    close(Jm, J, MIXED_J, "Jm vs J")


@pytest.mark.parametrize("p", [7, 9])
def test_degrees_inside_the_operator_stationary_shapes(ctx, p):
    """p = 7 and p = 9 run the operator-stationary M2L shapes of p = 6 and
    p = 10 with more padding (p = 9: a row block of zeros, a part-empty last k
    block): FP64 against the oracle 1e-10, mixed against FP64 1e-5 / 1e-4."""
    x, a = W.random_field(16, 4.0, 120 + p)
    h = L / 16
    u, _, J = _run(ctx, x, a, h, p, 2, 3)
    uo, Jo = OF.fmm(x, a, h, p, 2, periodic=3)
    close(u, uo, FP64, "u vs uo")
    close(J, Jo, FP64, "J vs Jo")
    um, _, Jm = _run(ctx, x, a, h, p, 2, 3, precision="mixed")
    close(um, u, MIXED_U, "um vs u")
    close(Jm, J, MIXED_J, "Jm vs J")


@pytest.mark.parametrize("level,K", [(2, 3), (4, 3), (4, 0), (5, 1), (5, 0)])
def test_reflection_orbit_m2l(ctx, level, K):
    """p = 10 runs the M2L of levels >= 4 by reflection orbits (one operator
    per orbit of the interaction list applied to the Walsh-Hadamard-combined
    sources, per-octant signs, class-blocked MFMAs; FP32 with the whole orbit
    operator double-buffered in LDS, FP64 through a ring of column slices;
    level 4 split over orbit ranges, level 5 whole).  FP64 against the oracle
    at 24 sampled particles (oracle.fmm.fmm_at) at 1e-10; mixed against FP64
    at 1e-5 / 4e-5 (u) and 1e-4 / 4e-4 (J); free space (missing sources
    beyond the domain) and periodic with and without the lattice.  Level 2
    (dense operators) is held to the whole oracle FMM."""
    ng = {2: 8, 4: 24, 5: 40}[level]
    x, a = W.random_field(ng, 4.0, 300 + 10 * level + K)
    h = L / ng
    print(f"[orbit-m2l] level={level} K={K} n={len(x)}", flush=True)
    u, _, J = _run(ctx, x, a, h, 10, level, K)
    um, _, Jm = _run(ctx, x, a, h, 10, level, K, precision="mixed")
    close(um, u, MIXED_U, "um vs u")
    close(Jm, J, MIXED_J, "Jm vs J")
    if level == 2:
        uo, Jo = OF.fmm(x, a, h, 10, level, periodic=K)
        close(u, uo, FP64, "u vs uo")
        close(J, Jo, FP64, "J vs Jo")
    else:
        t = np.sort(np.random.default_rng(level + K).choice(len(x), 24, replace=False))
        uo, Jo = OF.fmm_at(x, a, h, 10, level, t, periodic=K)
        close(u[t], uo, FP64, "u vs oracle (sampled)")
        close(J[t], Jo, FP64, "J vs oracle (sampled)")


def test_reflection_orbit_m2l_at_level_7(ctx):
    """The finest level the FP32 orbit kernel takes (level 7: 2^21 target cells,
    byte offsets into the class-major multipoles near 2^32), random particles
    in free space: mixed against FP64 (whose M2L at level 7 runs the dense
    operators) at 64 sampled particles, 1e-5 / 4e-5 (u) and 1e-4 / 4e-4 (J)."""
    import torch
    x, a = W.random_particles(1 << 17, 71)
    sigma = L / 512
    t = torch.from_numpy(np.sort(np.random.default_rng(3).choice(len(x), 64, replace=False))).cuda()
    out = {}
    for prec in ("fp64", "mixed"):
        u, _, J = ctx.eval(_dev(x), _dev(a), sigma, 10, 7, periodic=0, precision=prec, want_grad=True)
        out[prec] = (u[:, t].cpu().numpy().T, J[:, t].cpu().numpy().T)
        del u, J
    torch.cuda.empty_cache()
    close(out["mixed"][0], out["fp64"][0], MIXED_U, "u mixed vs fp64, level 7")
    close(out["mixed"][1], out["fp64"][1], MIXED_J, "J mixed vs fp64, level 7")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_far_field_view_adds_up_with_the_near_field(ctx, precision):
    """vm_debug_far evaluates the last evaluation's far field again (the
    evaluation itself adds it straight into its outputs): with the near field,
    the exact kernel over the 27 neighbour leaves and their images summed by
    the oracle's direct sum, it gives the velocity and gradient returned."""
    import itertools
    level, s = 2, 4
    x, a = W.particles_with_leaf_counts([8] * 64, level, 13)
    sigma, p, n = 0.12, 6, 512
    print(f"[fmm] far-field view {precision}", flush=True)
    u, _, J = _run(ctx, x, a, sigma, p, level, periodic=1, precision=precision)
    far = ctx.debug_far(n)
    _, perm, _ = ctx.debug_tree(n, level)
    c = np.floor(x / (L / s)).astype(np.int64)
    leaf = c[:, 0] + s * (c[:, 1] + s * c[:, 2])
    un, Jn = np.zeros((n, 3)), np.zeros((n, 3, 3))
    for t in range(s ** 3):
        ti = np.nonzero(leaf == t)[0]
        tc = np.array([t % s, (t // s) % s, t // (s * s)])
        xs, as_ = [], []
        for d in itertools.product((-1, 0, 1), repeat=3):
            nc = tc + np.array(d)
            js = np.nonzero(leaf == (nc % s)[0] + s * ((nc % s)[1] + s * (nc % s)[2]))[0]
            xs.append(x[js] + (nc // s) * L)
            as_.append(a[js])
        ud, Jd = D.direct(x[ti], np.concatenate(xs), np.concatenate(as_), sigma, L, K=0)
        un[ti], Jn[ti] = ud, Jd.reshape(-1, 3, 3)
    want_u = (u - un)[perm]
    want_J = (J - Jn).reshape(n, 9)[perm]
    # mixed: the outputs carry the FP32 near field's rounding (near field
    # larger than the far one), so the gate is the mixed one on the totals
    tol = 1e-11 if precision == "fp64" else 1e-5
    assert np.max(np.abs(far[:3].T - want_u)) < tol * np.max(np.abs(u))
    assert np.max(np.abs(far[3:].T - want_J)) < 10 * tol * np.max(np.abs(J))
