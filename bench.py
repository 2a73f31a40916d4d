"""Throughput of the FMM vortex-particle step on one MI355X.

A step is one Heun (RK2) step of the convection and stretching ODEs over
N = 256^3 vortex particles of a seeded random isotropic field (p = 10, leaf
level 6, 27^3 periodic images), inputs resident in HBM: two full FMM
evaluations of the regularised Biot-Savart velocity, its gradient and the
stretching term (tree build, P2M, M2M, lattice, L2L/M2L, L2P, P2P, combine)
and the update.  ``value`` counts evaluations per second (two per step).
Prints one JSON line: the headline fields, the roofline of the dominant
kernel (M2L or P2P) and of the others, the FP64 comparison, the adjoint, the
RBF interpolation of the initial lattice, the paper's time loop (Euler, core
spreading, reinitialisation every 10 steps) and the CPU oracle's rate on a
bounded sample.

    python bench.py [--steps K] [--warmup W] [--precision mixed|fp64]
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published peaks
    "hbm_gbs": 8000.0,
    "mfma_f32_tflops": 157.3,
    "mfma_f64_tflops": 78.6,
    "valu_f32_tflops": 157.3,
    "valu_f64_tflops": 78.6,
}
# Algorithmic work per unit, FMA = 2 flop:
P2P_FLOP_PER_PAIR = {"mixed": 79.0, "fp64": 69.0}   # counted from the pair kernels
# Gaussian sum: r = t - s (3), |r|^2 (5), scale (1), exp2 (1), three strength FMAs (6)
GAUSS_FLOP_PER_PAIR = 16.0
# The paper's base run (Sec. 4.1): time step (forward Euler in its loop),
# reinitialisation every 10 steps, Krylov drop tolerance
PAPER_DT = 0.005
PAPER_REINIT_EVERY = 10
PAPER_TOL = 1e-3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _sym_class(i):
    """Reflection class of the real coefficient at standard index i (bit a: sign
    -1 under the reflection of axis a)."""
    n = int(math.isqrt(i))
    r = i - n * n
    m, im = (r + 1) // 2, int(r > 0 and r % 2 == 0)
    return ((m & 1) ^ im) | (im << 1) | (((n + m) & 1) << 2)


def orbit_m2l_flop_per_target(p):
    """Flops of the orbit-form M2L per target cell (3 components, FMA = 2): per
    orbit of the octant-0 list, the class blocks (a, b) that survive its zero
    axes, |a| x |b| products each (the Walsh-Hadamard adds not counted)."""
    C = (p + 1) ** 2
    size = [0] * 8
    for i in range(C):
        size[_sym_class(i)] += 1
    macs = 0
    for rep in itertools.product(range(4), repeat=3):
        if max(rep) < 2:
            continue
        zmask = sum(1 << a for a in range(3) if rep[a] == 0)
        macs += sum(size[a] * size[b] for a in range(8) for b in range(8) if not ((a ^ b) & zmask))
    return 6.0 * macs


def m2l_translations(level, periodic):
    """Number of M2L translations over all levels of a uniform tree."""
    from itertools import product
    total = 0
    lstart = 1 if periodic else 2
    for l in range(lstart, level + 1):
        side = 1 << l
        if periodic:
            total += 189 * 8 ** l
            continue
        c = np.arange(side)
        for par in product((0, 1), repeat=3):
            # cells with coordinate parities `par`, offsets d_i in [-2-par_i, 3-par_i]
            per_dim = []
            for dd in range(3):
                cc = c[(c & 1) == par[dd]]
                per_dim.append((cc, np.arange(-2 - par[dd], 4 - par[dd])))
            cnt = 0
            for dx in per_dim[0][1]:
                for dy in per_dim[1][1]:
                    for dz in per_dim[2][1]:
                        if max(abs(dx), abs(dy), abs(dz)) < 2:
                            continue
                        nx = np.sum((per_dim[0][0] + dx >= 0) & (per_dim[0][0] + dx < side))
                        ny = np.sum((per_dim[1][0] + dy >= 0) & (per_dim[1][0] + dy < side))
                        nz = np.sum((per_dim[2][0] + dz >= 0) & (per_dim[2][0] + dz < side))
                        cnt += int(nx) * int(ny) * int(nz)
            total += cnt
    return total


def _morton_tables(level):
    side = 1 << level
    c = np.arange(side)
    spread = np.zeros(side, np.int64)
    for b in range(level):
        spread |= ((c >> b) & 1) << (3 * b)
    return spread


def near_pairs(start, level, periodic):
    counts = np.diff(start).astype(np.int64)
    side = 1 << level
    spread = _morton_tables(level)
    ix, iy, iz = np.meshgrid(np.arange(side), np.arange(side), np.arange(side), indexing="ij")
    key = spread[ix] | (spread[iy] << 1) | (spread[iz] << 2)
    cnt = counts[key]
    total = 0
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                if periodic:
                    nb = np.roll(cnt, shift=(-dx, -dy, -dz), axis=(0, 1, 2))
                    total += int(np.sum(cnt * nb))
                else:
                    sl_t = [slice(max(0, -d), side - max(0, d)) for d in (dx, dy, dz)]
                    sl_s = [slice(max(0, d), side - max(0, -d)) for d in (dx, dy, dz)]
                    total += int(np.sum(cnt[tuple(sl_t)] * cnt[tuple(sl_s)]))
    return total


def tree_bytes_per_particle(level, f32):
    """Algorithmic HBM bytes of the tree build per particle: keys (read x 24 B, write key and
    index 8 B), per radix pass (histogram reads the key 4 B; scatter reads and writes key and
    index 16 B), ranges (read the key 4 B), permute (read index 4 B, gather x and alpha 48 B,
    write the 32 B or 64 B particle record)."""
    npass = (3 * level + 7) // 8
    return 32 + 20 * npass + 4 + 52 + (32 if f32 else 64)


TREE_KERNELS = ("k_keys", "k_iota", "k_radix_hist", "k_radix_scatter", "k_scan_tiles", "k_scan_sums",
                "k_scan_add", "k_ranges", "k_permute")


def _traffic_summary(workload, precision):
    """The committed rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE, calibrated
    on a 1 GiB copy), or None when there is none or the kernel sources have changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}_{precision}.txt")
    if not os.path.exists(path):
        return None
    from paper_1110_2921_amd.rocprof_summary import sources_sha256
    with open(path) as f:
        d = json.load(f)
    return d if d.get("sources_sha256") == sources_sha256() else None


def measured_traffic(workload, precision, kernel, launches_per_eval=None):
    """HBM bytes per launch of `kernel` (see _traffic_summary), or None.  With
    `launches_per_eval`, the kernel's bytes per evaluation divided by its
    launches per evaluation (the profile then comes from an evaluations-only
    run, so every dispatch of the kernel belongs to an evaluation)."""
    d = _traffic_summary(workload, precision)
    k = None if d is None else d.get("kernels", {}).get(kernel)
    if k is None:
        return None
    if launches_per_eval and k.get("hbm_bytes_per_evaluation"):
        return k["hbm_bytes_per_evaluation"] / launches_per_eval
    return k["hbm_bytes_per_launch"]


def measured_phase_bytes(workload, precision, kernels):
    """HBM bytes per evaluation of all dispatches of `kernels` (names or name
    prefixes) in the committed summary of an evaluations-only run, or None."""
    d = _traffic_summary(workload, precision)
    if d is None:
        return None
    ks = d.get("kernels", {})
    hit = [v for k, v in ks.items() if any(k.startswith(x) for x in kernels)]
    if not hit or any(v.get("hbm_bytes_per_evaluation") is None for v in hit):
        return None
    return sum(v["hbm_bytes_per_evaluation"] for v in hit)


def measured_finest_launch(workload, precision, kernel):
    """(grid size, HBM bytes) of the largest launch shape of `kernel`, or None."""
    d = _traffic_summary(workload, precision)
    k = None if d is None else d.get("kernels", {}).get(kernel)
    if not k or not k.get("shapes"):
        return None
    sh = max(k["shapes"], key=lambda x: x["grid_size"])
    return sh["grid_size"], sh["hbm_bytes_per_dispatch"]


def measured_tree_bytes(workload, precision):
    """HBM bytes of the tree build per evaluation (sum over its kernels), or None."""
    d = _traffic_summary(workload, precision)
    if d is None or "k_keys" not in d.get("kernels", {}):
        return None
    ks = d["kernels"]
    evals = ks["k_keys"]["dispatches"]          # one key pass per evaluation
    return sum(ks[k]["hbm_bytes_per_launch"] * ks[k]["dispatches"] / evals for k in TREE_KERNELS if k in ks)


def direct_at(x, a, sigma, box_len, targets):
    """CPU leg: the oracle's exact free-space sum at the sampled particles."""
    from oracle import direct as oracle_direct

    return oracle_direct.direct(x[targets], x, a, sigma, box_len, K=0)


def cpu_baseline(w, x_full, a_full, targets):
    """The oracle timed on the host: its FMM on a 32^3 sample of the same recipe,
    and its direct sum (the exact regularised kernel over the 27 images S_1) at
    the sampled particles `targets` of the full workload.  Returns the baseline
    record and the direct-sum velocity and gradient at the targets, against
    which the GPU's accuracy is stated."""
    import resource

    import workloads as W
    from oracle import direct as oracle_direct
    from oracle import fmm as oracle_fmm
    from oracle import tree as oracle_tree

    def cpu_seconds():
        r = resource.getrusage(resource.RUSAGE_SELF)
        return r.ru_utime + r.ru_stime

    ng = 32
    x, a = W.random_field(ng, w.k0, seed=w.seed)
    h = 2 * math.pi / ng
    level = 3                     # 64 particles per leaf, as in the full workload
    reps = []
    c0 = cpu_seconds()
    for _ in range(3):            # median of three runs (about 5 s each on 16 cores)
        t0 = time.perf_counter()
        oracle_fmm.fmm(x, a, h, w.p, level, periodic=w.periodic)
        reps.append(time.perf_counter() - t0)
    # the threads the oracle kept busy on average: its CPU seconds over its wall seconds
    busy = (cpu_seconds() - c0) / sum(reps)
    t = sorted(reps)[1]
    n_sample = ng ** 3
    xw = oracle_tree.wrap(x_full, (0.0, 0.0, 0.0), w.box_len)
    c0 = cpu_seconds()
    t0 = time.perf_counter()
    ud, Jd = oracle_direct.direct(xw[targets], xw, a_full, w.sigma, w.box_len, K=1)
    td = time.perf_counter() - t0
    busy_d = (cpu_seconds() - c0) / td
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    rec = {"value": (n_sample / w.n) / t, "unit": "evals/s", "cores": round(busy, 1), "kind": "oracle",
           "cores_what": "average busy threads of the oracle FMM (process CPU time over wall time): its P2P "
                         "runs in C/OpenMP, the expansions in NumPy",
           "threads_available": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
           "cpu_model": model, "os_cpu_count": os.cpu_count(),
           "direct_pairs_per_s": len(targets) * w.n * 27 / td, "direct_cores": round(busy_d, 1),
           "sample": f"oracle CPU FMM (NumPy + C/OpenMP, FP64) on N={ng}^3 particles of the same recipe "
                     f"(k0={w.k0:g}, 64/leaf, p={w.p}, {3 ** w.periodic}^3 images), median of 3 runs {t:.1f} s, "
                     f"scaled by {n_sample}/{w.n} (cost linear in N at fixed particles per leaf); direct sum "
                     f"at {len(targets)} sampled particles of the full workload over S_1 ({td:.1f} s)",
           "seconds": t}
    return rec, ud, Jd


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rand256_periodic")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-check", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the accuracy against the direct sum and the p = 14 timings")
    ap.add_argument("--no-rbf", action="store_true")
    ap.add_argument("--no-truncation", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="also time a 32^3 evaluation eagerly and from a captured HIP graph")
    ap.add_argument("--tuning", action="store_true", help="also run the leaf-level tuner at this workload")
    ap.add_argument("--loop-steps", type=int, default=10,
                    help="steps of the paper's time loop to time (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="one 1 GiB device-to-device copy (known bytes) for counter calibration")
    ap.add_argument("--no-adaptive", action="store_true",
                    help="skip the adaptive-tree comparison on clustered particles")
    ap.add_argument("--evals-only", action="store_true",
                    help="time the Heun steps only (no other sections): the run the profiles are taken from")
    args = ap.parse_args()
    if args.evals_only:
        args.no_cpu_baseline = args.no_fp64_check = args.no_adjoint = args.no_accuracy = True
        args.no_rbf = args.no_truncation = args.no_adaptive = True
        args.loop_steps = 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_1110_2921_amd as vm
    import workloads as W

    w = W.WORKLOADS[args.workload]
    log(f"[bench] generating {w.name}: N={w.n}")
    t0 = time.perf_counter()
    x_np, a_np = W.make(w)
    log(f"[bench] inputs ready in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    x = torch.from_numpy(np.ascontiguousarray(x_np.T)).to(dev)
    a = torch.from_numpy(np.ascontiguousarray(a_np.T)).to(dev)
    n = w.n
    x0, a0 = x.clone(), a.clone()            # initial state, kept for the FP64 comparison
    u = torch.empty((3, n), dtype=torch.float64, device=dev)
    da = torch.empty((3, n), dtype=torch.float64, device=dev)
    J = torch.empty((9, n), dtype=torch.float64, device=dev)
    ctx = vm.FMM(0)
    kw = dict(periodic=w.periodic, box_len=w.box_len, scheme="classic")
    dt = PAPER_DT
    h3 = w.h ** 3

    def step(prec, xs, as_):
        ctx.rk2_step(xs, as_, w.sigma, w.p, w.level, dt, precision=prec, want_initial=True, out=(u, J), **kw)

    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for i in range(args.warmup):
        step(args.precision, x, a)
        log(f"[bench] warmup {i + 1}/{args.warmup}")
    x.copy_(x0)
    a.copy_(a0)
    torch.cuda.synchronize()

    ctx.set_timing(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    diag0 = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for i in range(args.steps):
        step(args.precision, x, a)
        if i == 0:
            diag0 = ctx.diagnostics(u, J, a0, h3)   # (E, Omega, Omega_p) at the initial state
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = ctx.timing()
    ctx.set_timing(False)
    gpu_ms = ev0.elapsed_time(ev1)
    n_eval = 2 * args.steps
    ms_per_step = 1000.0 * wall / args.steps
    log(f"[bench] {args.steps} RK2 steps: {ms_per_step:.2f} ms/step (events {gpu_ms / args.steps:.2f} ms)")
    for k, (ms, cnt) in phases.items():
        log(f"[bench]   {k:8s} {ms / n_eval:9.3f} ms/eval  launches {cnt / n_eval:.0f}")

    # energy / enstrophy after the steps (one more evaluation, untimed)
    ctx.eval(x, a, w.sigma, w.p, w.level, precision=args.precision, out=(u, da, J), **kw)
    diag1 = ctx.diagnostics(u, J, a, h3)
    d0 = diag0.cpu().numpy()
    d1 = diag1.cpu().numpy()
    drift = {"energy": float((d1[0] - d0[0]) / d0[0]), "enstrophy": float((d1[1] - d0[1]) / d0[1]),
             "particle_enstrophy": float((d1[2] - d0[2]) / d0[2]), "steps": args.steps, "dt": dt}
    log(f"[bench] relative drift over {args.steps} steps: E {drift['energy']:.3e} "
        f"Omega {drift['enstrophy']:.3e}")

    # work counts
    _, _, start = ctx.debug_tree(n, w.level)
    pairs = near_pairs(start, w.level, w.periodic > 0)
    ntr = m2l_translations(w.level, w.periodic > 0)
    C = (w.p + 1) ** 2
    m2l_flop = 6.0 * C * C * ntr
    p2p_ms = phases["p2p"][0] / n_eval
    m2l_ms = phases["m2l"][0] / n_eval
    m2l_launch = phases["m2l"][1] / n_eval
    p2p_flop = P2P_FLOP_PER_PAIR[args.precision] * pairs
    f32 = args.precision == "mixed"
    esz = 4 if f32 else 8
    # FP32 at p = 10: the orbit kernel from level 4 on (class-major pack of the
    # multipoles first), dense operator-stationary MFMAs below
    orbit = w.p == 10 and w.level >= 4
    lev0 = 1 if w.periodic else 2
    if orbit:
        m2l_kernel = ("k_m2l_sym<10> (levels 4+) + k_m2l_os<4,8,false> (levels < 4) + k_sym_pack" if f32 else
                      "k_m2l_sym64<10> (levels 4+) + k_translate<double,1,1,0,24> (levels < 4) + k_sym_pack")
        per_t = orbit_m2l_flop_per_target(w.p)
        m2l_flop = sum(8 ** l * (per_t if l >= 4 else 6.0 * C * C * 189) for l in range(lev0, w.level + 1))
    else:
        m2l_kernel = "k_translate<double,1,1,0,24>" if not f32 else "k_m2l_os"
    # HBM bytes of the whole M2L phase per evaluation (every launch of its kernels)
    m2l_traffic = measured_phase_bytes(w.name, args.precision,
                                       ("k_m2l_sym<", "k_m2l_os", "k_sym_pack<float>", "k_split_reduce<float>")
                                       if f32 else ("k_m2l_sym64", "k_translate<double,1,1,0,", "k_sym_pack<double>",
                                                    "k_split_reduce<double>"))
    # algorithmic bytes of the M2L phase: read M, read and write L at every level, the operators once
    cells = sum(8 ** l for l in range(lev0, w.level + 1))
    m2l_alg_bytes = cells * 3 * C * esz * 3 + 316 * C * C * esz
    roof_m2l = {"bound": "mfma", "kernel": f"{m2l_kernel} (M2L phase, all levels)",
                "flop_per_eval": m2l_flop,
                "achieved": m2l_flop / (m2l_ms * 1e-3) / 1e12,
                "peak": PEAKS["mfma_f32_tflops" if f32 else "mfma_f64_tflops"], "unit": "TFLOP/s",
                "traffic": m2l_traffic, "traffic_unit": "bytes per evaluation",
                "algorithmic_bytes_per_eval": m2l_alg_bytes, "launches_per_eval": m2l_launch}
    sym_name = "k_m2l_sym<10>" if f32 else "k_m2l_sym64<10>"
    fin = measured_finest_launch(w.name, args.precision, sym_name) if orbit else None
    if fin:
        roof_m2l["finest_level_launch"] = {"kernel": sym_name, "grid_size": fin[0], "hbm_bytes": fin[1],
                                           "algorithmic_bytes": 8 ** w.level * 3 * C * esz * 2}
    roof_m2l["frac"] = roof_m2l["achieved"] / roof_m2l["peak"]
    p2p_kernel = "k_p2p32" if f32 else "k_p2p64"
    roof_p2p = {"bound": "alu", "kernel": p2p_kernel,
                "achieved": p2p_flop / (p2p_ms * 1e-3) / 1e12,
                "peak": PEAKS["valu_f32_tflops" if f32 else "valu_f64_tflops"], "unit": "TFLOP/s",
                "traffic": measured_traffic(w.name, args.precision, p2p_kernel, 1), "traffic_unit": "bytes per launch",
                # the sorted records in, the near field out (u, raw gradient sums, strength sums: 15 doubles)
                "algorithmic_bytes_per_launch": n * (32 if f32 else 64) + n * 8 * 15}
    roof_p2p["frac"] = roof_p2p["achieved"] / roof_p2p["peak"]
    dominant = roof_p2p if p2p_ms >= m2l_ms else roof_m2l
    tree_ms = phases["tree"][0] / n_eval
    tree_bytes = tree_bytes_per_particle(w.level, f32) * n
    tree_meas = measured_tree_bytes(w.name, args.precision)
    roof_tree = {"bound": "hbm", "kernel": "tree (keys, radix passes, ranges, permute)",
                 "achieved": tree_bytes / (tree_ms * 1e-3) / 1e9, "peak": PEAKS["hbm_gbs"], "unit": "GB/s",
                 "traffic": tree_meas, "traffic_unit": "bytes per evaluation",
                 "measured_gbs": None if tree_meas is None else tree_meas / (tree_ms * 1e-3) / 1e9}
    roof_tree["frac"] = roof_tree["achieved"] / roof_tree["peak"]

    result = {
        "metric": "FMM evals/sec and P2P Ginteractions/s at N=256^3, p=10, rel-L2 err vs FP64",
        "value": n_eval / wall,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if f32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: N={w.ng}^3 cell-centred lattice in [0,2pi)^3, random-phase "
                               f"solenoidal field E(k)~k^4 exp(-2k^2/k0^2), k0={w.k0:g}, sigma=h, "
                               f"p={w.p}, leaf level {w.level} (64/leaf), {3 ** w.periodic}^3 periodic images, "
                               f"{args.precision} precision, classic stretching; step = one Heun RK2 step "
                               f"(2 evaluations, dt={dt})",
                   "n": n, "p": w.p, "level": w.level, "periodic_K": w.periodic,
                   "precision": args.precision, "parallelism": "single GPU"},
        "p2p_gpairs_per_s": pairs / (p2p_ms * 1e-3) / 1e9,
        "p2p_pairs": pairs,
        "m2l_translations": ntr,
        "phase_ms_per_eval": {k: v[0] / n_eval for k, v in phases.items()},
        "phase_note": "P2P runs on a side stream from the end of the tree build and overlaps P2M and whatever of "
                      "the far field the hardware schedules beside it, so phase times overlap; L2P waits for P2P "
                      "and adds the far field to the near field",
        "evals_per_step": 2,
        "drift": drift,
        "roofline": dominant,
        "roofline_kernels": {"m2l": roof_m2l, "p2p": roof_p2p, "tree": roof_tree},
    }

    if not args.no_fp64_check and args.precision == "mixed":
        # accuracy at the initial state, FP64 throughput and the FP64 drift
        um, dam = torch.empty_like(u), torch.empty_like(da)
        ctx.eval(x0, a0, w.sigma, w.p, w.level, precision="mixed", out=(um, dam, None), **kw)
        u64, da64 = torch.empty_like(u), torch.empty_like(da)
        ctx.eval(x0, a0, w.sigma, w.p, w.level, precision="fp64", out=(u64, da64, None), **kw)
        eu = float(torch.linalg.norm(um - u64) / torch.linalg.norm(u64))
        ed = float(torch.linalg.norm(dam - da64) / torch.linalg.norm(da64))
        del um, dam, u64, da64
        x.copy_(x0)
        a.copy_(a0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d64_0 = None
        for i in range(args.steps):
            step("fp64", x, a)
            if i == 0:
                d64_0 = ctx.diagnostics(u, J, a0, h3)
        torch.cuda.synchronize()
        t64 = (time.perf_counter() - t0) / (2 * args.steps)
        ctx.eval(x, a, w.sigma, w.p, w.level, precision="fp64", out=(u, da, J), **kw)
        e0 = d64_0.cpu().numpy()
        e1 = ctx.diagnostics(u, J, a, h3).cpu().numpy()
        result["rel_l2_u_vs_fp64"] = eu
        result["rel_l2_dalpha_vs_fp64"] = ed
        result["fp64_evals_per_s"] = 1.0 / t64
        result["mixed_speedup_vs_fp64"] = result["value"] * t64
        result["drift_fp64"] = {"energy": float((e1[0] - e0[0]) / e0[0]),
                                "enstrophy": float((e1[1] - e0[1]) / e0[1])}
        log(f"[bench] fp64 {t64 * 1e3:.1f} ms/eval; mixed vs fp64 rel-L2 u {eu:.2e} dalpha {ed:.2e}; "
            f"fp64 drift E {result['drift_fp64']['energy']:.3e}")

    if not args.no_accuracy:
        # accuracy against the exact sum (images S_1, the oracle's direct sum at 16 sampled
        # particles, computed in the CPU-baseline leg) at the headline degree and at
        # p = 14, where the FP64 error in u falls below 1e-6; both forms timed at p = 14
        # in the headline configuration
        targets = np.sort(np.random.default_rng(11).choice(n, 16, replace=False))
        tt = torch.from_numpy(targets).to(dev)
        acc_p = (w.p, 14)
        got = {}
        for pp in acc_p:
            for prec in ("fp64", "mixed"):
                ctx.eval(x0, a0, w.sigma, pp, w.level, periodic=1, box_len=w.box_len, precision=prec,
                         want_dalpha=False, out=(u, None, J))
                got[pp, prec] = (u[:, tt].cpu().numpy().T, J[:, tt].cpu().numpy().T)
        t14 = {}
        for prec in ("fp64", "mixed"):
            ctx.eval(x0, a0, w.sigma, 14, w.level, precision=prec, out=(u, da, None), **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                ctx.eval(x0, a0, w.sigma, 14, w.level, precision=prec, out=(u, da, None), **kw)
            torch.cuda.synchronize()
            t14[prec] = (time.perf_counter() - t0) / 3
        result["accuracy_vs_direct"] = {"targets": len(targets), "images": "S_1 (27 boxes)", "per_p": {}}
        result["p14"] = {"fp64_ms": 1e3 * t14["fp64"], "mixed_ms": 1e3 * t14["mixed"],
                         "mixed_speedup_vs_fp64": t14["fp64"] / t14["mixed"],
                         "what": "one evaluation (u, dalpha/dt) at p = 14 in the headline configuration"}
        log(f"[bench] p=14: fp64 {1e3 * t14['fp64']:.1f} ms, mixed {1e3 * t14['mixed']:.1f} ms per evaluation")
        pending_accuracy = (targets, acc_p, got)
    else:
        pending_accuracy = None

    if not args.no_adjoint:
        # reverse pass: gradient of L = h^3/2 sum |u|^2 with respect to x and alpha (the
        # forward evaluation is recomputed inside, the tree and expansions are not stored)
        ub = h3 * u
        ctx.adjoint(x, a, ub, w.sigma, w.p, w.level, periodic=w.periodic, box_len=w.box_len,
                    precision=args.precision)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            ctx.adjoint(x, a, ub, w.sigma, w.p, w.level, periodic=w.periodic, box_len=w.box_len,
                        precision=args.precision)
        torch.cuda.synchronize()
        ta = (time.perf_counter() - t0) / 3
        # the same gradient reusing the tree and gradient of the evaluation just made
        # (what the autograd backward pass does): evaluation + reusing adjoint
        Jr = torch.empty((9, n), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            ctx.eval(x, a, w.sigma, w.p, w.level, precision=args.precision, want_dalpha=False, out=(u, None, Jr),
                     **kw)
            ctx.adjoint(x, a, ub, w.sigma, w.p, w.level, periodic=w.periodic, box_len=w.box_len,
                        precision=args.precision, grad=Jr)
        torch.cuda.synchronize()
        tvg = (time.perf_counter() - t0) / 3
        del Jr
        result["adjoint"] = {"gradients_per_s": 1.0 / ta, "ms": 1e3 * ta, "precision": args.precision,
                             "value_and_gradient_ms": 1e3 * tvg,
                             "what": "dL/dx and dL/dalpha of L = h^3/2 sum |u|^2: ms with the forward state "
                                     "recomputed inside; value_and_gradient_ms: one evaluation (u, J) plus "
                                     "the adjoint reusing its tree and gradient (the autograd path)"}
        log(f"[bench] adjoint {1e3 * ta:.1f} ms per gradient; evaluation + reusing adjoint {1e3 * tvg:.1f} ms")

    if not args.no_truncation:
        # the M2L truncated to n + n' <= p: time and distance from the square truncation
        ctx.eval(x0, a0, w.sigma, w.p, w.level, precision=args.precision, out=(u, da, None), **kw)
        ut = torch.empty_like(u)
        ctx.eval(x0, a0, w.sigma, w.p, w.level, precision=args.precision, out=(ut, None, None),
                 truncation="triangular", **kw)
        torch.cuda.synchronize()
        ctx.set_timing(True)
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.eval(x0, a0, w.sigma, w.p, w.level, precision=args.precision, out=(ut, None, None),
                     truncation="triangular", **kw)
        torch.cuda.synchronize()
        tt = (time.perf_counter() - t0) / reps
        ph = ctx.timing()
        ctx.set_timing(False)
        dtri = float(torch.linalg.norm(ut - u) / torch.linalg.norm(u))
        result["triangular_truncation"] = {
            "evals_per_s": 1.0 / tt, "ms": 1e3 * tt, "m2l_ms": ph["m2l"][0] / reps,
            "rel_l2_u_vs_square": dtri, "products_per_component": "2926 of 14641 at p = 10",
            "what": "M2L keeping target degree n and source degree n' with n + n' <= p (zero tiles skipped)"}
        log(f"[bench] triangular truncation: {1e3 * tt:.1f} ms/eval (M2L {ph['m2l'][0] / reps:.1f} ms), "
            f"rel-L2 u vs square {dtri:.2e}")
        del ut

    if not args.no_rbf:
        # RBF reinitialisation of the initial lattice: strengths that reproduce
        # omega = alpha / h^3 at the particles, GMRES from h^3 omega at the
        # default tolerance 1e-3 (relative residual drop)
        om = a0 / h3
        gam = torch.empty_like(a0)
        rkw = dict(periodic=w.periodic, box_len=w.box_len, precision=args.precision, out=gam)
        ctx.rbf_solve(x0, om, w.sigma, h3, w.level, tol=PAPER_TOL, max_iter=100, **rkw)
        torch.cuda.synchronize()
        ctx.set_timing(True)
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            _, iters, resid = ctx.rbf_solve(x0, om, w.sigma, h3, w.level, tol=PAPER_TOL, max_iter=100, **rkw)
        torch.cuda.synchronize()
        tr = (time.perf_counter() - t0) / reps
        ph = ctx.timing()
        ctx.set_timing(False)
        gauss_ms = ph["gauss"][0] / ph["gauss"][1]
        products = ph["gauss"][1] / reps
        gauss_kernel = "k_gauss<float,vmfmm::Part32>" if f32 else "k_gauss<double,vmfmm::Part64>"
        roof_gauss = {"bound": "alu", "kernel": gauss_kernel + " (with the strength packing)",
                      "achieved": GAUSS_FLOP_PER_PAIR * pairs / (gauss_ms * 1e-3) / 1e12,
                      "peak": PEAKS["valu_f32_tflops" if f32 else "valu_f64_tflops"], "unit": "TFLOP/s",
                      "traffic": measured_traffic(w.name, args.precision, gauss_kernel),
                      "traffic_unit": "bytes per launch"}
        roof_gauss["frac"] = roof_gauss["achieved"] / roof_gauss["peak"]
        result["rbf"] = {"ms": 1e3 * tr, "iterations": iters, "products": products, "resid": resid,
                         "tol": PAPER_TOL, "precision": args.precision, "gauss_ms_per_product": gauss_ms,
                         "gauss_gpairs_per_s": pairs / (gauss_ms * 1e-3) / 1e9,
                         "krylov_ms": ph["krylov"][0] / reps, "tree_ms": ph["tree"][0] / reps,
                         "vs_rk2_step": 1e3 * tr / ms_per_step, "roofline": roof_gauss,
                         "what": "gamma with A gamma = omega on the initial lattice (neighbour-list Gaussian "
                                 "sums, GMRES(20) from h^3 omega)"}
        log(f"[bench] rbf solve {1e3 * tr:.1f} ms, {iters} iterations ({products:.0f} products, "
            f"{gauss_ms:.2f} ms each), resid {resid:.2e}; {1e3 * tr / ms_per_step:.2f} RK2 steps")
        del om, gam

    if not args.no_rbf:
        # velocity on the grid of the spectral method (cell corners, N points) from the
        # particles, and its shell energy spectrum
        c = torch.arange(w.ng, dtype=torch.float64, device=dev) * (w.box_len / w.ng)
        Y = torch.stack(torch.meshgrid(c, c, c, indexing="ij"), dim=0).reshape(3, -1).contiguous()
        del c
        kmax = w.ng // 2
        ctx.eval_at(x0, a0, Y, w.sigma, w.p, w.level, periodic=w.periodic, box_len=w.box_len,
                    precision=args.precision)
        ctx.energy_spectrum(u, w.ng, kmax)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ug, _ = ctx.eval_at(x0, a0, Y, w.sigma, w.p, w.level, periodic=w.periodic, box_len=w.box_len,
                            precision=args.precision)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        spec = ctx.energy_spectrum(ug, w.ng, kmax)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        sp = spec.cpu().numpy()
        result["grid_spectrum"] = {"points": int(Y.shape[1]), "eval_at_ms": 1e3 * (t1 - t0),
                                   "spectrum_ms": 1e3 * (t2 - t1), "kmax": kmax,
                                   "peak_shell": int(np.argmax(sp)), "energy": float(sp.sum()),
                                   "what": "velocity of the particles at the N grid points (vm_fmm_eval_at) "
                                           "and its shell energy spectrum (vm_energy_spectrum)"}
        log(f"[bench] grid velocity {1e3 * (t1 - t0):.1f} ms, spectrum {1e3 * (t2 - t1):.1f} ms "
            f"(peak shell {int(np.argmax(sp))})")
        del Y, ug, spec

    if args.loop_steps > 0:
        # the paper's loop from the initial state: forward Euler, dt = 0.005, core
        # spreading with nu = lambda / Re_lambda (Re_lambda = 50, u' = 1, lambda = 2/k0
        # for this spectrum), reinitialisation every 10 steps at tolerance 1e-3
        nu = 2.0 / w.k0 / 50.0
        x.copy_(x0)
        a.copy_(a0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sg, diag, prods, resid = ctx.run(x, a, w.sigma, w.p, w.level, dt, args.loop_steps, nu=nu,
                                         integrator="euler", reinit_every=PAPER_REINIT_EVERY, ng=w.ng,
                                         tol=PAPER_TOL, max_iter=100,
                                         periodic=w.periodic, box_len=w.box_len, precision=args.precision,
                                         want_diag=True)
        torch.cuda.synchronize()
        tl = time.perf_counter() - t0
        dg = diag.cpu().numpy()
        result["time_loop"] = {"steps": args.loop_steps, "ms_per_step": 1e3 * tl / args.loop_steps,
                               "integrator": "euler", "dt": dt, "nu": nu, "reinit_every": PAPER_REINIT_EVERY,
                               "tol": PAPER_TOL,
                               "gmres_products": prods, "gmres_resid": resid, "sigma_end": sg,
                               "energy_drift": float((dg[-1, 0] - dg[0, 0]) / dg[0, 0]),
                               "what": "Euler steps with core spreading and lattice reinitialisation (RBF), "
                                       "diagnostics every step, from the initial state"}
        log(f"[bench] time loop: {args.loop_steps} Euler steps with reinitialisation every 10: "
            f"{1e3 * tl / args.loop_steps:.1f} ms/step ({prods} GMRES products)")
        x.copy_(x0)
        a.copy_(a0)

    if args.tuning:
        # auto-tuned leaf level for the benchmark's particles (leaves >= 4 sigma)
        lv, lms = ctx.tune_level(x0, a0, w.sigma, w.p, periodic=w.periodic, box_len=w.box_len,
                                 precision=args.precision)
        result["level_tuning"] = {"level": lv, "ms_per_level": {str(k): v for k, v in sorted(lms.items())},
                                  "what": "fastest leaf level with leaves at least 4 sigma wide (vm_tune_level)"}
        log(f"[bench] tuned leaf level {lv}: " + ", ".join(f"level {k} {v:.1f} ms" for k, v in sorted(lms.items())))

    if args.graph:
        # a small problem (32^3, p = 8) is launch-bound: one evaluation eagerly and
        # replayed from a HIP graph captured on the library's stream
        ws = W.WORKLOADS["rand32_periodic"]
        xs_np, as_np = W.make(ws)
        xs = torch.from_numpy(np.ascontiguousarray(xs_np.T)).to(dev)
        as_ = torch.from_numpy(np.ascontiguousarray(as_np.T)).to(dev)
        us = torch.empty((3, ws.n), dtype=torch.float64, device=dev)
        das = torch.empty_like(us)
        skw = dict(periodic=ws.periodic, box_len=ws.box_len, precision=args.precision, out=(us, das, None))
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            for _ in range(3):
                ctx.eval(xs, as_, ws.sigma, ws.p, ws.level, **skw)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=st):
            ctx.eval(xs, as_, ws.sigma, ws.p, ws.level, **skw)
        torch.cuda.synchronize()
        reps = 50
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.eval(xs, as_, ws.sigma, ws.p, ws.level, **skw)
        torch.cuda.synchronize()
        te = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        for _ in range(reps):
            graph.replay()
        torch.cuda.synchronize()
        tg = (time.perf_counter() - t0) / reps
        result["graph_small"] = {"workload": f"{ws.name}: N={ws.ng}^3, p={ws.p}, level {ws.level}",
                                 "eager_ms": 1e3 * te, "graph_ms": 1e3 * tg,
                                 "what": "one evaluation, eager (host launches) and replayed from a captured HIP graph"}
        log(f"[bench] 32^3 evaluation: eager {1e3 * te:.3f} ms, graph replay {1e3 * tg:.3f} ms")
        del graph, xs, as_, us, das

    pending_adaptive = None
    if not args.no_adaptive:
        # clustered particles (Gaussian clusters and a uniform tenth, free space):
        # the adaptive hybrid tree with its tuned leaf size against the uniform
        # tree at its tuned level, both FP64 at p = 10; the accuracy of both
        # against the exact sum at sampled particles comes with the CPU leg
        na, pa = 1 << 19, 10
        xa_np, aa_np = W.clustered_particles(na, seed=41)
        sg = w.box_len / 1024
        max_level = 8                 # leaves at least 4 sigma wide
        xa = torch.from_numpy(np.ascontiguousarray(xa_np.T)).to(dev)
        aa = torch.from_numpy(np.ascontiguousarray(aa_np.T)).to(dev)
        # the uniform tree at the finest level with no more leaves than particles
        # (lv) and one finer (leaves still >= 4 sigma); coarser levels put thousands
        # of clustered particles in one leaf, whose near field one wave then runs
        # alone for seconds; the faster of the two is the uniform figure
        lv = 0
        while lv < 10 and w.box_len / 2 ** (lv + 1) >= 4 * sg and 8 ** (lv + 1) <= na:
            lv += 1
        levels = [lv] + ([lv + 1] if w.box_len / 2 ** (lv + 1) >= 4 * sg else [])
        log(f"[bench] clustered {na}: uniform tree at levels {levels}, tuning the adaptive leaf size")
        nc, nms = ctx.tune_ncrit(xa, aa, sg, pa, max_level, periodic=0, box_len=w.box_len, reps=1)
        log(f"[bench] adaptive ncrit {nc}: " + ", ".join(f"{k}: {v:.1f} ms" for k, v in sorted(nms.items())))
        reps = 3

        def timed(fn):
            out = fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                out = fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps, out

        uni = {}
        for l in levels:
            uni[l] = timed(lambda: ctx.eval(xa, aa, sg, pa, l, box_len=w.box_len, precision="fp64", want_grad=True))
            log(f"[bench] clustered uniform level {l}: {1e3 * uni[l][0]:.1f} ms per evaluation")
        lbest = min(uni, key=lambda l: uni[l][0])
        timings = {"uniform": uni[lbest]}
        timings["adaptive"] = timed(lambda: ctx.eval_adaptive(xa, aa, sg, pa, nc, max_level, box_len=w.box_len,
                                                              want_grad=True))
        log(f"[bench] clustered adaptive: {1e3 * timings['adaptive'][0]:.1f} ms per evaluation")
        ctx.set_timing(True)
        ctx.eval_adaptive(xa, aa, sg, pa, nc, max_level, box_len=w.box_len, want_grad=True)
        torch.cuda.synchronize()
        ad_phases = {k: v[0] for k, v in ctx.timing().items() if v[1]}
        ctx.set_timing(False)
        log("[bench] adaptive phases: " + ", ".join(f"{k} {v:.2f}" for k, v in ad_phases.items()) + " ms")
        cells = ctx.debug_adaptive("cells")
        lists = {k: int(len(ctx.debug_adaptive(k))) for k in ("p2p", "m2l", "m2p", "p2l")}
        tga = np.sort(np.random.default_rng(12).choice(na, 16, replace=False))
        got_a = {k: (v[1][0][:, tga].cpu().numpy().T, v[1][2][:, tga].cpu().numpy().T) for k, v in timings.items()}
        result["adaptive"] = {
            "workload": f"{na} particles in 8 Gaussian clusters (std 1/64 .. 1/8 of the box) and a uniform tenth, "
                        f"free space, sigma = box/1024, p = {pa}, FP64, u + J + dalpha/dt",
            "uniform": {"level": lbest, "ms": 1e3 * timings["uniform"][0],
                        "ms_per_level": {str(l): 1e3 * v[0] for l, v in uni.items()},
                        "what": "the faster of the finest level with no more leaves than particles and one finer "
                                "(leaves at least 4 sigma wide)"},
            "adaptive": {"ncrit": nc, "max_level": max_level, "ms": 1e3 * timings["adaptive"][0],
                         "tuning_ms_per_ncrit": {str(k): v for k, v in sorted(nms.items())},
                         "cells": int(len(cells)), "leaves": int(cells[:, 5].sum()),
                         "deepest_leaf_level": int(cells[cells[:, 5] == 1, 1].max()), "lists": lists,
                         "phase_ms": ad_phases},
            "speedup_vs_uniform": timings["uniform"][0] / timings["adaptive"][0]}
        log(f"[bench] clustered {na}: uniform level {lbest} {1e3 * timings['uniform'][0]:.1f} ms, adaptive ncrit {nc} "
            f"{1e3 * timings['adaptive'][0]:.1f} ms ({len(cells)} cells)")
        pending_adaptive = (xa_np, aa_np, sg, tga, got_a)
        del xa, aa, timings, uni

    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        tg = pending_accuracy[0] if pending_accuracy else np.zeros(0, np.int64)
        result["cpu_baseline"], ud, Jd = cpu_baseline(w, x_np, a_np, tg)
        if pending_accuracy:
            _, acc_p, got = pending_accuracy
            for pp in acc_p:
                e = {}
                for prec in ("fp64", "mixed"):
                    ug, Jg = got[pp, prec]
                    e[prec] = {"u": float(np.linalg.norm(ug - ud) / np.linalg.norm(ud)),
                               "J": float(np.linalg.norm(Jg - Jd.reshape(-1, 9)) / np.linalg.norm(Jd))}
                result["accuracy_vs_direct"]["per_p"][str(pp)] = e
                log(f"[bench] p={pp} vs direct sum: fp64 u {e['fp64']['u']:.2e} J {e['fp64']['J']:.2e}; "
                    f"mixed u {e['mixed']['u']:.2e} J {e['mixed']['J']:.2e}")
            result["rel_l2_u_vs_direct"] = result["accuracy_vs_direct"]["per_p"][str(w.p)]["mixed"]["u"]
        if pending_adaptive:
            xa_np, aa_np, sg, tga, got_a = pending_adaptive
            ud_a, Jd_a = direct_at(xa_np, aa_np, sg, w.box_len, tga)
            for k, (ug, Jg) in got_a.items():
                result["adaptive"][k]["rel_l2_vs_direct"] = {
                    "u": float(np.linalg.norm(ug - ud_a) / np.linalg.norm(ud_a)),
                    "J": float(np.linalg.norm(Jg - Jd_a.reshape(-1, 9)) / np.linalg.norm(Jd_a)),
                    "targets": len(tga)}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
