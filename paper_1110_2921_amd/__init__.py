"""MI355X-native FMM for the regularised Biot-Savart velocity and stretching.

Python face of ``libvmfmm.so`` (see ``include/vmfmm.h``): torch supplies the
device memory and the stream, every step of the evaluation runs in the
library's HIP kernels.

    ctx = FMM()                         # device 0, torch's current stream
    u, dadt, J = ctx.eval(x, alpha, sigma, p=10, level=6, periodic=3,
                          precision="mixed", want_grad=True)

``x`` and ``alpha`` are float64 CUDA tensors of shape (3, n) (SoA, the
library's layout; (n, 3) inputs are transposed into a copy).
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _lib

PRECISIONS = {"fp64": 0, "mixed": 1}
SCHEMES = {"classic": 0, "transpose": 1}
INTEGRATORS = {"euler": 0, "heun": 1}
TRUNCATIONS = {"square": 0, "triangular": 1}


def _soa(t, torch):
    if t.dim() != 2 or 3 not in t.shape:
        raise ValueError("expected a (3, n) or (n, 3) tensor")
    if t.shape[0] != 3:
        t = t.t()
    if t.dtype != torch.float64:
        raise TypeError("positions and strengths must be float64")
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU")
    return t.contiguous()


class FMM:
    """One library context (workspace + operator cache) on one device/stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._torch = torch
        self._lib = _lib.load()
        self.device = device
        h = ctypes.c_void_p()
        st = self._lib.vm_create(ctypes.byref(h), device, ctypes.c_void_p(self._stream_ptr(stream)))
        if st != _lib.VM_OK:
            raise _lib.VmError(st, "vm_create failed (no HIP device?)")
        self._h = h

    def _stream_ptr(self, stream):
        torch = self._torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return int(s.cuda_stream)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.vm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != _lib.VM_OK:
            msg = self._lib.vm_last_error(self._h).decode()
            raise _lib.VmError(st, msg)

    def eval(self, x, alpha, sigma, p, level, periodic=0, box_lo=(0.0, 0.0, 0.0),
             box_len=2 * math.pi, precision="fp64", scheme="classic", want_grad=False,
             want_dalpha=True, check_domain=False, stream=None, out=None, truncation="square"):
        """Velocity (3, n), stretching (3, n) or None, gradient (9, n) or None."""
        torch = self._torch
        x = _soa(x, torch)
        alpha = _soa(alpha, torch)
        n = x.shape[1]
        if alpha.shape[1] != n:
            raise ValueError("x and alpha differ in length")
        self._check(self._lib.vm_set_stream(self._h, ctypes.c_void_p(self._stream_ptr(stream))))
        if out is None:
            u = torch.empty((3, n), dtype=torch.float64, device=x.device)
            da = torch.empty((3, n), dtype=torch.float64, device=x.device) if want_dalpha else None
            J = torch.empty((9, n), dtype=torch.float64, device=x.device) if want_grad else None
        else:
            u, da, J = out
        opts = self._opts(periodic, box_lo, box_len, precision, scheme, check_domain, truncation)
        st = self._lib.vm_fmm_eval(self._h, n, ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(alpha.data_ptr()), float(sigma), int(p), int(level),
                                   ctypes.byref(opts), ctypes.c_void_p(u.data_ptr()),
                                   ctypes.c_void_p(da.data_ptr() if da is not None else 0),
                                   ctypes.c_void_p(J.data_ptr() if J is not None else 0))
        self._check(st)
        return u, da, J

    def eval_at(self, x, alpha, y, sigma, p, level, periodic=0, box_lo=(0.0, 0.0, 0.0), box_len=2 * math.pi,
                precision="fp64", want_grad=False, check_domain=False, stream=None, truncation="square"):
        """Velocity (3, m) and gradient (9, m) or None at the points y."""
        torch = self._torch
        x = _soa(x, torch)
        alpha = _soa(alpha, torch)
        y = _soa(y, torch)
        n, m = x.shape[1], y.shape[1]
        if alpha.shape[1] != n:
            raise ValueError("x and alpha differ in length")
        self._check(self._lib.vm_set_stream(self._h, ctypes.c_void_p(self._stream_ptr(stream))))
        u = torch.empty((3, m), dtype=torch.float64, device=x.device)
        J = torch.empty((9, m), dtype=torch.float64, device=x.device) if want_grad else None
        opts = self._opts(periodic, box_lo, box_len, precision, "classic", check_domain, truncation)
        self._check(self._lib.vm_fmm_eval_at(self._h, n, ctypes.c_void_p(x.data_ptr()),
                                             ctypes.c_void_p(alpha.data_ptr()), m, ctypes.c_void_p(y.data_ptr()),
                                             float(sigma), int(p), int(level), ctypes.byref(opts),
                                             ctypes.c_void_p(u.data_ptr()),
                                             ctypes.c_void_p(J.data_ptr() if J is not None else 0)))
        return u, J

    def eval_adaptive(self, x, alpha, sigma, p, ncrit, max_level, periodic=0, box_lo=(0.0, 0.0, 0.0),
                      box_len=2 * math.pi, scheme="classic", want_dalpha=True, want_grad=False,
                      check_domain=False, stream=None):
        """vm_fmm_eval_adaptive (FP64): (u, dalpha/dt or None, J or None), (3, n) / (9, n)."""
        torch = self._torch
        x = _soa(x, torch)
        alpha = _soa(alpha, torch)
        n = x.shape[1]
        if alpha.shape[1] != n:
            raise ValueError("x and alpha differ in length")
        self._check(self._lib.vm_set_stream(self._h, ctypes.c_void_p(self._stream_ptr(stream))))
        u = torch.empty((3, n), dtype=torch.float64, device=x.device)
        da = torch.empty((3, n), dtype=torch.float64, device=x.device) if want_dalpha else None
        J = torch.empty((9, n), dtype=torch.float64, device=x.device) if want_grad else None
        opts = self._opts(periodic, box_lo, box_len, "fp64", scheme, check_domain)
        self._check(self._lib.vm_fmm_eval_adaptive(self._h, n, ctypes.c_void_p(x.data_ptr()),
                                                   ctypes.c_void_p(alpha.data_ptr()), float(sigma), int(p),
                                                   int(ncrit), int(max_level), ctypes.byref(opts),
                                                   ctypes.c_void_p(u.data_ptr()),
                                                   ctypes.c_void_p(da.data_ptr() if da is not None else 0),
                                                   ctypes.c_void_p(J.data_ptr() if J is not None else 0)))
        return u, da, J

    def tune_ncrit(self, x, alpha, sigma, p, max_level, periodic=0, box_lo=(0.0, 0.0, 0.0), box_len=2 * math.pi,
                   reps=2, stream=None):
        """vm_tune_ncrit: (fastest ncrit, {ncrit: ms per evaluation})."""
        torch = self._torch
        x = _soa(x, torch)
        alpha = _soa(alpha, torch)
        n = x.shape[1]
        self._check(self._lib.vm_set_stream(self._h, ctypes.c_void_p(self._stream_ptr(stream))))
        opts = self._opts(periodic, box_lo, box_len, "fp64", "classic", False)
        best = ctypes.c_int()
        ms = np.zeros(8, np.float64)
        self._check(self._lib.vm_tune_ncrit(self._h, n, ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(alpha.data_ptr()), float(sigma), int(p), int(max_level),
                                            ctypes.byref(opts), int(reps), ctypes.byref(best),
                                            ctypes.c_void_p(ms.ctypes.data)))
        return best.value, {8 << i: float(v) for i, v in enumerate(ms) if v >= 0}

    def debug_adaptive(self, what):
        """vm_debug_adaptive: int64 array, (ncell, 6) cells, (m, 3) lists or (n,) permutation."""
        names = {"cells": 0, "p2p": 1, "m2l": 2, "m2p": 3, "p2l": 4, "perm": 5}
        w = names[what]
        rows = ctypes.c_int64()
        self._check(self._lib.vm_debug_adaptive(self._h, w, None, ctypes.byref(rows)))
        width = 6 if w == 0 else (1 if w == 5 else 3)
        out = np.zeros(max(rows.value, 1) * width, np.int32)
        self._check(self._lib.vm_debug_adaptive(self._h, w, ctypes.c_void_p(out.ctypes.data), ctypes.byref(rows)))
        out = out[:rows.value * width].astype(np.int64)
        return out if w == 5 else out.reshape(-1, width)

    def adjoint(self, x, alpha, u_bar, sigma, p, level, periodic=0, box_lo=(0.0, 0.0, 0.0),
                box_len=2 * math.pi, precision="fp64", want_x=True, want_alpha=True, stream=None,
                truncation="square", grad=None):
        """(x_bar, alpha_bar), each (3, n) or None: the transposed FMM applied to u_bar.

        With ``grad`` (the (9, n) gradient output of the context's last ``eval``
        of the same x and alpha) the forward state is reused instead of
        recomputed (``vm_fmm_adjoint_reuse``)."""
        torch = self._torch
        x = _soa(x, torch)
        alpha = _soa(alpha, torch)
        u_bar = _soa(u_bar, torch)
        n = x.shape[1]
        self._check(self._lib.vm_set_stream(self._h, ctypes.c_void_p(self._stream_ptr(stream))))
        xb = torch.empty((3, n), dtype=torch.float64, device=x.device) if want_x else None
        ab = torch.empty((3, n), dtype=torch.float64, device=x.device) if want_alpha else None
        opts = self._opts(periodic, box_lo, box_len, precision, "classic", False, truncation)
        if grad is not None:
            self._check(self._lib.vm_fmm_adjoint_reuse(
                self._h, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(alpha.data_ptr()), float(sigma), int(p),
                int(level), ctypes.byref(opts), ctypes.c_void_p(grad.data_ptr()), ctypes.c_void_p(u_bar.data_ptr()),
                ctypes.c_void_p(xb.data_ptr() if xb is not None else 0),
                ctypes.c_void_p(ab.data_ptr() if ab is not None else 0)))
            return xb, ab
        self._check(self._lib.vm_fmm_adjoint(self._h, n, ctypes.c_void_p(x.data_ptr()),
                                             ctypes.c_void_p(alpha.data_ptr()), float(sigma), int(p), int(level),
                                             ctypes.byref(opts), ctypes.c_void_p(u_bar.data_ptr()),
                                             ctypes.c_void_p(xb.data_ptr() if xb is not None else 0),
                                             ctypes.c_void_p(ab.data_ptr() if ab is not None else 0)))
        return xb, ab

    def _opts(self, periodic, box_lo, box_len, precision, scheme, check_domain, truncation="square"):
        return _lib.VmOpts((ctypes.c_double * 3)(*box_lo), float(box_len), int(periodic),
                           PRECISIONS[precision], SCHEMES[scheme], int(bool(check_domain)),
                           TRUNCATIONS[truncation])

    def rk2_step(self, x, alpha, sigma, p, level, dt, periodic=0, box_lo=(0.0, 0.0, 0.0),
                 box_len=2 * math.pi, precision="fp64", scheme="classic", want_initial=False,
                 stream=None, out=None, truncation="square"):
        """Heun step, in place on x and alpha ((3, n) contiguous float64 CUDA tensors).

        Returns (u0, J0) at the initial state when ``want_initial`` (written into
        ``out`` = (u0, J0) when given), else None."""
        torch = self._torch
        for t in (x, alpha):
            if t.dim() != 2 or t.shape[0] != 3 or not t.is_contiguous() or t.dtype != torch.float64:
                raise ValueError("rk2_step updates (3, n) contiguous float64 tensors in place")
        n = x.shape[1]
        self._check(self._lib.vm_set_stream(self._h, ctypes.c_void_p(self._stream_ptr(stream))))
        u0 = J0 = None
        if want_initial:
            if out is not None:
                u0, J0 = out
            else:
                u0 = torch.empty((3, n), dtype=torch.float64, device=x.device)
                J0 = torch.empty((9, n), dtype=torch.float64, device=x.device)
        opts = self._opts(periodic, box_lo, box_len, precision, scheme, False, truncation)
        self._check(self._lib.vm_rk2_step(self._h, n, ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(alpha.data_ptr()), float(sigma), int(p), int(level),
                                          ctypes.byref(opts), float(dt),
                                          ctypes.c_void_p(u0.data_ptr() if u0 is not None else 0),
                                          ctypes.c_void_p(J0.data_ptr() if J0 is not None else 0)))
        return (u0, J0) if want_initial else None

    def diagnostics(self, u, grad, alpha, h3, stream=None):
        """(E, Omega, Omega_p) as a float64 CUDA tensor of 3 (FP64 reductions)."""
        torch = self._torch
        n = u.shape[1]
        self._check(self._lib.vm_set_stream(self._h, ctypes.c_void_p(self._stream_ptr(stream))))
        out = torch.empty(3, dtype=torch.float64, device=u.device)
        self._check(self._lib.vm_diagnostics(self._h, n, ctypes.c_void_p(u.data_ptr()),
                                             ctypes.c_void_p(grad.data_ptr() if grad is not None else 0),
                                             ctypes.c_void_p(alpha.data_ptr() if alpha is not None else 0),
                                             float(h3), ctypes.c_void_p(out.data_ptr())))
        return out

    def diagnostics_noalloc(self, u, grad, alpha, h3, out, stream=None):
        """vm_diagnostics_noalloc: (E, Omega, Omega_p) written into `out` (a float64
        CUDA tensor of 3 the caller owns); the library allocates nothing."""
        n = u.shape[1]
        self._check(self._lib.vm_set_stream(self._h, ctypes.c_void_p(self._stream_ptr(stream))))
        self._check(self._lib.vm_diagnostics_noalloc(self._h, n, ctypes.c_void_p(u.data_ptr()),
                                                     ctypes.c_void_p(grad.data_ptr() if grad is not None else 0),
                                                     ctypes.c_void_p(alpha.data_ptr() if alpha is not None else 0),
                                                     float(h3), ctypes.c_void_p(out.data_ptr())))
        return out

    def gauss_sum(self, x, gamma, sigma, level, periodic=0, box_lo=(0.0, 0.0, 0.0), box_len=2 * math.pi,
                  precision="fp64", stream=None, out=None):
        """Gaussian smoothing sum over the neighbour list, (3, n) float64."""
        torch = self._torch
        x = _soa(x, torch)
        gamma = _soa(gamma, torch)
        n = x.shape[1]
        if gamma.shape[1] != n:
            raise ValueError("x and gamma differ in length")
        self._check(self._lib.vm_set_stream(self._h, ctypes.c_void_p(self._stream_ptr(stream))))
        om = torch.empty((3, n), dtype=torch.float64, device=x.device) if out is None else out
        opts = self._opts(periodic, box_lo, box_len, precision, "classic", False)
        self._check(self._lib.vm_gauss_sum(self._h, n, ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(gamma.data_ptr()), float(sigma), int(level),
                                           ctypes.byref(opts), ctypes.c_void_p(om.data_ptr())))
        return om

    def gauss_eval(self, x, gamma, y, sigma, level, periodic=0, box_lo=(0.0, 0.0, 0.0), box_len=2 * math.pi,
                   precision="fp64", stream=None, out=None):
        """Gaussian sum of the particles (x, gamma) at the points y, (3, m) float64."""
        torch = self._torch
        x = _soa(x, torch)
        gamma = _soa(gamma, torch)
        y = _soa(y, torch)
        n, m = x.shape[1], y.shape[1]
        if gamma.shape[1] != n:
            raise ValueError("x and gamma differ in length")
        self._check(self._lib.vm_set_stream(self._h, ctypes.c_void_p(self._stream_ptr(stream))))
        om = torch.empty((3, m), dtype=torch.float64, device=x.device) if out is None else out
        opts = self._opts(periodic, box_lo, box_len, precision, "classic", False)
        self._check(self._lib.vm_gauss_eval(self._h, n, ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(gamma.data_ptr()), m, ctypes.c_void_p(y.data_ptr()),
                                            float(sigma), int(level), ctypes.byref(opts),
                                            ctypes.c_void_p(om.data_ptr())))
        return om

    def reinit(self, x, alpha, sigma, ng, sigma0, level, tol=1e-3, max_iter=100, periodic=0,
               box_lo=(0.0, 0.0, 0.0), box_len=2 * math.pi, precision="fp64", stream=None):
        """Reinitialisation onto the ng^3 lattice, in place on x and alpha ((3, n)
        contiguous float64 CUDA tensors); returns (iters, resid) of the solve."""
        torch = self._torch
        self._inplace(x, alpha)
        n = x.shape[1]
        self._check(self._lib.vm_set_stream(self._h, ctypes.c_void_p(self._stream_ptr(stream))))
        opts = self._opts(periodic, box_lo, box_len, precision, "classic", False)
        iters = ctypes.c_int(0)
        resid = ctypes.c_double(0.0)
        self._check(self._lib.vm_reinit(self._h, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(alpha.data_ptr()),
                                        float(sigma), int(ng), float(sigma0), int(level), ctypes.byref(opts),
                                        float(tol), int(max_iter), ctypes.byref(iters), ctypes.byref(resid)))
        return iters.value, resid.value

    def run(self, x, alpha, sigma, p, level, dt, steps, nu=0.0, integrator="euler", reinit_every=0, ng=0,
            tol=1e-3, max_iter=100, periodic=0, box_lo=(0.0, 0.0, 0.0), box_len=2 * math.pi, precision="fp64",
            scheme="classic", want_diag=False, stream=None, truncation="square"):
        """The time loop, in place on x and alpha.  Returns (sigma at the end,
        diagnostics (steps, 3) CUDA tensor or None, GMRES products, largest
        relative residual of the reinitialisations)."""
        torch = self._torch
        self._inplace(x, alpha)
        n = x.shape[1]
        self._check(self._lib.vm_set_stream(self._h, ctypes.c_void_p(self._stream_ptr(stream))))
        opts = self._opts(periodic, box_lo, box_len, precision, scheme, False, truncation)
        loop = _lib.VmLoop(INTEGRATORS[integrator], float(dt), float(nu), int(steps), int(reinit_every), int(ng),
                           float(tol), int(max_iter))
        diag = torch.empty((max(steps, 1), 3), dtype=torch.float64, device=x.device) if want_diag else None
        sg = ctypes.c_double(float(sigma))
        prods = ctypes.c_int(0)
        resid = ctypes.c_double(0.0)
        self._check(self._lib.vm_run(self._h, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(alpha.data_ptr()),
                                     ctypes.byref(sg), int(p), int(level), ctypes.byref(opts), ctypes.byref(loop),
                                     ctypes.c_void_p(diag.data_ptr() if diag is not None else 0),
                                     ctypes.byref(prods), ctypes.byref(resid)))
        return sg.value, (diag[:steps] if diag is not None else None), prods.value, resid.value

    def tune_level(self, x, alpha, sigma, p, periodic=0, box_lo=(0.0, 0.0, 0.0), box_len=2 * math.pi,
                   precision="mixed", min_leaf_sigmas=4.0, reps=2, truncation="square", stream=None):
        """Fastest admissible leaf level for these particles: (level, {level: ms})."""
        torch = self._torch
        x = _soa(x, torch)
        alpha = _soa(alpha, torch)
        n = x.shape[1]
        self._check(self._lib.vm_set_stream(self._h, ctypes.c_void_p(self._stream_ptr(stream))))
        opts = self._opts(periodic, box_lo, box_len, precision, "classic", False, truncation)
        level = ctypes.c_int(-1)
        ms = np.zeros(11, np.float64)
        self._check(self._lib.vm_tune_level(self._h, n, ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(alpha.data_ptr()), float(sigma), int(p),
                                            ctypes.byref(opts), float(min_leaf_sigmas), int(reps),
                                            ctypes.byref(level), ctypes.c_void_p(ms.ctypes.data)))
        return level.value, {l: float(v) for l, v in enumerate(ms) if v >= 0}

    def energy_spectrum(self, u, ng, kmax, stream=None):
        """Shell energy spectrum E[0..kmax] (CUDA float64) of a velocity (3, ng^3)
        on the ng^3 lattice of the periodic cube (x index slowest)."""
        torch = self._torch
        u = _soa(u, torch)
        if u.shape[1] != ng ** 3:
            raise ValueError("u must hold ng^3 lattice points")
        self._check(self._lib.vm_set_stream(self._h, ctypes.c_void_p(self._stream_ptr(stream))))
        E = torch.empty(kmax + 1, dtype=torch.float64, device=u.device)
        self._check(self._lib.vm_energy_spectrum(self._h, int(ng), ctypes.c_void_p(u.data_ptr()), int(kmax),
                                                 ctypes.c_void_p(E.data_ptr())))
        return E

    def _inplace(self, x, alpha):
        torch = self._torch
        for t in (x, alpha):
            if t.dim() != 2 or t.shape[0] != 3 or not t.is_contiguous() or t.dtype != torch.float64 or not t.is_cuda:
                raise ValueError("x and alpha are updated in place: (3, n) contiguous float64 CUDA tensors")

    def rbf_solve(self, x, omega, sigma, h3, level, tol=1e-3, max_iter=100, periodic=0, box_lo=(0.0, 0.0, 0.0),
                  box_len=2 * math.pi, precision="fp64", stream=None, out=None):
        """Strengths (3, n) float64 reproducing omega at the particles, with the
        products spent and the relative residual reached: (gamma, iters, resid)."""
        torch = self._torch
        x = _soa(x, torch)
        omega = _soa(omega, torch)
        n = x.shape[1]
        if omega.shape[1] != n:
            raise ValueError("x and omega differ in length")
        self._check(self._lib.vm_set_stream(self._h, ctypes.c_void_p(self._stream_ptr(stream))))
        gam = torch.empty((3, n), dtype=torch.float64, device=x.device) if out is None else out
        opts = self._opts(periodic, box_lo, box_len, precision, "classic", False)
        iters = ctypes.c_int(0)
        resid = ctypes.c_double(0.0)
        self._check(self._lib.vm_rbf_solve(self._h, n, ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(omega.data_ptr()), float(sigma), float(h3), int(level),
                                           ctypes.byref(opts), float(tol), int(max_iter),
                                           ctypes.c_void_p(gam.data_ptr()), ctypes.byref(iters),
                                           ctypes.byref(resid)))
        return gam, iters.value, resid.value

    def set_timing(self, enable=True):
        self._check(self._lib.vm_set_timing(self._h, int(bool(enable))))

    def timing(self):
        """{phase: (milliseconds, launches)} of the last timed evaluation."""
        ms = np.zeros(len(_lib.PHASES), np.float64)
        cnt = np.zeros(len(_lib.PHASES), np.int32)
        self._check(self._lib.vm_get_timing(self._h, ctypes.c_void_p(ms.ctypes.data),
                                            ctypes.c_void_p(cnt.ctypes.data)))
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(_lib.PHASES)}

    def debug_tree(self, n, level):
        torch = self._torch
        keys = torch.empty(n, dtype=torch.int32, device="cuda")
        perm = torch.empty(n, dtype=torch.int32, device="cuda")
        start = torch.empty((1 << (3 * level)) + 1, dtype=torch.int32, device="cuda")
        self._check(self._lib.vm_debug_tree(self._h, ctypes.c_void_p(keys.data_ptr()),
                                            ctypes.c_void_p(perm.data_ptr()),
                                            ctypes.c_void_p(start.data_ptr())))
        torch.cuda.synchronize()
        return (keys.cpu().numpy().view(np.uint32).astype(np.int64), perm.cpu().numpy().astype(np.int64),
                start.cpu().numpy().astype(np.int64))

    def debug_expansions(self, which, level, p, mixed=False):
        """Multipoles (which=0) or locals (1) at `level`: array (8^level, 3, C)."""
        torch = self._torch
        nbytes = ctypes.c_int64()
        self._check(self._lib.vm_debug_expansions(self._h, which, level, None, ctypes.byref(nbytes)))
        buf = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        self._check(self._lib.vm_debug_expansions(self._h, which, level, ctypes.c_void_p(buf.data_ptr()),
                                                  ctypes.byref(nbytes)))
        torch.cuda.synchronize()
        C = (p + 1) ** 2
        kp = (C + 31) // 32 * 32
        arr = buf.cpu().numpy().view(np.float32 if mixed else np.float64).reshape(-1, 3, kp)
        return arr[:, :, :C].astype(np.float64)

    def debug_far(self, n):
        torch = self._torch
        out = torch.empty((12, n), dtype=torch.float64, device="cuda")
        self._check(self._lib.vm_debug_far(self._h, ctypes.c_void_p(out.data_ptr())))
        torch.cuda.synchronize()
        return out.cpu().numpy()


# keyword arguments of FMM.eval that velocity() passes on, and the subset the
# adjoint takes (the stretching form does not enter u)
_VELOCITY_KW = {"periodic", "box_lo", "box_len", "precision", "scheme", "check_domain", "stream", "truncation"}
_ADJOINT_KW = {"periodic", "box_lo", "box_len", "precision", "stream", "truncation"}


def _velocity_function():
    import torch

    class VortexFMM(torch.autograd.Function):
        """u = FMM(x, alpha); backward runs the library's transposed FMM."""

        @staticmethod
        def forward(ctx, x, alpha, fmm, kw):
            # The SoA tensors the library reads are kept for the backward pass: while
            # they are alive no other allocation can take their addresses, so the
            # library's check that its last evaluation was this one (the x and alpha
            # addresses among the arguments) cannot be fooled by a temporary copy
            # of a later call landing at the same address.
            xs = _soa(x, torch)
            als = _soa(alpha, torch)
            need = ctx.needs_input_grad[0] or ctx.needs_input_grad[1]
            # the gradient output lets the backward pass reuse this evaluation's tree
            u, _, J = fmm.eval(xs, als, want_dalpha=False, want_grad=need, **kw)
            ctx.save_for_backward(xs, als)
            ctx.fmm = fmm
            ctx.kw = kw
            ctx.J = J
            ctx.versions = (xs._version, als._version)
            ctx.aos = (x.shape[0] != 3, alpha.shape[0] != 3)
            return u

        @staticmethod
        def backward(ctx, u_bar):
            xs, als = ctx.saved_tensors
            kw = {k: v for k, v in ctx.kw.items() if k in _ADJOINT_KW or k in ("sigma", "p", "level")}
            args = dict(want_x=ctx.needs_input_grad[0], want_alpha=ctx.needs_input_grad[1], **kw)
            u_bar = u_bar.contiguous()
            xb = ab = None
            if ctx.J is not None and ctx.versions == (xs._version, als._version):
                try:
                    xb, ab = ctx.fmm.adjoint(xs, als, u_bar, grad=ctx.J, **args)
                except _lib.VmError as e:
                    # the context evaluated something else since the forward pass
                    if e.status != _lib.VM_EINVAL:
                        raise
            if xb is None and ab is None:
                xb, ab = ctx.fmm.adjoint(xs, als, u_bar, **args)
            # gradients in the layout of the inputs
            if xb is not None and ctx.aos[0]:
                xb = xb.t()
            if ab is not None and ctx.aos[1]:
                ab = ab.t()
            return xb, ab, None, None

    return VortexFMM


_VORTEX_FMM = None


def velocity(x, alpha, fmm, sigma, p, level, **kw):
    """Differentiable velocity (3, n) of particles x, alpha (float64 CUDA tensors,
    (3, n) or (n, 3); gradients come back in the inputs' layout).

    Gradients with respect to x and alpha come from the discrete adjoint of the
    same FMM (``vm_fmm_adjoint``, or ``vm_fmm_adjoint_reuse`` when the context's
    last evaluation is still this one).  Keyword arguments: those of ``FMM.eval``
    that describe the evaluation -- periodic, box_lo, box_len, precision,
    scheme, check_domain, stream, truncation."""
    global _VORTEX_FMM
    bad = set(kw) - _VELOCITY_KW
    if bad:
        raise TypeError("velocity() does not take " + ", ".join(sorted(bad)))
    if _VORTEX_FMM is None:
        _VORTEX_FMM = _velocity_function()
    kw = dict(kw, sigma=sigma, p=p, level=level)
    return _VORTEX_FMM.apply(x, alpha, fmm, kw)


def debug_offsets():
    lib = _lib.load()
    out = np.zeros((316, 3), np.int8)
    cnt = ctypes.c_int()
    st = lib.vm_debug_offsets(out.ctypes.data, ctypes.byref(cnt))
    if st != _lib.VM_OK:
        raise _lib.VmError(st, "vm_debug_offsets")
    return out[:cnt.value]


def debug_list(level, periodic, key):
    lib = _lib.load()
    src = np.zeros(189, np.int32)
    d = np.zeros((189, 3), np.int8)
    img = np.zeros((189, 3), np.int8)
    cnt = ctypes.c_int()
    st = lib.vm_debug_list(int(level), int(periodic), int(key), src.ctypes.data, d.ctypes.data,
                           img.ctypes.data, ctypes.byref(cnt))
    if st != _lib.VM_OK:
        raise _lib.VmError(st, "vm_debug_list")
    c = cnt.value
    return src[:c].copy(), d[:c].copy(), img[:c].copy()


def debug_operator(kind, p, index):
    lib = _lib.load()
    C = (p + 1) ** 2
    out = np.zeros((3 * p * p if kind == 4 else C, C), np.float64)
    st = lib.vm_debug_operator(int(kind), int(p), int(index), out.ctypes.data)
    if st != _lib.VM_OK:
        raise _lib.VmError(st, "vm_debug_operator")
    return out
