"""ctypes binding of ``libvmfmm.so`` (argument marshalling only).

The library is built in-tree by ``paper_1110_2921_amd.build``; if it is
missing the import of the product path fails loudly, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvmfmm.so")

PHASES = ("tree", "p2m", "m2m", "lattice", "l2l", "m2l", "l2p", "p2p", "gauss", "krylov", "lists", "p2l", "m2p")

VM_OK, VM_EINVAL, VM_ENOMEM, VM_EDEVICE, VM_EDOMAIN = 0, -1, -2, -3, -4
STATUS_NAMES = {0: "VM_OK", -1: "VM_EINVAL", -2: "VM_ENOMEM", -3: "VM_EDEVICE", -4: "VM_EDOMAIN"}

# every symbol include/vmfmm.h declares
EXPORTS = ("vm_create", "vm_destroy", "vm_set_stream", "vm_last_error", "vm_fmm_eval", "vm_fmm_eval_at", "vm_fmm_eval_adaptive", "vm_tune_ncrit",
           "vm_fmm_adjoint", "vm_fmm_adjoint_reuse", "vm_rk2_step", "vm_diagnostics", "vm_diagnostics_noalloc", "vm_gauss_sum", "vm_gauss_eval", "vm_rbf_solve",
           "vm_reinit", "vm_run", "vm_energy_spectrum", "vm_tune_level",
           "vm_set_timing", "vm_get_timing", "vm_debug_tree", "vm_debug_expansions", "vm_debug_far", "vm_debug_offsets", "vm_debug_list", "vm_debug_adaptive",
           "vm_debug_operator")


class VmOpts(ctypes.Structure):
    _fields_ = [("box_lo", ctypes.c_double * 3), ("box_len", ctypes.c_double),
                ("periodic", ctypes.c_int), ("precision", ctypes.c_int), ("scheme", ctypes.c_int),
                ("check_domain", ctypes.c_int), ("truncation", ctypes.c_int)]


class VmLoop(ctypes.Structure):
    _fields_ = [("integrator", ctypes.c_int), ("dt", ctypes.c_double), ("nu", ctypes.c_double),
                ("steps", ctypes.c_int), ("reinit_every", ctypes.c_int), ("ng", ctypes.c_int),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int)]


class VmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_LIB = None


def load():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1110_2921_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p
    lib.vm_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, vp]
    lib.vm_create.restype = ctypes.c_int
    lib.vm_destroy.argtypes = [vp]
    lib.vm_destroy.restype = None
    lib.vm_set_stream.argtypes = [vp, vp]
    lib.vm_set_stream.restype = ctypes.c_int
    lib.vm_last_error.argtypes = [vp]
    lib.vm_last_error.restype = ctypes.c_char_p
    lib.vm_fmm_eval.argtypes = [vp, i64, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(VmOpts), dp, dp, dp]
    lib.vm_fmm_eval.restype = ctypes.c_int
    lib.vm_fmm_adjoint_reuse.argtypes = [vp, i64, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(VmOpts), dp, dp, dp, dp]
    lib.vm_fmm_adjoint_reuse.restype = ctypes.c_int
    lib.vm_fmm_eval_at.argtypes = [vp, i64, dp, dp, i64, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(VmOpts), dp, dp]
    lib.vm_fmm_eval_at.restype = ctypes.c_int
    lib.vm_fmm_eval_adaptive.argtypes = [vp, i64, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(VmOpts), dp, dp, dp]
    lib.vm_fmm_eval_adaptive.restype = ctypes.c_int
    lib.vm_tune_ncrit.argtypes = [vp, i64, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(VmOpts), ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp]
    lib.vm_tune_ncrit.restype = ctypes.c_int
    lib.vm_debug_adaptive.argtypes = [vp, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int64)]
    lib.vm_debug_adaptive.restype = ctypes.c_int
    lib.vm_fmm_adjoint.argtypes = [vp, i64, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(VmOpts), dp, dp, dp]
    lib.vm_fmm_adjoint.restype = ctypes.c_int
    lib.vm_rk2_step.argtypes = [vp, i64, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(VmOpts), ctypes.c_double, dp, dp]
    lib.vm_rk2_step.restype = ctypes.c_int
    lib.vm_diagnostics.argtypes = [vp, i64, dp, dp, dp, ctypes.c_double, dp]
    lib.vm_diagnostics.restype = ctypes.c_int
    lib.vm_diagnostics_noalloc.argtypes = [vp, i64, dp, dp, dp, ctypes.c_double, dp]
    lib.vm_diagnostics_noalloc.restype = ctypes.c_int
    lib.vm_gauss_sum.argtypes = [vp, i64, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(VmOpts), dp]
    lib.vm_gauss_sum.restype = ctypes.c_int
    lib.vm_gauss_eval.argtypes = [vp, i64, dp, dp, i64, dp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(VmOpts),
                                  dp]
    lib.vm_gauss_eval.restype = ctypes.c_int
    lib.vm_reinit.argtypes = [vp, i64, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                              ctypes.POINTER(VmOpts), ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                              ctypes.POINTER(ctypes.c_double)]
    lib.vm_reinit.restype = ctypes.c_int
    lib.vm_run.argtypes = [vp, i64, dp, dp, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int,
                           ctypes.POINTER(VmOpts), ctypes.POINTER(VmLoop), dp, ctypes.POINTER(ctypes.c_int),
                           ctypes.POINTER(ctypes.c_double)]
    lib.vm_run.restype = ctypes.c_int
    lib.vm_rbf_solve.argtypes = [vp, i64, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 ctypes.POINTER(VmOpts), ctypes.c_double, ctypes.c_int, dp,
                                 ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
    lib.vm_rbf_solve.restype = ctypes.c_int
    lib.vm_tune_level.argtypes = [vp, i64, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(VmOpts),
                                  ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_void_p]
    lib.vm_tune_level.restype = ctypes.c_int
    lib.vm_energy_spectrum.argtypes = [vp, ctypes.c_int, dp, ctypes.c_int, dp]
    lib.vm_energy_spectrum.restype = ctypes.c_int
    lib.vm_set_timing.argtypes = [vp, ctypes.c_int]
    lib.vm_set_timing.restype = ctypes.c_int
    lib.vm_get_timing.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p]
    lib.vm_get_timing.restype = ctypes.c_int
    lib.vm_debug_tree.argtypes = [vp, dp, dp, dp]
    lib.vm_debug_tree.restype = ctypes.c_int
    lib.vm_debug_expansions.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(ctypes.c_int64)]
    lib.vm_debug_expansions.restype = ctypes.c_int
    lib.vm_debug_far.argtypes = [vp, vp]
    lib.vm_debug_far.restype = ctypes.c_int
    lib.vm_debug_offsets.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]
    lib.vm_debug_offsets.restype = ctypes.c_int
    lib.vm_debug_list.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]
    lib.vm_debug_list.restype = ctypes.c_int
    lib.vm_debug_operator.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    lib.vm_debug_operator.restype = ctypes.c_int
    _LIB = lib
    return lib
