"""ctypes binding of libfdtd.so (C ABI declared in include/fdtd.h).

Argument marshalling only: every step of the time-stepping runs in the HIP
library.  Loading fails loudly if the compiled library is absent.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdtd.so")

FDTD_OK = 0
STATUS = {0: "FDTD_OK", -1: "FDTD_EINVAL", -2: "FDTD_ENOMEM", -3: "FDTD_EDEVICE",
          -4: "FDTD_EUNSUPPORTED", -5: "FDTD_ENONFINITE", -6: "FDTD_ENOTCONVERGED"}
SCHEMES = {"adi": 0, "lod1": 1, "ss1": 1, "ss2": 2, "lod2": 3,
           "dyakonov": 4, "dy": 4, "douglas_gunn": 5, "dg": 5, "crank_nicolson": 6, "cn": 6}
FORMS = {"fundamental": 0, "conventional": 1}
DTYPES = {"f32": 0, "f64": 1, "f32_f64solve": 2, "f32_refine": 3, "f32_plain": 4}

EXPORTS = ("fdtd_plan", "fdtd_get_refined", "fdtd_set_graph", "fdtd_set_order", "fdtd_set_stencil",
           "fdtd_stencil_optimized", "fdtd_run", "fdtd_step", "fdtd_set_step",
           "fdtd_set_timing",
           "fdtd_last_timing", "fdtd_get_kernel_config", "fdtd_set_kernel_config", "fdtd_autotune",
           "fdtd_grad_eps", "fdtd_plan_batch", "fdtd_run_batch", "fdtd_diff_norm", "fdtd_diff_norm_noalloc",
           "fdtd_set_cg", "fdtd_last_cg", "fdtd_destroy", "fdtd_strerror")


class FdtdDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("dt", ctypes.c_double), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("dz", ctypes.c_double), ("scheme", ctypes.c_int), ("form", ctypes.c_int),
                ("dtype", ctypes.c_int), ("eps_r", ctypes.c_void_p), ("mu_r", ctypes.c_void_p),
                ("boundary", ctypes.c_int)]


class FdtdSource(ctypes.Structure):
    _fields_ = [("i", ctypes.c_int), ("j", ctypes.c_int), ("k", ctypes.c_int),
                ("f0", ctypes.c_double), ("tau", ctypes.c_double), ("t0", ctypes.c_double),
                ("amp", ctypes.c_double)]


class FdtdKernelConfig(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int), ("tile_x", ctypes.c_int), ("block_threads", ctypes.c_int),
                ("remap", ctypes.c_int)]


class FdtdError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)}")


_lib = None


def lib() -> ctypes.CDLL:
    """Load libfdtd.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.fdtd_plan.argtypes = [ctypes.POINTER(FdtdDesc), vp, ctypes.POINTER(vp)]
    L.fdtd_get_refined.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    L.fdtd_set_graph.argtypes = [vp, ctypes.c_int]
    L.fdtd_set_order.argtypes = [vp, ctypes.c_int]
    L.fdtd_set_stencil.argtypes = [vp, ctypes.c_double]
    L.fdtd_stencil_optimized.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    L.fdtd_run.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int,
                           ctypes.POINTER(FdtdSource), ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    L.fdtd_step.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(FdtdSource)]
    L.fdtd_set_step.argtypes = [vp, ctypes.c_longlong]
    L.fdtd_set_timing.argtypes = [vp, ctypes.c_int]
    L.fdtd_last_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int)]
    L.fdtd_get_kernel_config.argtypes = [vp, ctypes.c_int, ctypes.POINTER(FdtdKernelConfig)]
    L.fdtd_set_kernel_config.argtypes = [vp, ctypes.c_int, ctypes.POINTER(FdtdKernelConfig)]
    L.fdtd_autotune.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    L.fdtd_grad_eps.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int,
                                ctypes.POINTER(FdtdSource), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.POINTER(ctypes.c_double), vp]
    L.fdtd_plan_batch.argtypes = [ctypes.POINTER(FdtdDesc), ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.fdtd_run_batch.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int]
    L.fdtd_diff_norm.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                 ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_double)]
    L.fdtd_diff_norm_noalloc.argtypes = L.fdtd_diff_norm.argtypes
    L.fdtd_set_cg.argtypes = [vp, ctypes.c_double, ctypes.c_int]
    L.fdtd_last_cg.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double)]
    L.fdtd_destroy.argtypes = [vp]
    L.fdtd_strerror.argtypes = [ctypes.c_int]
    L.fdtd_strerror.restype = ctypes.c_char_p
    for name in ("fdtd_plan", "fdtd_get_refined", "fdtd_set_graph", "fdtd_set_order", "fdtd_set_stencil",
                 "fdtd_stencil_optimized", "fdtd_run", "fdtd_step", "fdtd_set_step", "fdtd_set_timing",
                 "fdtd_last_timing", "fdtd_get_kernel_config", "fdtd_set_kernel_config", "fdtd_autotune",
                 "fdtd_grad_eps", "fdtd_plan_batch", "fdtd_run_batch", "fdtd_diff_norm", "fdtd_diff_norm_noalloc",
                 "fdtd_set_cg", "fdtd_last_cg", "fdtd_destroy"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(status: int, what: str) -> None:
    if status != FDTD_OK:
        raise FdtdError(status, what)
