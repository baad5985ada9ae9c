"""ctypes binding to libctrlalm.so (the C ABI of include/ct.h).

Argument marshalling only: every step of the reconstruction runs in the library's HIP kernels. Tensors
are torch CUDA (HIP) tensors; their data pointers and torch's current stream are passed through.
The binding raises if the shared library is missing or fails to load -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctrlalm.so")

CT_OK, CT_ERR_INVALID_ARG, CT_ERR_OOM, CT_ERR_HIP, CT_ERR_UNSUPPORTED, CT_ERR_DIVERGED = range(6)
STATUS_NAMES = {0: "CT_OK", 1: "CT_ERR_INVALID_ARG", 2: "CT_ERR_OOM", 3: "CT_ERR_HIP", 4: "CT_ERR_UNSUPPORTED",
                5: "CT_ERR_DIVERGED"}

#: Every entry point declared in include/ct.h.
EXPORTS = ("ct_geom_create", "ct_geom_destroy", "ct_forward", "ct_forward_noalloc", "ct_back", "ct_fbp", "ct_rlalm_params_default",
           "ct_rlalm_solve", "ct_rlalm_solve_batched", "ct_rlalm_prepare", "ct_rlalm_init", "ct_rlalm_iterate",
           "ct_rlalm_kernel_times", "ct_rlalm_status", "ct_cost", "ct_last_error", "ct_unet_num_params",
           "ct_unet_create", "ct_unet_destroy", "ct_unet_set_params", "ct_helix_create", "ct_helix_destroy",
           "ct_helix_forward", "ct_helix_back", "ct_helix_solve", "ct_unet_get_params", "ct_unet_forward", "ct_unet_gradient", "ct_unet_train_step",
           "ct_unet_input")


class GeomDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("nb", ctypes.c_int), ("du", ctypes.c_double), ("u_offset", ctypes.c_double), ("det", ctypes.c_int),
                ("nviews", ctypes.c_int), ("beta0", ctypes.c_double), ("span", ctypes.c_double),
                ("dso", ctypes.c_double), ("dsd", ctypes.c_double), ("nsubsets", ctypes.c_int),
                ("storage", ctypes.c_int)]


class RlalmParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("niters", ctypes.c_int), ("rho_mode", ctypes.c_int),
                ("rho_fixed", ctypes.c_double), ("potential", ctypes.c_int), ("delta", ctypes.c_double),
                ("beta", ctypes.c_double), ("huber", ctypes.c_int), ("algorithm", ctypes.c_int),
                ("subset_order", ctypes.c_int), ("kappa", ctypes.c_int), ("start", ctypes.c_int),
                ("init_full", ctypes.c_int), ("dl_scale", ctypes.c_double), ("x_ref", ctypes.c_void_p),
                ("mu_water", ctypes.c_double), ("fov_radius", ctypes.c_double), ("use_graph", ctypes.c_int),
                ("time_kernels", ctypes.c_int), ("unet", ctypes.c_void_p), ("forward_split", ctypes.c_int),
                ("diverge_factor", ctypes.c_double), ("diverge_window", ctypes.c_int)]


class HelixDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("dx", ctypes.c_double),
                ("dy", ctypes.c_double), ("dz", ctypes.c_double), ("zc", ctypes.c_double), ("nb", ctypes.c_int),
                ("du", ctypes.c_double), ("u_offset", ctypes.c_double), ("nr", ctypes.c_int), ("dw", ctypes.c_double),
                ("w_offset", ctypes.c_double), ("nviews", ctypes.c_int), ("views_per_turn", ctypes.c_int),
                ("beta0", ctypes.c_double), ("z0", ctypes.c_double), ("feed", ctypes.c_double),
                ("dso", ctypes.c_double), ("dsd", ctypes.c_double), ("nsubsets", ctypes.c_int)]


class KernelTimes(ctypes.Structure):
    _fields_ = [("n_forward", ctypes.c_longlong), ("n_update", ctypes.c_longlong), ("ms_forward", ctypes.c_double),
                ("ms_update", ctypes.c_double)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("fp_waves", ctypes.c_int), ("largest_first", ctypes.c_int), ("ms_subiteration", ctypes.c_double),
                ("persistent", ctypes.c_int), ("blocks_per_cu", ctypes.c_int), ("forward_split", ctypes.c_int)]


class TraceRow(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int), ("seconds", ctypes.c_double), ("rmsd_hu", ctypes.c_double),
                ("rho", ctypes.c_double), ("finite", ctypes.c_int), ("rmsd_hu_all", ctypes.c_double),
                ("cost", ctypes.c_double)]


class CtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load libctrlalm.so (raises FileNotFoundError / OSError when it is absent or broken)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(f"{LIB_PATH} is missing: build it with paper_1512_04564_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong
    L.ct_geom_create.argtypes = [ctypes.POINTER(GeomDesc), ctypes.POINTER(vp)]
    L.ct_geom_destroy.argtypes = [vp]
    L.ct_geom_destroy.restype = None
    L.ct_forward.argtypes = [vp, i, vp, vp, vp]
    L.ct_forward_noalloc.argtypes = [vp, i, vp, vp, vp]
    L.ct_back.argtypes = [vp, i, vp, vp, vp]
    L.ct_fbp.argtypes = [vp, vp, vp, vp]
    L.ct_rlalm_params_default.argtypes = [ctypes.POINTER(RlalmParams)]
    L.ct_rlalm_params_default.restype = None
    L.ct_rlalm_solve.argtypes = [vp, ctypes.POINTER(RlalmParams), vp, vp, vp, ctypes.POINTER(TraceRow), vp]
    L.ct_rlalm_solve_batched.argtypes = [ctypes.POINTER(vp), i, ctypes.POINTER(RlalmParams), ctypes.POINTER(vp),
                                         ctypes.POINTER(vp), ctypes.POINTER(vp), i, ctypes.POINTER(BatchConfig), vp]
    L.ct_rlalm_prepare.argtypes = [vp, ctypes.POINTER(RlalmParams), vp, vp, vp, vp]
    L.ct_rlalm_init.argtypes = [vp, ctypes.POINTER(RlalmParams), vp, vp, vp, vp, vp, vp, vp]
    L.ct_rlalm_iterate.argtypes = [vp, ctypes.POINTER(RlalmParams), vp, vp, vp, vp, vp, vp, vp, ll, ll, vp]
    L.ct_rlalm_kernel_times.argtypes = [vp, ctypes.POINTER(KernelTimes)]
    L.ct_rlalm_status.argtypes = [vp]
    L.ct_cost.argtypes = [vp, ctypes.POINTER(RlalmParams), vp, vp, vp, vp, vp, vp]
    L.ct_last_error.restype = ctypes.c_char_p
    L.ct_helix_create.argtypes = [ctypes.POINTER(HelixDesc), ctypes.POINTER(vp)]
    L.ct_helix_destroy.argtypes = [vp]
    L.ct_helix_destroy.restype = None
    L.ct_helix_forward.argtypes = [vp, i, vp, vp, vp]
    L.ct_helix_back.argtypes = [vp, i, vp, vp, vp]
    L.ct_helix_solve.argtypes = [vp, ctypes.POINTER(RlalmParams), vp, vp, vp, vp]
    fp, u8p, dp = ctypes.POINTER(ctypes.c_float), vp, ctypes.POINTER(ctypes.c_double)
    L.ct_unet_num_params.argtypes = []
    L.ct_unet_create.argtypes = [vp, i, i, i, ctypes.POINTER(vp)]
    L.ct_unet_destroy.argtypes = [vp]
    L.ct_unet_destroy.restype = None
    L.ct_unet_set_params.argtypes = [vp, vp]
    L.ct_unet_get_params.argtypes = [vp, vp]
    L.ct_unet_forward.argtypes = [vp, vp, vp, i, i, i, vp]
    L.ct_unet_gradient.argtypes = [vp, vp, vp, u8p, i, i, i, dp, vp, vp]
    L.ct_unet_train_step.argtypes = [vp, vp, vp, u8p, i, i, i, ctypes.c_float, dp, vp]
    L.ct_unet_input.argtypes = [vp, vp, ctypes.c_double, vp, vp]
    for name in EXPORTS:
        if name not in ("ct_geom_destroy", "ct_rlalm_params_default", "ct_last_error", "ct_unet_destroy",
                        "ct_unet_num_params", "ct_helix_destroy"):
            getattr(L, name).restype = ctypes.c_int
    L.ct_unet_num_params.restype = ctypes.c_size_t
    _lib = L
    return L


def check(status: int) -> None:
    if status != CT_OK:
        msg = load().ct_last_error()
        raise CtError(status, msg.decode() if msg else "")
