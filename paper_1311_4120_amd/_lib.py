"""ctypes view of the C ABI in include/jgb.h (argument marshalling only).

Loads the in-tree libjgb.so; there is no fallback: if the library is missing
or does not load, importing this module raises ImportError.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjgb.so")

JGB_OK = 0
JGB_ERR_INVALID_ARG = 1
JGB_ERR_UNSUPPORTED = 2
JGB_ERR_OUT_OF_MEMORY = 3
JGB_ERR_DEVICE = 4
STATUS_NAMES = {0: "JGB_OK", 1: "JGB_ERR_INVALID_ARG", 2: "JGB_ERR_UNSUPPORTED",
                3: "JGB_ERR_OUT_OF_MEMORY", 4: "JGB_ERR_DEVICE"}

COULOMB_3D, COULOMB_2D, DIPOLE_3D, DIPOLE_2D, POISSON_2D = 0, 1, 2, 3, 4
NUM_STAGES = 13
STAGE_NAMES = ["fwd_fft_z", "fwd_fft_y", "fwd_fft_x", "interp", "spread", "spread_reduce",
               "inv_fft_x", "inv_fft_y", "inv_fft_z", "energy", "split_unmix", "split_symbol", "interp_reduce"]
FP64, MIXED = 0, 1
FLAG_NONE = 0
FLAG_AUTOTUNE = 1
FLAG_SPLIT = 2
FLAG_INTERP_TILES = 4
FLAG_SPREAD_RINGS = 8
FLAG_RADIAL_GGQ = 16
FLAG_GAUSSIAN_KERNEL = 32
THETA_GL, COSTHETA_GL = 0, 1


class Params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("box", ctypes.c_double * 3),
        ("kernel", ctypes.c_int32),
        ("dipole_axis", ctypes.c_double * 3),
        ("lam", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("n_r", ctypes.c_int32),
        ("n_theta", ctypes.c_int32),
        ("n_phi", ctypes.c_int32),
        ("theta_rule", ctypes.c_int32),
        ("kmax", ctypes.c_double),
        ("device", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("flags", ctypes.c_uint32),
        ("window", ctypes.c_double * 2),
        ("dipole_axis2", ctypes.c_double * 3),
        ("alpha", ctypes.c_double),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("nf", ctypes.c_int64 * 3),
        ("n_nodes", ctypes.c_int64),
        ("n_half", ctypes.c_int64),
        ("width", ctypes.c_int32),
        ("beta", ctypes.c_double),
        ("kmax", ctypes.c_double),
        ("workspace_bytes", ctypes.c_int64),
        ("interp_chunk", ctypes.c_int32),
        ("spread_chunk", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("window", ctypes.c_double * 2),
        ("origin_coef", ctypes.c_double),
        ("radial_c", ctypes.c_double),
    ]


class GpeParams(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("potential", Params),
        ("trap", ctypes.c_double * 3),
        ("V", ctypes.c_void_p),
        ("beta", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("imaginary", ctypes.c_int32),
    ]


GPE_ENERGY_NAMES = ["norm", "kinetic", "trap", "local", "nonlocal", "total", "mu"]


NOALLOC_SCRATCH_BYTES = 128 << 20   # JGB_NOALLOC_SCRATCH_BYTES


class JgbError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libjgb.so not built: run `python -m paper_1311_4120_amd.build` "
                          "(or __graft_entry__.build()) first; there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    st = ctypes.c_int
    sig = {
        "jgb_plan": (st, [ctypes.POINTER(Params), ctypes.POINTER(P)]),
        "jgb_potential": (st, [P, P, P, P]),
        "jgb_potential_noalloc": (st, [P, P, P, P]),
        "jgb_energy": (st, [P, P, P]),
        "jgb_potential_backward": (st, [P, P, P]),
        "jgb_transform": (st, [P, P, P]),
        "jgb_nodes": (st, [P, P, P, P]),
        "jgb_density": (st, [P, P, P]),
        "jgb_psi_gradient": (st, [P, P, P, P, ctypes.c_double, P]),
        "jgb_plan_info": (st, [P, ctypes.POINTER(Info)]),
        "jgb_destroy": (st, [P]),
        "jgb_last_error": (ctypes.c_char_p, []),
        "jgb_timing_begin": (st, [P, ctypes.c_int]),
        "jgb_batch_create": (st, [ctypes.POINTER(Params), ctypes.c_int, ctypes.c_int, ctypes.POINTER(P)]),
        "jgb_batch_bind": (st, [P, ctypes.POINTER(P), ctypes.POINTER(P), P]),
        "jgb_batch_run": (st, [P]),
        "jgb_batch_launches": (st, [P, ctypes.POINTER(ctypes.c_int)]),
        "jgb_batch_plan": (st, [P, ctypes.c_int, ctypes.POINTER(P)]),
        "jgb_batch_destroy": (st, [P]),
        "jgb_timing_end": (st, [P, P, P]),
        "jgb_gpe_create": (st, [ctypes.POINTER(GpeParams), ctypes.POINTER(P)]),
        "jgb_gpe_step": (st, [P, P, ctypes.c_int, ctypes.c_int]),
        "jgb_gpe_energy": (st, [P, P, P]),
        "jgb_gpe_destroy": (st, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def check(status):
    if status != JGB_OK:
        msg = lib.jgb_last_error()
        raise JgbError(status, msg.decode() if msg else "")
    return status
