"""ctypes declarations of the libfewha C ABI (include/fewha.h).

Argument marshalling only: every computation runs in the HIP library.  The
library must have been built (``python paper_2202_11945_amd/build.py``); a
missing library raises at import time, there is no fallback.
"""

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_long, c_ubyte, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libfewha.so")

FEWHA_OK = 0
STATUS = {0: "FEWHA_OK", -1: "FEWHA_EINVAL", -2: "FEWHA_ENOMEM", -3: "FEWHA_EDEVICE",
          -4: "FEWHA_ESTATE", -5: "FEWHA_EGEOM", -6: "FEWHA_ENUMERIC"}
FEWHA_NGS, FEWHA_LGS = 0, 1
FEWHA_TABLE_FILTER, FEWHA_TABLE_PRIOR, FEWHA_TABLE_PRECOND, FEWHA_TABLE_MASK = 0, 1, 2, 3
STAGES = ["IDWT_RES", "IDWT_GLOB", "P_GAMMA", "GAMMA_T", "P_T", "FDWT_GLOB", "FDWT_RES", "UPDATE"]


class fewha_wfs_desc(ctypes.Structure):
    _fields_ = [("kind", c_int), ("n_subap", c_int), ("theta_x", c_double), ("theta_y", c_double),
                ("H", c_double), ("sigma", c_double), ("launch_x", c_double), ("launch_y", c_double),
                ("tt_removal", c_int), ("mask", POINTER(c_ubyte))]


class fewha_layer_desc(ctypes.Structure):
    _fields_ = [("h", c_double), ("n", c_int), ("levels", c_int), ("cn2", c_double)]


class fewha_dm_desc(ctypes.Structure):
    _fields_ = [("h", c_double), ("n_act", c_int), ("pitch", c_double)]


class fewha_tuning(ctypes.Structure):
    _fields_ = [("dwt_resident", c_int), ("pt_rows", c_int), ("streams", c_int), ("res_split", c_int),
                ("pt_split", c_int), ("glob_fuse", c_int), ("reserved", c_int * 2)]


class FewhaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, str(status)), msg))
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError("libfewha.so is not built (%s); run python paper_2202_11945_amd/build.py" % LIB_PATH)

# torch ships its own HIP runtime under the same soname; loading torch first
# makes the library bind to that one runtime instead of a second copy, so
# device pointers and streams from torch are valid in the library.
import torch  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)

_P = c_void_p
_FP = c_void_p  # device float* / const float*
_SIGS = {
    "fewha_create": (c_int, [POINTER(c_void_p), c_int]),
    "fewha_set_stream": (c_int, [_P, c_void_p]),
    "fewha_set_pupil": (c_int, [_P, c_double, c_double]),
    "fewha_set_wfs": (c_int, [_P, c_int, POINTER(fewha_wfs_desc)]),
    "fewha_set_layers": (c_int, [_P, c_int, POINTER(fewha_layer_desc), c_double]),
    "fewha_set_prior": (c_int, [_P, c_double, c_double, c_double, c_double]),
    "fewha_set_noise": (c_int, [_P, c_double, c_double, c_double]),
    "fewha_set_control": (c_int, [_P, c_double]),
    "fewha_set_loop": (c_int, [_P, c_int]),
    "fewha_set_augmentation": (c_int, [_P, c_int]),
    "fewha_set_refresh": (c_int, [_P, c_int]),
    "fewha_set_solve_coarse": (c_int, [_P, c_int]),
    "fewha_batch_set_solve_coarse": (c_int, [_P, c_int]),
    "fewha_set_frame_count": (c_int, [_P, c_long]),
    "fewha_batch_set_refresh": (c_int, [_P, c_int]),
    "fewha_batch_set_frame_count": (c_int, [_P, c_long]),
    "fewha_set_photons": (c_int, [_P, c_int, POINTER(c_double)]),
    "fewha_set_fitting": (c_int, [_P, c_int, POINTER(fewha_dm_desc), c_int, POINTER(c_double), c_int, c_int,
                                  c_double]),
    "fewha_set_tuning": (c_int, [_P, POINTER(fewha_tuning)]),
    "fewha_finalize": (c_int, [_P]),
    "fewha_sizes": (c_int, [_P, POINTER(c_long), POINTER(c_long), POINTER(c_long), POINTER(c_long),
                            POINTER(c_long)]),
    "fewha_get_table": (c_int, [_P, c_int, POINTER(c_double), c_long]),
    "fewha_apply_A": (c_int, [_P, _FP, _FP]),
    "fewha_apply_AT": (c_int, [_P, _FP, _FP]),
    "fewha_apply_M": (c_int, [_P, _FP, _FP]),
    "fewha_rhs": (c_int, [_P, _FP, _FP]),
    "fewha_reconstruct": (c_int, [_P, _FP, _FP, _FP, _FP, c_int]),
    "fewha_reconstruct_noalloc": (c_int, [_P, _FP, _FP, _FP, _FP, c_int]),
    "fewha_reconstruct_streamed": (c_int, [_P, c_void_p, _FP, _FP, _FP, c_int, c_int]),
    "fewha_solve": (c_int, [_P, _FP, _FP, c_int, c_double, POINTER(c_int), POINTER(c_double)]),
    "fewha_solve_map": (c_int, [_P, _FP, _FP, _FP, c_int, c_double, POINTER(c_int), POINTER(c_double)]),
    "fewha_apply_Winv": (c_int, [_P, _FP, _FP]),
    "fewha_apply_WinvT": (c_int, [_P, _FP, _FP]),
    "fewha_param_grads": (c_int, [_P, _FP, _FP, _FP, c_void_p]),
    "fewha_batch_create": (c_int, [POINTER(c_void_p), POINTER(c_void_p), c_int]),
    "fewha_batch_create_tuned": (c_int, [POINTER(c_void_p), POINTER(c_void_p), c_int, POINTER(fewha_tuning)]),
    "fewha_batch_solve": (c_int, [_P, POINTER(c_void_p), POINTER(c_void_p), c_int, c_double, POINTER(c_int),
                                  POINTER(c_double)]),
    "fewha_batch_solve_map": (c_int, [_P, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p), c_int, c_double,
                                      POINTER(c_int), POINTER(c_double)]),
    "fewha_batch_apply_Winv": (c_int, [_P, POINTER(c_void_p), POINTER(c_void_p)]),
    "fewha_batch_apply_WinvT": (c_int, [_P, POINTER(c_void_p), POINTER(c_void_p)]),
    "fewha_batch_param_grads": (c_int, [_P, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                        POINTER(c_void_p)]),
    "fewha_batch_set_stream": (c_int, [_P, c_void_p]),
    "fewha_batch_reconstruct": (c_int, [_P, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                        POINTER(c_void_p), c_int, c_int]),
    "fewha_batch_time_stage": (c_int, [_P, c_int, c_int, POINTER(c_double), POINTER(c_long)]),
    "fewha_batch_destroy": (None, [_P]),
    "fewha_last_error": (c_char_p, [_P]),
    "fewha_batch_last_error": (c_char_p, [_P]),
    "fewha_destroy": (None, [_P]),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f

EXPORTED = sorted(_SIGS)
