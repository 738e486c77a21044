"""ctypes view of the C ABI in include/dmdmi.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
# DMDMI_LIBRARY selects another build of the same library (the host-sanitized one in tests)
LIB_PATH = os.environ.get("DMDMI_LIBRARY") or os.path.join(HERE, "libdmdmi.so")

c_int32, c_int64, c_double, c_void_p, c_size_t = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                                  ctypes.c_void_p, ctypes.c_size_t)

# enums (mirror include/dmdmi.h)
DMD_OK = 0
DMD_ERR_ARG = 1
DMD_ERR_SHAPE = 2
DMD_ERR_WORKSPACE = 3
DMD_ERR_NONFINITE = 4
DMD_ERR_CHOL_BREAKDOWN = 5
DMD_ERR_RANK = 6
DMD_ERR_EIG_NOCONV = 7
DMD_ERR_DOMAIN = 8
DMD_ERR_OVERFLOW = 9
DMD_ERR_HIP = 10
DMD_ERR_UNSUPPORTED = 11
DMD_ERR_IO = 12

DMD_F32, DMD_F64 = 0, 1
FIT_MIXED, FIT_FP64_RANDOMIZED, FIT_FP64_EXACT = 0, 1, 2
RECON_FP64, RECON_FP32, RECON_BF16, RECON_BF16X3 = 0, 1, 2, 3
FIT_ASYNC, FIT_CHECK_FINITE, FIT_OPTDMD = 1, 2, 4
INFO_WORDS = 8
MAX_SMALL = 192
MAX_SKETCH = 160
MAX_RANK = 160
NOALLOC_SCRATCH_BYTES = 8 << 20


class FitOpts(ctypes.Structure):
    _fields_ = [("r", c_int32), ("p", c_int32), ("q", c_int32), ("precision", c_int32),
                ("dt", c_double), ("rank_tol", c_double), ("omega", c_void_p),
                ("flags", ctypes.c_uint32), ("optdmd_trials", c_int32)]


class ModelStruct(ctypes.Structure):
    _fields_ = [("n", c_int64), ("r", c_int32), ("dtype", c_int32), ("dt", c_double),
                ("phi", c_void_p), ("ldphi", c_int64), ("lam", c_void_p), ("b", c_void_p),
                ("sigma", c_void_p), ("kind", c_void_p), ("info", c_void_p)]


class SceneStruct(ctypes.Structure):
    _fields_ = [("x", c_void_p), ("xp", c_void_p), ("n", c_int64), ("ncols", c_int32),
                ("xdtype", c_int32), ("ldx", c_int64), ("ldxp", c_int64), ("opts", FitOpts),
                ("ws", c_void_p), ("ws_bytes", c_size_t)]


class EditStruct(ctypes.Structure):
    _fields_ = [("freq_cut", c_double), ("weight", c_double * 2), ("re_scale", c_double * 2),
                ("re_shift", c_double * 2), ("im_scale", c_double * 2)]


_SIGS = {
    "dmd_abi_version": (c_int32, []),
    "dmd_status_string": (ctypes.c_char_p, [c_int32]),
    "dmd_phi_ld": (c_int64, [c_int32]),
    "dmd_fit_workspace_size": (c_int32, [c_int64, c_int32, c_int32, ctypes.POINTER(FitOpts),
                                         ctypes.POINTER(c_size_t)]),
    "dmd_fit": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_int64, c_int64, c_int32,
                          ctypes.POINTER(FitOpts), c_void_p, c_size_t, ctypes.POINTER(ModelStruct)]),
    "dmd_reconstruct_workspace_size": (c_int32, [c_int32, c_int32, c_int32, ctypes.POINTER(c_size_t)]),
    "dmd_reconstruct": (c_int32, [c_void_p, ctypes.POINTER(ModelStruct), ctypes.POINTER(c_int64), c_int32,
                                  c_int32, c_void_p, c_int64, c_void_p, c_size_t]),
    "dmd_reconstruct_noalloc": (c_int32, [c_void_p, ctypes.POINTER(ModelStruct), ctypes.POINTER(c_int64), c_int32,
                                          c_int32, c_void_p, c_int64, c_void_p]),
    "dmd_refit_workspace_size": (c_int32, [c_int64, c_int32, c_int32, ctypes.POINTER(c_size_t)]),
    "dmd_refit_prepare": (c_int32, [c_void_p, ctypes.POINTER(ModelStruct), c_void_p, c_int64, ctypes.POINTER(c_int64),
                                    c_int32, c_void_p, c_size_t]),
    "dmd_refit_loss_grad": (c_int32, [c_void_p, ctypes.POINTER(ModelStruct), c_void_p, c_void_p, c_int32, c_void_p,
                                      c_void_p, c_size_t]),
    "dmd_reconstruct_prepare": (c_int32, [c_void_p, ctypes.POINTER(ModelStruct), ctypes.POINTER(c_int64),
                                          ctypes.POINTER(c_double), c_int32, c_int32, c_void_p, c_size_t]),
    "dmd_reconstruct_apply": (c_int32, [c_void_p, ctypes.POINTER(ModelStruct), c_int32, c_int32, c_void_p, c_int64,
                                        c_void_p, c_size_t]),
    "dmd_integrate": (c_int32, [c_void_p, ctypes.POINTER(ModelStruct), ctypes.POINTER(c_double), c_int32,
                                c_int32, c_void_p, c_int64, c_void_p, c_size_t]),
    "dmd_edit_modes": (c_int32, [c_void_p, ctypes.POINTER(ModelStruct), ctypes.POINTER(EditStruct), c_void_p,
                                 c_void_p, c_void_p, c_void_p]),
    "dmd_rollout_workspace_size": (c_int32, [c_int64, c_int32, c_int32, c_int32, ctypes.POINTER(c_size_t)]),
    "dmd_rollout": (c_int32, [c_void_p, ctypes.POINTER(ModelStruct), c_void_p, c_void_p, c_int64, c_int32, c_int32,
                              c_void_p, c_int64, c_void_p, c_void_p, c_size_t]),
    "dmd_upsample_workspace_size": (c_int32, [c_int64, c_int32, c_int32, c_int32, ctypes.POINTER(c_size_t)]),
    "dmd_upsample": (c_int32, [c_void_p, ctypes.POINTER(ModelStruct), c_void_p, c_void_p, c_int64, c_int32,
                               ctypes.POINTER(c_int32), c_int32, c_void_p, c_int64, c_void_p, c_void_p, c_size_t]),
    "dmd_lowres_project": (c_int32, [c_void_p, c_int32, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                                     c_int64, c_int32, c_int32, c_int32, c_int32, c_int32]),
    "dmd_project_workspace_size": (c_int32, [c_int64, c_int32, ctypes.POINTER(c_size_t)]),
    "dmd_project": (c_int32, [c_void_p, ctypes.POINTER(ModelStruct), c_void_p, c_void_p, c_void_p, c_size_t]),
    "dmd_loss_grad_workspace_size": (c_int32, [c_int64, c_int32, c_int32, c_int32, ctypes.POINTER(c_size_t)]),
    "dmd_loss_grad": (c_int32, [c_void_p, ctypes.POINTER(ModelStruct), c_void_p, c_void_p, c_void_p, c_int64,
                                ctypes.POINTER(c_int64), c_int32, c_void_p, c_void_p, c_size_t]),
    "dmd_fit_batched": (c_int32, [c_void_p, c_int32, ctypes.POINTER(SceneStruct), ctypes.POINTER(ModelStruct),
                                  c_int32, ctypes.POINTER(c_void_p)]),
    "dmd_graph_launch": (c_int32, [c_void_p, c_void_p]),
    "dmd_graph_destroy": (c_int32, [c_void_p]),
    "dmd_autotune_reconstruct": (c_int32, [c_void_p, ctypes.POINTER(ModelStruct), c_int32, c_int32, c_void_p,
                                           c_int64, c_void_p, c_size_t, ctypes.c_char_p,
                                           ctypes.POINTER(c_int32)]),
    "dmd_autotune_load": (c_int32, [ctypes.c_char_p]),
    "dmd_autotune_fit": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_int64, c_int64, c_int32,
                                   ctypes.POINTER(FitOpts), c_void_p, c_size_t, ctypes.POINTER(ModelStruct),
                                   ctypes.c_char_p]),
    "dmd_status_word": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(c_int32)]),
    "dmd_model_save": (c_int32, [c_void_p, ctypes.POINTER(ModelStruct), ctypes.c_char_p]),
    "dmd_model_file_info": (c_int32, [ctypes.c_char_p, ctypes.POINTER(c_int64), ctypes.POINTER(c_int32),
                                      ctypes.POINTER(c_int32), ctypes.POINTER(c_double)]),
    "dmd_model_load": (c_int32, [c_void_p, ctypes.c_char_p, ctypes.POINTER(ModelStruct)]),
}

_lock = threading.Lock()
_lib = None


class DMDError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: status {code} ({status_string(code)})")


def lib():
    """The loaded libdmdmi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
                L = ctypes.CDLL(LIB_PATH)
                for name, (res, args) in _SIGS.items():
                    f = getattr(L, name)
                    f.restype = res
                    f.argtypes = args
                _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().dmd_status_string(int(code)).decode()


def check(code: int, where: str):
    if code != DMD_OK:
        raise DMDError(code, where)
