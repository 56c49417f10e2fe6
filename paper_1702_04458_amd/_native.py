"""ctypes loader for ``libdbp.so`` (argument marshalling only).

The library is built in-tree by ``paper_1702_04458_amd.build``.  If it is
missing, loading raises: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# DBP_LIBRARY may name another build of the same library (e.g. to compare two
# builds on one device); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("DBP_LIBRARY") or os.path.join(_HERE, "libdbp.so")

# Entry points declared in include/dbp.h: (name, restype, argtypes)
_vp, _i, _f, _u8p, _fp = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p
SIGNATURES = {
    "dbp_version": (ctypes.c_char_p, []),
    "dbp_strerror": (ctypes.c_char_p, [_i]),
    "dbp_last_error": (ctypes.c_char_p, []),
    "dbp_detect_workspace_bytes": (ctypes.c_size_t, [_i, _i, _i]),
    "dbp_detect_admm": (_i, [_vp, _vp, _vp, _u8p, _vp, _vp, ctypes.c_size_t, _i, _i, _i, _i, _i, _i,
                             _f, _f, _f, _f, _i, _i, _i, _vp]),
    "dbp_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "dbp_detect_admm_noalloc": (_i, [_vp, _vp, _vp, _u8p, _vp, _i, _i, _i, _i, _i, _i, _f, _f, _f, _f, _i, _i, _i,
                                     _vp]),
    "dbp_autotune": (_i, [_i, _vp, _vp, _vp, _i, _i, _i, _i, _i, _i, _vp, ctypes.POINTER(_i)]),
    "dbp_autotune_get": (_i, [_i, _i, _i]),
    "dbp_factor_bytes": (ctypes.c_size_t, [_i, _i, _i]),
    "dbp_factor_admm": (_i, [_vp, _vp, _i, _i, _i, _i, _f, _i, _vp]),
    "dbp_detect_admm_factored": (_i, [_vp, _vp, _vp, _vp, _u8p, _vp, _vp, ctypes.c_size_t, _i, _i, _i, _i, _i, _i,
                                      _f, _f, _f, _f, _i, _i, _vp]),
    "dbp_channel_h16_bytes": (ctypes.c_size_t, [_i, _i, _i, _i]),
    "dbp_flag_nonfinite": (_i, [_vp, _i, _i, _vp, _vp]),
    "dbp_pack_channel_h16": (_i, [_vp, _vp, _i, _i, _i, _i, _vp]),
    "dbp_factor_admm_h16": (_i, [_vp, _vp, _vp, _i, _i, _i, _i, _f, _i, _vp]),
    "dbp_detect_admm_factored_h16": (_i, [_vp, _vp, _vp, _vp, _u8p, _vp, _i, _i, _i, _i, _i, _i, _f, _f, _f, _f,
                                          _i, _i, _vp]),
    "dbp_detect_cg": (_i, [_vp, _vp, _vp, _u8p, _vp, _vp, ctypes.c_size_t, _i, _i, _i, _i, _i, _i, _f, _f, _i, _i,
                           _vp]),
    "dbp_precode_admm": (_i, [_vp, _i, _vp, _vp, _fp, _fp, _i, _i, _i, _i, _i, _i, _i, _f, _f, _f, _vp]),
    "dbp_server_create": (_i, [_i, ctypes.c_size_t, _i, ctypes.POINTER(ctypes.c_void_p)]),
    "dbp_server_destroy": (_i, [_vp]),
    "dbp_server_submit": (_i, [_vp, _vp, _vp, _vp, _u8p, _i, _i, _i, _i, _i, _i, _f, _f, _i, _i, _i, _i,
                               ctypes.POINTER(ctypes.c_uint64)]),
    "dbp_channel_load": (_i, [_vp, _vp, _i, _i, _i, _i, _f, _i, _i, ctypes.POINTER(ctypes.c_uint64)]),
    "dbp_channel_free": (_i, [_vp, ctypes.c_uint64]),
    "dbp_server_submit_factored": (_i, [_vp, ctypes.c_uint64, _vp, _vp, _u8p, _i, _i, _f, _i, _i, _i,
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "dbp_server_poll": (_i, [_vp, ctypes.c_uint64, ctypes.POINTER(_i), ctypes.POINTER(ctypes.c_double)]),
    "dbp_server_wait": (_i, [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "dbp_server_set_batching": (_i, [_vp, _i]),
    "dbp_server_stats": (_i, [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_i), ctypes.POINTER(ctypes.c_uint64)]),
}

class Frame(ctypes.Structure):
    """dbp_frame of include/dbp.h (one frame of a batched detection call)."""
    _fields_ = [("H", ctypes.c_void_p), ("y", ctypes.c_void_p), ("s_hat", ctypes.c_void_p),
                ("hard", ctypes.c_void_p), ("status", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t),
                ("n_sc", ctypes.c_int), ("n_sym", ctypes.c_int), ("B", ctypes.c_int), ("C", ctypes.c_int),
                ("T", ctypes.c_int), ("reg", ctypes.c_int), ("qam", ctypes.c_int),
                ("rho", ctypes.c_float), ("gamma", ctypes.c_float), ("N0", ctypes.c_float), ("Es", ctypes.c_float)]


SIGNATURES["dbp_detect_admm_batch"] = (ctypes.c_int, [ctypes.POINTER(Frame), ctypes.c_int, ctypes.c_int,
                                                      ctypes.c_void_p])

_lib = None


class DbpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1702_04458_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code: int) -> None:
    if code != 0:
        L = lib()
        raise DbpError(code, f"{L.dbp_strerror(code).decode()}: {L.dbp_last_error().decode()}")
