"""ctypes binding of libgeninv (argument marshalling only).

Every function here converts torch tensors to the library's column-major
device-pointer convention, calls one C entry point and wraps the outputs.
All arithmetic runs in the HIP kernels of libgeninv.so; there is no CPU or
PyTorch fallback: if the library is missing or a tensor is not on a GPU the
call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgeninv.so")

_c_int_p = ctypes.POINTER(ctypes.c_int)
_lib = None
_lock = threading.Lock()

GENINV_OK = 0
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENONFINITE", -5: "ENOTSPD", -6: "ENOTSUP",
                -7: "EACCURACY", -8: "ESCRATCH"}
GENINV_EACCURACY = -7
# geninv_precision
GENINV_FP64, GENINV_MIXED_BF16, GENINV_MIXED_INT8 = 0, 1, 2


class GeninvError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = load().geninv_strerror(status).decode()
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} ({msg})")


# (name, restype, argtypes) of every exported entry point
_VP = ctypes.c_void_p
_SIGS = [
    ("geninv_create", ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int, _VP]),
    ("geninv_destroy", ctypes.c_int, [_VP]),
    ("geninv_set_stream", ctypes.c_int, [_VP, _VP]),
    ("geninv_set_host_sync", ctypes.c_int, [_VP, ctypes.c_int]),
    ("geninv_set_workspace_limit", ctypes.c_int, [_VP, ctypes.c_size_t]),
    ("geninv_set_debug", ctypes.c_int, [_VP, ctypes.c_int]),
    ("geninv_debug_poison", ctypes.c_int, [_VP]),
    ("geninv_sync_status", ctypes.c_int, [_VP]),
    ("geninv_strerror", ctypes.c_char_p, [ctypes.c_int]),
    ("geninv_version", ctypes.c_int, []),
    ("geninv_workspace_bytes", ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                 ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    ("geninv_dgeninv", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, ctypes.c_double,
                                      _VP, ctypes.c_int, _c_int_p, _VP]),
    ("geninv_dlstsq", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, _VP,
                                     ctypes.c_int, ctypes.c_double, _VP, ctypes.c_int, _c_int_p]),
    ("geninv_dlstsq_noalloc", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, _VP,
                                             ctypes.c_int, ctypes.c_double, _VP, ctypes.c_int, _c_int_p]),
    ("geninv_noalloc_capacity", ctypes.c_size_t, []),
    ("geninv_dgram", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, _VP, ctypes.c_int,
                                    ctypes.c_int]),
    ("geninv_dfrchol", ctypes.c_int, [_VP, ctypes.c_int, _VP, ctypes.c_int, ctypes.c_double, _VP, ctypes.c_int,
                                      _VP, _VP, _VP, _c_int_p]),
    ("geninv_dspdinv", ctypes.c_int, [_VP, ctypes.c_int, _VP, ctypes.c_int, _VP, ctypes.c_int]),
    ("geninv_dspdinv_ns", ctypes.c_int, [_VP, ctypes.c_int, _VP, ctypes.c_int, _VP, ctypes.c_int, ctypes.c_int,
                                         _c_int_p, ctypes.POINTER(ctypes.c_double)]),
    ("geninv_dchain", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, _VP,
                                     ctypes.c_int, _VP, ctypes.c_int, _VP, ctypes.c_int]),
    ("geninv_mixed", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _VP,
                                    ctypes.c_int, _c_int_p, _VP, ctypes.POINTER(ctypes.c_double)]),
    ("geninv_mgemm", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    _VP, ctypes.c_int, _VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP,
                                    ctypes.c_int]),
    ("geninv_bslice", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, _VP, ctypes.c_int, _VP]),
    ("geninv_bgram", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, ctypes.c_int, _VP,
                                    ctypes.c_int]),
    ("geninv_bchain", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, _VP,
                                     ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int]),
    ("geninv_inc_gram", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP,
                                       ctypes.c_int, _VP, ctypes.c_int, _VP, ctypes.c_int, _VP, ctypes.c_int]),
    ("geninv_dlstsq_gram", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, _VP, ctypes.c_int,
                                          ctypes.c_double, _VP, ctypes.c_int, _c_int_p]),
    ("geninv_inc_factor", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, ctypes.c_double, _VP,
                                         ctypes.c_int, _VP, _VP, _VP, ctypes.c_int, _c_int_p,
                                         ctypes.POINTER(ctypes.c_double)]),
    ("geninv_factored_lstsq", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, _VP,
                                             ctypes.c_int, _VP, ctypes.c_int, _VP, ctypes.c_int]),
    ("geninv_batch_plan_create", ctypes.c_int, [_VP, ctypes.POINTER(_VP), ctypes.c_int, _c_int_p, _c_int_p,
                                                ctypes.c_int, ctypes.POINTER(_VP), _c_int_p, ctypes.POINTER(_VP),
                                                _c_int_p, ctypes.POINTER(_VP), _c_int_p, ctypes.c_double, _VP]),
    ("geninv_batch_plan_destroy", ctypes.c_int, [_VP]),
    ("geninv_lstsq_batched", ctypes.c_int, [_VP, ctypes.c_int, _c_int_p, _c_int_p, ctypes.c_int,
                                            ctypes.POINTER(_VP), _c_int_p, ctypes.POINTER(_VP), _c_int_p,
                                            ctypes.c_double, ctypes.POINTER(_VP), _c_int_p, _VP, _c_int_p]),
    ("geninv_batch_plan_run", ctypes.c_int, [_VP, ctypes.c_int]),
    ("geninv_batch_plan_graph_fallbacks", ctypes.c_int, [_VP]),
    ("geninv_batch_plan_autotune", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_char_p, _c_int_p, _c_int_p,
                                                  ctypes.POINTER(ctypes.c_double), _c_int_p]),
    ("geninv_batch_plan_set_pivots", ctypes.c_int, [_VP, ctypes.POINTER(_VP)]),
    ("geninv_batch_plan_config", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int]),
    ("geninv_batch_plan_get_config", ctypes.c_int, [_VP, _c_int_p, _c_int_p]),
    ("geninv_prof_classes", ctypes.c_int, []),
    ("geninv_prof_name", ctypes.c_char_p, [ctypes.c_int]),
    ("geninv_prof_enable", ctypes.c_int, [_VP, ctypes.c_uint]),
    ("geninv_prof_read", ctypes.c_int, [_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_double)]),
    ("geninv_dgemm", ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, _VP, ctypes.c_int, _VP, ctypes.c_int, ctypes.c_double, _VP,
                                    ctypes.c_int]),
]


def load(path: str = LIB_PATH):
    """Load libgeninv.so (built in-tree by paper_0804_4809_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise RuntimeError(f"{path} is not built: run `python -m paper_0804_4809_amd.build`")
            lib = ctypes.CDLL(path)
            for name, res, args in _SIGS:
                f = getattr(lib, name)
                f.restype = res
                f.argtypes = args
            _lib = lib
    return _lib


def exported_names():
    return [s[0] for s in _SIGS]
