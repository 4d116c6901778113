"""ctypes binding of libcosim.so (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
_LOCK = threading.Lock()
_LIB = None

c_int = ctypes.c_int
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p
c_char_p = ctypes.c_char_p
P = ctypes.POINTER

# name -> (restype, argtypes); mirrors include/cosim.h and include/cosim_sparam.h
SIGNATURES = {
    "cosim_last_error": (c_char_p, []),
    "cosim_version": (c_int, []),
    "cosim_geometry_create": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p, P(c_void_p)]),
    "cosim_geometry_destroy": (c_int, [c_void_p]),
    "cosim_geometry_size": (c_int, [c_void_p, P(c_int), P(c_int)]),
    "cosim_assemble": (c_int, [c_void_p, c_int, c_void_p, c_double, c_void_p, P(c_void_p)]),
    "cosim_plan_destroy": (c_int, [c_void_p]),
    "cosim_plan_size": (c_int, [c_void_p, P(c_int), P(c_int)]),
    "cosim_plan_factorisations": (c_int, [c_void_p, P(ctypes.c_longlong)]),
    "cosim_plan_reserve": (c_int, [c_void_p, c_int, c_int]),
    "cosim_plan_copy_G": (c_int, [c_void_p, c_void_p, c_void_p]),
    "cosim_plan_copy_M": (c_int, [c_void_p, c_void_p]),
    "cosim_plan_copy_phi": (c_int, [c_void_p, c_void_p]),
    "cosim_solve": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "cosim_field": (c_int, [c_void_p, c_int, c_int, c_void_p, c_int, c_int, c_void_p, c_void_p]),
    "cosim_field_backward": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "cosim_loss_and_grad": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, c_int,
                                    c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "cosim_loss_and_grad_noalloc": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                            c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "cosim_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "cosim_assemble_ex": (c_int, [c_void_p, c_int, c_void_p, c_double, c_int, c_void_p, P(c_void_p)]),
    "cosim_assemble_component": (c_int, [c_void_p, c_int, c_void_p, c_double, c_int, c_int, c_void_p,
                                         P(c_void_p)]),
    "cosim_plan_set_drive": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_double,
                                     c_void_p]),
    "cosim_plan_set_refinement": (c_int, [c_void_p, c_int, c_int, c_double]),
    "cosim_loss_and_grad_many": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                         c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                         c_void_p]),
    "cosim_adam_step": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                c_double, c_double, c_double, c_void_p]),
    "cosim_plan_set_variant": (c_int, [c_void_p, c_int, c_int]),
    "cosim_plan_get_variant": (c_int, [c_void_p, c_int, P(c_int), P(c_int)]),
    "cosim_plan_autotune": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, c_int,
                                    c_int, c_int, c_void_p, c_void_p]),
    "cosim_plan_timing": (c_int, [c_void_p, c_int]),
    "cosim_plan_timing_read": (c_int, [c_void_p, c_void_p, c_int, P(c_int)]),
    "cosim_loss_and_grad_params": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                           c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                           c_void_p, c_void_p, c_void_p]),
    "cosim_resonant_capacitance": (c_int, [c_void_p, c_int, c_void_p, c_int, c_void_p, c_void_p]),
    "cosim_tanh_projection": (c_int, [ctypes.c_int64, c_void_p, c_double, c_double, c_void_p,
                                      c_void_p, c_void_p]),
    "cosim_clip": (c_int, [ctypes.c_int64, c_void_p, c_double, c_double, c_void_p]),
    "cosim_sp_create": (c_int, [c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                c_int, c_void_p, c_void_p, c_void_p, c_int, c_void_p, P(c_void_p)]),
    "cosim_sp_destroy": (c_int, [c_void_p]),
    "cosim_sp_reserve": (c_int, [c_void_p, c_int]),
    "cosim_sp_field": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "cosim_sp_loss_and_grad": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_int, c_int, c_int,
                                       c_void_p, c_void_p, c_void_p, c_void_p]),
    "cosim_sp_rc": (c_int, [c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_double, c_void_p,
                            c_int, c_void_p]),
    "cosim_sp_rc_backward": (c_int, [c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_double,
                                     c_void_p, c_int, c_void_p, c_void_p]),
}

STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EUNSUPPORTED"}


class CosimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cosim error {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def library_path() -> str:
    return os.environ.get("COSIM_LIBRARY", os.path.join(_HERE, "libcosim.so"))


def load_library() -> ctypes.CDLL:
    """Load libcosim.so (built in-tree by paper_2503_18479_amd.build).
    There is no fallback: a missing library is an error."""
    global _LIB
    with _LOCK:
        if _LIB is None:
            path = library_path()
            if not os.path.exists(path):
                raise RuntimeError(
                    f"{path} is missing: build it with `python -m paper_2503_18479_amd.build` "
                    "(or __graft_entry__.build())")
            lib = ctypes.CDLL(path)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _LIB = lib
    return _LIB


def check(code: int) -> None:
    if code != 0:
        msg = load_library().cosim_last_error()
        raise CosimError(code, msg.decode() if msg else "")
