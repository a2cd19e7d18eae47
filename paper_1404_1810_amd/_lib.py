"""ctypes declarations of the C ABI in include/amqft.h (argument marshalling
only: no arithmetic happens in Python).  The shared library is the in-tree
``libamqft.so``; if it is missing this module raises -- there is no CPU or
PyTorch fallback."""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamqft.so")

# enums of include/amqft.h
C128, C64, C32H, C32B, C32I = 0, 1, 2, 3, 4
OK, ERR_INVALID_ARG, ERR_NOT_POW2, ERR_UNSUPPORTED, ERR_ALLOC, ERR_HIP = range(6)
RDFT, DCT0, DST0 = 0, 1, 2
FLAG_ONTHEFLY_CONSTANTS = 1
FLAG_NO_AUTOTUNE = 2
FLAG_FORCE_MULTIPASS = 4
FLAG_FORCE_LARGE = 8
FLAG_TRANSPOSED_ADJOINT = 16
FLAG_IN_PLACE = 32
NOALLOC_SCRATCH_BYTES = 64 << 20

#: every function the header declares, with its ctypes signature
SIGNATURES = {
    "amqft_plan_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_uint]),
    "amqft_plan_create_many": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int64, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_uint]),
    "amqft_plan_create_real": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int64, ctypes.c_int64,
                                              ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint]),
    "amqft_exec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "amqft_exec_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "amqft_power_loss_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "amqft_exec_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                        ctypes.c_void_p]),
    "amqft_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "amqft_plan_describe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_size_t]),
    "amqft_plan_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "amqft_plan_constants": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64]),
    "amqft_exec_noalloc": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "amqft_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "amqft_last_hip_error": (ctypes.c_char_p, []),
    "amqft_version": (ctypes.c_char_p, []),
}

_lock = threading.Lock()
_lib = None


def load():
    """Load libamqft.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libamqft.so is not built (run `python -m paper_1404_1810_amd.build`); "
                               "the AM-QFT path has no CPU fallback")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


class AmqftError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        msg = lib.amqft_status_string(status).decode()
        hip = lib.amqft_last_hip_error().decode()
        super().__init__("%s: %s%s" % (where, msg, (" (" + hip + ")") if hip and status == ERR_HIP else ""))
        self.status = status


def check(status: int, where: str) -> None:
    if status != OK:
        raise AmqftError(status, where)
