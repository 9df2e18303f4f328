"""ctypes declarations of include/nasg.h (argument marshalling only).

Loads the in-tree libnasg.so and fails loudly when it is missing: there is no
fallback implementation.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnasg.so")

NASG_OK, NASG_E_ARG, NASG_E_SHAPE, NASG_E_ALIGN, NASG_E_HIP = range(5)
NASG_F32, NASG_BF16 = 0, 1
STATUS_NAMES = {0: "NASG_OK", 1: "NASG_E_ARG", 2: "NASG_E_SHAPE", 3: "NASG_E_ALIGN", 4: "NASG_E_HIP"}

# every symbol include/nasg.h declares
EXPORTED = [
    "nasg_num_weights", "nasg_packed_bytes", "nasg_workspace_bytes", "nasg_create", "nasg_destroy",
    "nasg_last_error", "nasg_pack", "nasg_forward", "nasg_query", "nasg_pdf", "nasg_sample",
    "nasg_loss_grad", "nasg_adam_step", "nasg_train_step", "nasg_blend_ramp", "nasg_pdf_grad",
    "nasg_train_step_noalloc",
]


class Config(ctypes.Structure):
    _fields_ = [
        ("hidden", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("n_lobes", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("eps", ctypes.c_float), ("lr", ctypes.c_float),
        ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("adam_eps", ctypes.c_float),
        ("max_batch", ctypes.c_int64), ("selection", ctypes.c_int32), ("mis_fraction", ctypes.c_float),
        ("isotropic", ctypes.c_int32), ("encoding", ctypes.c_int32),
    ]


class State(ctypes.Structure):
    _fields_ = [
        ("w", ctypes.c_void_p), ("grad", ctypes.c_void_p), ("adam_m", ctypes.c_void_p),
        ("adam_v", ctypes.c_void_p), ("wpack", ctypes.c_void_p), ("step", ctypes.c_void_p),
        ("flags", ctypes.c_void_p), ("stats", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
    ]


class NasgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """The loaded library; raises if libnasg.so has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2303_08064_amd.build` "
                          "(there is no non-HIP fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    S = ctypes.c_int
    sig = {
        "nasg_num_weights": (ctypes.c_size_t, [ctypes.POINTER(Config)]),
        "nasg_packed_bytes": (ctypes.c_size_t, [ctypes.POINTER(Config)]),
        "nasg_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Config)]),
        "nasg_create": (S, [ctypes.POINTER(Config), ctypes.POINTER(State), ctypes.POINTER(P)]),
        "nasg_destroy": (None, [P]),
        "nasg_last_error": (ctypes.c_char_p, []),
        "nasg_pack": (S, [P, P]),
        "nasg_forward": (S, [P, P, I64, I64, P, P]),
        "nasg_query": (S, [P, P, P, I64, I64, P, P, P, P, P]),
        "nasg_pdf": (S, [P, P, P, I64, I64, P, P]),
        "nasg_sample": (S, [P, P, P, I64, I64, P, P, P]),
        "nasg_pdf_grad": (S, [P, P, P, I64, I64, P, P, P]),
        "nasg_loss_grad": (S, [P, P, P, P, P, I64, I64, P]),
        "nasg_adam_step": (S, [P, P]),
        "nasg_train_step": (S, [P, P, P, P, P, I64, I64, P]),
        "nasg_train_step_noalloc": (S, [P, P, P, P, P, I64, I64, P]),
        "nasg_blend_ramp": (ctypes.c_float, [I64, ctypes.c_int32, ctypes.c_int32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status):
    if status != NASG_OK:
        raise NasgError(status, load().nasg_last_error().decode())
