"""ctypes loader for libsym.so (the HIP kernels behind include/sym.h).

There is no fallback: if the library is missing or cannot be loaded, every call
raises. Build it with ``__graft_entry__.build()`` (or ``python -m
paper_1808_02281_amd.build``).
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsym.so")

SYM_OK = 0
SYM_F32 = 1
SYM_F64 = 2
ALGORITHMS = {"auto": 0, "direct": 1, "factored": 2}

# Every symbol include/sym.h declares.
EXPORTS = (
    "sym_coeffs",
    "sym_workspace_bytes",
    "sym_action",
    "sym_force",
    "sym_force_static",
    "sym_action_grad",
    "md_leapfrog",
    "sym_pack",
    "sym_unpack",
    "sym_set_coeffs_override",
    "sym_set_force_algorithm",
    "sym_strerror",
    "sym_profile_enable",
    "sym_profile_collect",
    "sym_batch_workspace_bytes",
    "sym_force_batch",
    "sym_batch_autotune",
    "sym_fat_workspace_bytes",
    "sym_fat_links",
    "sym_fat_force",
    "sym_wilson_workspace_bytes",
    "sym_wilson_force",
    "sym_pack_spinor",
    "sym_unpack_spinor",
    "sym_check_links",
    "sym_reunitarise",
)
FAT_MODES = {"grad": 0, "force": 1}
FAT_REUSE_LINKS = 2


class SymError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first (__graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    dp = ctypes.POINTER(ctypes.c_double)
    vp = ctypes.c_void_p
    L.sym_coeffs.argtypes = [ctypes.c_double, dp, dp]
    L.sym_coeffs.restype = ctypes.c_int
    L.sym_workspace_bytes.argtypes = [i32p, ctypes.c_int]
    L.sym_workspace_bytes.restype = ctypes.c_size_t
    L.sym_action.argtypes = [i32p, ctypes.c_double, ctypes.c_double, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp]
    L.sym_action.restype = ctypes.c_int
    L.sym_force.argtypes = [i32p, ctypes.c_double, ctypes.c_double, ctypes.c_int, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.sym_force.restype = ctypes.c_int
    L.sym_force_static.argtypes = [i32p, ctypes.c_double, ctypes.c_double, ctypes.c_int, vp, vp, vp, vp]
    L.sym_force_static.restype = ctypes.c_int
    L.sym_action_grad.argtypes = [i32p, ctypes.c_double, ctypes.c_double, ctypes.c_int, vp, vp, vp, vp,
                                  ctypes.c_size_t, vp]
    L.sym_action_grad.restype = ctypes.c_int
    L.md_leapfrog.argtypes = [i32p, ctypes.c_double, ctypes.c_double, ctypes.c_int, vp, vp, ctypes.c_double,
                              ctypes.c_int32, vp, vp, ctypes.c_size_t, vp]
    L.md_leapfrog.restype = ctypes.c_int
    L.sym_pack.argtypes = [i32p, ctypes.c_int, vp, vp, vp]
    L.sym_pack.restype = ctypes.c_int
    L.sym_unpack.argtypes = [i32p, ctypes.c_int, vp, vp, vp]
    L.sym_unpack.restype = ctypes.c_int
    L.sym_set_coeffs_override.argtypes = [dp]
    L.sym_set_coeffs_override.restype = ctypes.c_int
    L.sym_set_force_algorithm.argtypes = [ctypes.c_int]
    L.sym_set_force_algorithm.restype = ctypes.c_int
    L.sym_strerror.argtypes = [ctypes.c_int]
    L.sym_strerror.restype = ctypes.c_char_p
    L.sym_profile_enable.argtypes = [ctypes.c_int]
    L.sym_profile_enable.restype = ctypes.c_int
    L.sym_profile_collect.argtypes = [ctypes.c_int, ctypes.c_char_p, dp, i32p]
    L.sym_profile_collect.restype = ctypes.c_int
    L.sym_batch_workspace_bytes.argtypes = [ctypes.c_int, i32p, ctypes.c_int]
    L.sym_batch_workspace_bytes.restype = ctypes.c_size_t
    L.sym_force_batch.argtypes = [ctypes.c_int, i32p, ctypes.c_double, ctypes.c_double, ctypes.c_int, vp, vp, vp, vp,
                                  ctypes.c_size_t, vp]
    L.sym_force_batch.restype = ctypes.c_int
    L.sym_batch_autotune.argtypes = [ctypes.c_int, i32p, ctypes.c_double, ctypes.c_double, ctypes.c_int, vp, vp, vp,
                                     ctypes.c_size_t, vp, i32p, ctypes.c_int32, i32p, ctypes.POINTER(ctypes.c_float),
                                     i32p]
    L.sym_batch_autotune.restype = ctypes.c_int
    L.sym_fat_workspace_bytes.argtypes = [i32p, ctypes.c_int]
    L.sym_fat_workspace_bytes.restype = ctypes.c_size_t
    L.sym_fat_links.argtypes = [i32p, ctypes.c_int, dp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.sym_fat_links.restype = ctypes.c_int
    L.sym_fat_force.argtypes = [i32p, ctypes.c_int, dp, vp, vp, vp, vp, ctypes.c_int, vp, ctypes.c_size_t, vp]
    L.sym_fat_force.restype = ctypes.c_int
    L.sym_wilson_workspace_bytes.argtypes = [i32p, ctypes.c_int]
    L.sym_wilson_workspace_bytes.restype = ctypes.c_size_t
    L.sym_wilson_force.argtypes = [i32p, ctypes.c_int, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp, vp,
                                   ctypes.c_size_t, vp]
    L.sym_wilson_force.restype = ctypes.c_int
    L.sym_pack_spinor.argtypes = [i32p, ctypes.c_int, vp, vp, vp]
    L.sym_pack_spinor.restype = ctypes.c_int
    L.sym_unpack_spinor.argtypes = [i32p, ctypes.c_int, vp, vp, vp]
    L.sym_unpack_spinor.restype = ctypes.c_int
    L.sym_check_links.argtypes = [i32p, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp]
    L.sym_check_links.restype = ctypes.c_int
    L.sym_reunitarise.argtypes = [i32p, ctypes.c_int, vp, vp]
    L.sym_reunitarise.restype = ctypes.c_int
    _lib = L
    return L


def dims(L):
    return (ctypes.c_int32 * 4)(*[int(v) for v in L])


def check(fn, status):
    if status != SYM_OK:
        raise SymError(fn, status, lib().sym_strerror(status).decode())
    return status
