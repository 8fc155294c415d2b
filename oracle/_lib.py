"""Build and load the oracle's C part (sparse Cholesky). Test infrastructure."""
import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "orc_chol.c")
LIB = os.path.join(_HERE, "liborc.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = ctypes.CDLL(LIB)
        i64, i32p, i64p, dp, vp = (ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)
        L.orc_chol_factor.argtypes = [i64, i64p, i32p, dp, ctypes.c_int,
                                      ctypes.POINTER(vp)]
        L.orc_chol_factor.restype = ctypes.c_int
        L.orc_chol_solve.argtypes = [vp, dp, i64]
        L.orc_chol_solve.restype = None
        L.orc_chol_nnz.argtypes = [vp]
        L.orc_chol_nnz.restype = i64
        L.orc_chol_export.argtypes = [vp, i64p, i32p, dp, i32p]
        L.orc_chol_export.restype = None
        L.orc_chol_free.argtypes = [vp]
        L.orc_chol_free.restype = None
        _lib = L
    return _lib
