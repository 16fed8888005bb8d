"""Build and load the oracle's plain-C helpers (oracle/orc.c) with gcc.

Test infrastructure only.  The shared object is written next to the source
(oracle/liborc.so); it is git-ignored and rebuilt by ``build_oracle()``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

# -ffp-contract=off: the error-free transformations must not be fused.
CFLAGS = ["-O2", "-fPIC", "-shared", "-std=c11", "-fno-fast-math",
          "-ffp-contract=off", "-fopenmp"]


def build_oracle() -> str:
    """Compile oracle/orc.c into oracle/liborc.so (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        L.orc_axpby_fma.argtypes = [ctypes.c_int64, D, P, D, P]
        L.orc_axpby_fma.restype = None
        L.orc_dot2_gemm.argtypes = [I, I, I, P, I, P, I, P, I]
        L.orc_dot2_gemm.restype = None
        L.orc_dot2_residual.argtypes = [I, I, P, I, P, I, P, I, P, I]
        L.orc_dot2_residual.restype = None
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = I
        _lib = L
    return _lib
