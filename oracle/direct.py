"""ctypes binding of the C direct-sum oracle (test infrastructure).

``build()`` compiles ``csrc/lgf_oracle.c`` with gcc/OpenMP into
``oracle/liblgf_oracle.so``.  ``direct_sum`` evaluates
u(n) = dx^2 * sum_m G(n - m) f(m) over explicit cell lists
(paper Sec. 2.2, eq. lgf_convolution).
"""
import ctypes
import os
import subprocess

import numpy as np

from . import lgf_table

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "lgf_oracle.c")
_LIB = os.path.join(_HERE, "liblgf_oracle.so")
_lib = None


def build(force=True):
    """Compile the C oracle (gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_direct_sum.argtypes = [dp, ctypes.c_int, ctypes.c_int64, ip, dp,
                                          ctypes.c_int64, ip, ctypes.c_double, dp]
        lib.oracle_direct_sum.restype = None
        lib.oracle_G_points.argtypes = [dp, ctypes.c_int, ctypes.c_int64, ip, dp]
        lib.oracle_G_points.restype = None
        lib.oracle_far_field.argtypes = [ctypes.c_double] * 3
        lib.oracle_far_field.restype = ctypes.c_double
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_num_threads.restype = None
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def num_threads():
    return int(_load().oracle_num_threads())


def set_num_threads(n):
    """OpenMP threads of later direct sums (timing the oracle on fewer cores)."""
    _load().oracle_set_num_threads(int(n))


def G_points(ijk):
    """G at integer points via the C lookup (near table + far series)."""
    lib = _load()
    ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
    C = np.ascontiguousarray(lgf_table.near_cube())
    out = np.empty(len(ijk))
    lib.oracle_G_points(_dp(C), lgf_table.R_NEAR, len(ijk), _ip(ijk), _dp(out))
    return out


def direct_sum(src_ijk, f, tgt_ijk, dx=1.0):
    """u[t] = dx^2 * sum_s G(tgt_t - src_s) f_s, all in float64."""
    lib = _load()
    src = np.ascontiguousarray(src_ijk, dtype=np.int32).reshape(-1, 3)
    tgt = np.ascontiguousarray(tgt_ijk, dtype=np.int32).reshape(-1, 3)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
    assert len(f) == len(src)
    C = np.ascontiguousarray(lgf_table.near_cube())
    u = np.empty(len(tgt))
    lib.oracle_direct_sum(_dp(C), lgf_table.R_NEAR, len(src), _ip(src), _dp(f),
                          len(tgt), _ip(tgt), float(dx) * float(dx), _dp(u))
    return u
