"""ctypes front end of the C oracle (``mips_oracle.c``).  TEST INFRASTRUCTURE ONLY.

Result definition (Section II-B problem statement, Section II-C brute force):
for each user the K items with the largest inner product, with the keys summed
in float64 left to right over the factors and ties broken by the lower item
index.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mips_oracle.c")
_LIB = os.path.join(_HERE, "libmips_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain IEEE double, no contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared",
               "-fPIC", "-std=c99", "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        f32p = ctypes.POINTER(ctypes.c_float)
        f64p = ctypes.POINTER(ctypes.c_double)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_key.restype = ctypes.c_double
        lib.oracle_key.argtypes = [f32p, f32p, ctypes.c_int32]
        lib.oracle_user_keys.restype = None
        lib.oracle_user_keys.argtypes = [f32p, f32p, ctypes.c_int64, ctypes.c_int32, f64p]
        lib.oracle_pair_keys.restype = ctypes.c_int
        lib.oracle_pair_keys.argtypes = [f32p, ctypes.c_int64, f32p, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.c_int32, i32p, f64p]
        lib.oracle_topk.restype = ctypes.c_int
        lib.oracle_topk.argtypes = [f32p, ctypes.c_int64, f32p, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, i32p, f64p, ctypes.c_int32]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = [ctypes.c_int32]
        _lib = lib
    return _lib


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def key(u, i) -> float:
    """FP64 key of one pair, summed left to right."""
    u, up = _f32(u)
    i, ip = _f32(i)
    assert u.shape == i.shape and u.ndim == 1
    return _load().oracle_key(up, ip, u.shape[0])


def user_keys(u, I) -> np.ndarray:
    """Keys of one user against every item."""
    u, up = _f32(u)
    I, Ip = _f32(I)
    out = np.empty(I.shape[0], dtype=np.float64)
    _load().oracle_user_keys(up, Ip, I.shape[0], I.shape[1],
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def pair_keys(U, I, idx) -> np.ndarray:
    """Keys of the pairs (r, idx[r, k]): float64 [n_u, K]."""
    U, Up = _f32(U)
    I, Ip = _f32(I)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    assert idx.ndim == 2 and idx.shape[0] == U.shape[0]
    out = np.empty(idx.shape, dtype=np.float64)
    rc = _load().oracle_pair_keys(Up, U.shape[0], Ip, I.shape[0], U.shape[1], idx.shape[1],
                                  idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError("pair_keys: index out of range")
    return out


def topk(U, I, K: int, mode: int = 1, nthreads: int = 0):
    """Top-K per user: (idx int32 [n_u, K], key float64 [n_u, K]).

    mode 0 sorts all items per user; mode 1 keeps a sorted K-list.
    """
    U, Up = _f32(U)
    I, Ip = _f32(I)
    assert U.ndim == 2 and I.ndim == 2 and U.shape[1] == I.shape[1]
    n_u, f = U.shape
    n_i = I.shape[0]
    idx = np.empty((n_u, K), dtype=np.int32)
    kk = np.empty((n_u, K), dtype=np.float64)
    rc = _load().oracle_topk(Up, n_u, Ip, n_i, f, K, mode,
                             idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             kk.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nthreads)
    if rc != 0:
        raise ValueError(f"oracle_topk failed with {rc}")
    return idx, kk


def num_threads(nthreads: int = 0) -> int:
    return _load().oracle_num_threads(nthreads)
