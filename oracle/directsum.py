"""ctypes wrapper of the plain-C FP64 direct sum (oracle/directsum.c).

TEST INFRASTRUCTURE ONLY (see package docstring).  `build_lib()` compiles it
with gcc -fopenmp into oracle/_directsum.so; `load()` loads it, compiling first
if it is missing.
"""
import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "directsum.c")
_LIB = os.path.join(_HERE, "_directsum.so")
_lib = None


def build_lib():
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"])
    return _LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_lib()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.acom_oracle_directsum.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_int, P(ctypes.c_double), P(ctypes.c_double),
            ctypes.c_int, P(ctypes.c_longlong), P(ctypes.c_float), P(ctypes.c_float), P(ctypes.c_float),
            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
            P(ctypes.c_double), P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_double), P(ctypes.c_double),
            ctypes.c_int]
        lib.acom_oracle_directsum.restype = ctypes.c_int
        lib.acom_oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def zone_scores(plan, offsets, qx, qy, I, nthreads=0):
    """Per pattern and zone: best value over (n, mirror), its n and mirror, and the
    two cyclic neighbours in that branch.  Inputs are the stored FP32 peaks."""
    lib = load()
    prm = plan["params"]
    P = np.ascontiguousarray(plan["P"], dtype=np.float64)
    Z, N, R = P.shape
    q_s = np.ascontiguousarray(plan["q_s"], dtype=np.float64)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    qx = np.ascontiguousarray(qx, dtype=np.float32)
    qy = np.ascontiguousarray(qy, dtype=np.float32)
    I = np.ascontiguousarray(I, dtype=np.float32)
    n = len(off) - 1
    zs = np.zeros((n, Z))
    zn = np.zeros((n, Z), dtype=np.int32)
    zm = np.zeros((n, Z), dtype=np.int32)
    cm1 = np.zeros((n, Z))
    cp1 = np.zeros((n, Z))
    sigma = prm.sigma if prm.sigma is not None else 0.5 * prm.delta
    rc = lib.acom_oracle_directsum(Z, N, R, _ptr(P, ctypes.c_double), _ptr(q_s, ctypes.c_double), n,
                                   _ptr(off, ctypes.c_longlong), _ptr(qx, ctypes.c_float),
                                   _ptr(qy, ctypes.c_float), _ptr(I, ctypes.c_float), prm.delta,
                                   prm.gamma, prm.omega, prm.kind, sigma, _ptr(zs, ctypes.c_double),
                                   _ptr(zn, ctypes.c_int), _ptr(zm, ctypes.c_int),
                                   _ptr(cm1, ctypes.c_double), _ptr(cp1, ctypes.c_double), int(nthreads))
    if rc != 0:
        raise MemoryError("oracle direct sum: allocation failed")
    return {"score": zs, "n": zn, "mirror": zm, "cm1": cm1, "cp1": cp1}


def num_threads():
    return load().acom_oracle_num_threads()
