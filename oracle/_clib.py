"""Loader for the oracle's C integrals (oracle/scvt_oracle.c).

Test infrastructure only: the tests, the smoke check and the benchmark's CPU
baseline may import it; the product path never does.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scvt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_scvt.so")

RHO_CONST, RHO_TANH, RHO_X3, RHO_X16 = 0, 1, 2, 3
_KIND = {"const": RHO_CONST, "tanh": RHO_TANH, "x3": RHO_X3, "x16": RHO_X16}


class CDensity(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("geodesic", ctypes.c_int32),
        ("nbumps", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("xc", ctypes.c_double * 6),
        ("beta", ctypes.c_double * 2),
        ("alpha", ctypes.c_double * 2),
        ("amp", ctypes.c_double * 2),
        ("gamma", ctypes.c_double),
        ("w_lon", ctypes.c_double),
        ("w_lat", ctypes.c_double),
    ]


def build(force=False):
    """Compile the oracle's C file with gcc (plain FP64, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
           "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


class CRule(ctypes.Structure):
    _fields_ = [("nq", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("lam", ctypes.c_double * 48), ("w", ctypes.c_double * 16)]


def crule(lam, w):
    """A rule as the C struct: lam (nq, 3) barycentric points, w (nq,)."""
    r = CRule()
    r.nq = len(w)
    for q in range(len(w)):
        for k in range(3):
            r.lam[3 * q + k] = float(lam[q][k])
        r.w[q] = float(w[q])
    return r


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_rule7.argtypes = [dp, dp]
        L.oracle_rho.argtypes = [ctypes.POINTER(CDensity), dp]
        L.oracle_rho.restype = ctypes.c_double
        L.oracle_rho_many.argtypes = [ctypes.POINTER(CDensity), ctypes.c_int64, dp, dp]
        L.oracle_triangle_integrals.argtypes = [ctypes.POINTER(CDensity), dp, dp, dp, dp,
                                                ctypes.c_int, ctypes.POINTER(CRule), dp]
        L.oracle_cell_integrals.argtypes = [ctypes.c_int64, dp, ctypes.POINTER(ctypes.c_int64), dp,
                                            ctypes.POINTER(CDensity), ctypes.c_int,
                                            ctypes.POINTER(CRule), dp, dp, dp]
        L.oracle_cell_integrals.restype = ctypes.c_int
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def cdensity(d):
    """Convert a density description (dict) into the C struct."""
    c = CDensity()
    c.kind = _KIND[d["kind"]]
    c.geodesic = 1 if d.get("geodesic", False) else 0
    xcs = d.get("xc", [])
    c.nbumps = len(xcs)
    for k, xc in enumerate(xcs[:2]):
        for j in range(3):
            c.xc[3 * k + j] = float(xc[j])
    for name in ("beta", "alpha", "amp"):
        vals = d.get(name, [])
        arr = getattr(c, name)
        for k, v in enumerate(vals[:2]):
            arr[k] = float(v)
    c.gamma = float(d.get("gamma", 0.0))
    c.w_lon = float(d.get("w_lon", 1.0))
    c.w_lat = float(d.get("w_lat", 1.0))
    return c


def ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
