"""Build and load the host build of the HIP path's geometry (tests/host)."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "host", "cellcheck.cpp")
HDR = os.path.join(ROOT, "paper_1709_06924_amd", "csrc", "cellgeom.h")
LIB = os.path.join(HERE, "host", "libcellcheck.so")

_lib = None


def build():
    if os.path.exists(LIB) and os.path.getmtime(LIB) >= max(os.path.getmtime(SRC), os.path.getmtime(HDR)):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.dirname(HDR), "-x", "hip", SRC, "-o", tmp]
    subprocess.check_call(cmd, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(LIB)
    return _lib


def P(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def cells(Z, rad, cap=64):
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    n = len(Z)
    rad = np.ascontiguousarray(np.broadcast_to(rad, (n,)), dtype=np.float64)
    st = np.zeros(n, np.int32)
    deg = np.zeros(n, np.int32)
    nbr = np.zeros((n, 32), np.int32)
    verts = np.zeros((n, 32, 6))
    R = np.zeros(n)
    lib().hc_cells(ctypes.c_int64(n), P(Z), P(rad), P(st), P(deg), P(nbr), P(verts), P(R),
                   ctypes.c_int(cap))
    return st, deg, nbr, verts, R


def clip(Z, i):
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    deg = np.zeros(1, np.int32)
    nbr = np.zeros(32, np.int32)
    verts = np.zeros((32, 6))
    flags = np.zeros(1, np.int32)
    R = np.zeros(1)
    lib().hc_clip(ctypes.c_int64(len(Z)), P(Z), ctypes.c_int64(i), P(deg), P(nbr), P(verts),
                  P(flags), P(R))
    return int(deg[0]), nbr, verts, int(flags[0]), float(R[0])


class CDensity(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("geodesic", ctypes.c_int32), ("nbumps", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("xc", ctypes.c_double * 6), ("beta", ctypes.c_double * 2),
                ("alpha", ctypes.c_double * 2), ("amp", ctypes.c_double * 2),
                ("gamma", ctypes.c_double), ("w_lon", ctypes.c_double), ("w_lat", ctypes.c_double),
                ("k2", ctypes.c_double * 2), ("K", ctypes.c_double * 2),
                ("bK", ctypes.c_double * 2), ("Ks", ctypes.c_double * 2),
                ("cc", ctypes.c_double * 2), ("Kt", ctypes.c_double * 2),
                ("poly_r2", ctypes.c_double * 2), ("poly_near2", ctypes.c_double * 2),
                ("poly_tab", ctypes.c_void_p), ("poly_n", ctypes.c_int64),
                ("polyx_tab", ctypes.c_void_p * 2), ("polyx_n", ctypes.c_int64)]


KIND = {"const": 0, "tanh": 1, "x3": 2, "x16": 3}


def cdensity(d):
    c = CDensity()
    c.kind = KIND[d["kind"]]
    c.geodesic = 1 if d.get("geodesic") else 0
    xcs = d.get("xc", [])
    c.nbumps = len(xcs)
    for k, xc in enumerate(xcs[:2]):
        for j in range(3):
            c.xc[3 * k + j] = xc[j]
    for name in ("beta", "alpha", "amp"):
        for k, v in enumerate(d.get(name, [])[:2]):
            getattr(c, name)[k] = v
    c.gamma = d.get("gamma", 0.0)
    c.w_lon = d.get("w_lon", 1.0)
    c.w_lat = d.get("w_lat", 1.0)
    return c


def quad(z, E, verts, density, levels=2, rule=7):
    z = np.ascontiguousarray(z, dtype=np.float64)
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    out = np.zeros(5)
    D = cdensity(density)
    lib().hc_quad(P(z), ctypes.c_int(E), P(verts), ctypes.byref(D), ctypes.c_int(levels),
                  ctypes.c_int(rule), P(out))
    return out


def quad_poly(z, E, verts, density, levels=2, rule=7, force=0):
    """Cell integrals through the per-cell density polynomial as the kernel
    chooses it (force 1: only the expansion in t, 2: only in x); returns
    (integrals, mode) with mode 2 for x, 1 for t, or None if the cell does
    not qualify."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    out = np.zeros(5)
    D = cdensity(density)
    mode = lib().hc_quad_poly(P(z), ctypes.c_int(E), P(verts), ctypes.byref(D),
                              ctypes.c_int(levels), ctypes.c_int(rule), P(out), ctypes.c_int(force))
    return (out, mode) if mode else None


def rho_poly(z, density, Y, mode=0):
    """rho at unit points Y from generator z's table entry (mode 0: the
    expansion in t, 1: in x) and directly; also the x entry's radius."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    poly = np.zeros(len(Y))
    exact = np.zeros(len(Y))
    lim = np.zeros(1)
    D = cdensity(density)
    lib().hc_rho_poly(P(z), ctypes.byref(D), ctypes.c_int64(len(Y)), P(Y), P(poly), P(exact),
                      ctypes.c_int(mode), P(lim))
    return poly, exact, float(lim[0])


def quad_mixed_poly(z, E, verts, density, levels=2, rule=7):
    """Mixed-precision cell integrals through the FP32 expansions in x (one
    or two bumps), or None if the cell does not qualify."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    out = np.zeros(5)
    D = cdensity(density)
    ok = lib().hc_quad_mixed_poly(P(z), ctypes.c_int(E), P(verts), ctypes.byref(D),
                                  ctypes.c_int(levels), ctypes.c_int(rule), P(out))
    return out if ok else None


def quad_mixed(z, E, verts, density, levels=2, rule=7):
    z = np.ascontiguousarray(z, dtype=np.float64)
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    out = np.zeros(5)
    D = cdensity(density)
    lib().hc_quad_mixed(P(z), ctypes.c_int(E), P(verts), ctypes.byref(D), ctypes.c_int(levels),
                        ctypes.c_int(rule), P(out))
    return out


def grid(n):
    GBW = np.zeros(3, np.int32)
    dd = np.zeros(3)
    lib().hc_grid(ctypes.c_int64(n), P(GBW), P(dd))
    return GBW, dd


def window(GBW, dd, z, rt, maxw=63):
    out = np.zeros(5, np.int32)
    D = np.zeros(1)
    z = np.ascontiguousarray(z, dtype=np.float64)
    lib().hc_window(P(GBW), P(dd), P(z), ctypes.c_double(rt), ctypes.c_int(maxw), P(out), P(D))
    return out, float(D[0])


def cell_on_face(GBW, dd, Pts, f):
    Pts = np.ascontiguousarray(Pts, dtype=np.float64)
    out = np.zeros(len(Pts), np.int64)
    lib().hc_cell_on_face(P(GBW), P(dd), ctypes.c_int64(len(Pts)), P(Pts), ctypes.c_int(f), P(out))
    return out


def home_face(Pts):
    Pts = np.ascontiguousarray(Pts, dtype=np.float64)
    out = np.zeros(len(Pts), np.int32)
    lib().hc_home_face(ctypes.c_int64(len(Pts)), P(Pts), P(out))
    return out


def exp2_n(u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    lib().hc_exp(ctypes.c_int64(len(u)), P(u), P(out))
    return out


def leaves2(A, B, C):
    abc = np.ascontiguousarray(np.concatenate([A, B, C]), dtype=np.float64)
    out = np.zeros(16 * 18)
    lib().hc_leaves2(P(abc), P(out))
    out = out.reshape(16, 2, 3, 3)
    return out[:, 0], out[:, 1]
