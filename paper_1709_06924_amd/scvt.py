"""ctypes binding of libscvt.so (include/scvt.h): argument marshalling only.

Every step of the hot path runs in the HIP library; this module converts
numpy arrays / torch tensors to pointers and status codes to exceptions.  It
raises ImportError when the library has not been built -- there is no CPU
fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscvt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libscvt.so is not built; run `python -m paper_1709_06924_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

SCVT_OK, SCVT_NOT_CONVERGED, SCVT_PENDING = 0, 1, 2
FP64, MIXED = 0, 1
KIND = {"const": 0, "tanh": 1, "x3": 2, "x16": 3}
KERNEL_CELLS, KERNEL_FALLBACK, KERNEL_GRID, KERNEL_LBFGS, KERNEL_EVAL, KERNEL_QUAD = 0, 1, 2, 3, 4, 5
KERNEL_CELLS_WIDE = 6
REFINE_NOALLOC_MAX_N = 655362  # scvt.h SCVT_REFINE_NOALLOC_MAX_N
RECORD_RING = 4096  # scvt.h SCVT_RECORD_RING
VMAX = 32


class Density(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("geodesic", ctypes.c_int32), ("nbumps", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("xc", ctypes.c_double * 6),
                ("beta", ctypes.c_double * 2), ("alpha", ctypes.c_double * 2),
                ("amp", ctypes.c_double * 2), ("gamma", ctypes.c_double),
                ("w_lon", ctypes.c_double), ("w_lat", ctypes.c_double)]


class Config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m_hist", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("rho", Density), ("quad_levels", ctypes.c_int32),
                ("ls_max_evals", ctypes.c_int32), ("ls_c1", ctypes.c_double),
                ("curv_eps", ctypes.c_double), ("ls_noise", ctypes.c_double),
                ("keep_cells", ctypes.c_int32),
                ("method", ctypes.c_int32), ("quad_rule", ctypes.c_int32),
                ("k_max", ctypes.c_int32), ("hip_stream", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int64), ("n_evals", ctypes.c_int64), ("F", ctypes.c_double),
                ("grad_norm2", ctypes.c_double), ("step_inf", ctypes.c_double),
                ("alpha", ctypes.c_double), ("n_fallback", ctypes.c_int64),
                ("n_degenerate", ctypes.c_int64), ("status", ctypes.c_int32),
                ("hist_len", ctypes.c_int32), ("n_lloyd_fallback", ctypes.c_int64),
                ("n_wide", ctypes.c_int64 * 2)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["n_wide"] = list(d["n_wide"])
        return d


_vp, _dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
_H = ctypes.c_void_p
_sig = {
    "scvt_config_init": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.c_int64]),
    "scvt_create": (ctypes.c_int, [ctypes.POINTER(Config), _vp, ctypes.c_int, ctypes.POINTER(_H)]),
    "scvt_step": (ctypes.c_int, [_H, ctypes.POINTER(Info)]),
    "scvt_get_records": (ctypes.c_int, [_H, ctypes.c_int64, ctypes.POINTER(Info),
                                        ctypes.POINTER(ctypes.c_int64)]),
    "scvt_solve": (ctypes.c_int, [_H, ctypes.c_int64, ctypes.c_double, ctypes.POINTER(Info)]),
    "scvt_solve_rel": (ctypes.c_int, [_H, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.POINTER(Info)]),
    "scvt_energy": (ctypes.c_int, [_H, _dp, _vp, _vp, _vp, ctypes.c_int]),
    "scvt_get_generators": (ctypes.c_int, [_H, _vp, ctypes.c_int]),
    "scvt_get_vectors": (ctypes.c_int, [_H, ctypes.c_int, _vp, ctypes.c_int]),
    "scvt_direction": (ctypes.c_int, [_H, _vp, ctypes.c_int, _dp]),
    "scvt_get_cells": (ctypes.c_int, [_H, ctypes.c_int32, _vp, _vp, _vp, _vp]),
    "scvt_get_state": (ctypes.c_int, [_H, _vp, ctypes.POINTER(ctypes.c_size_t)]),
    "scvt_set_state": (ctypes.c_int, [_H, _vp, ctypes.c_size_t]),
    "scvt_set_timing": (ctypes.c_int, [_H, ctypes.c_int]),
    "scvt_kernel_time": (ctypes.c_int, [_H, ctypes.c_int, _dp, ctypes.POINTER(ctypes.c_int64)]),
    "scvt_destroy": (None, [_H]),
    "scvt_num_generators": (ctypes.c_int, [_H, ctypes.POINTER(ctypes.c_int64)]),
    "scvt_refine": (ctypes.c_int, [_H, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]),
    "scvt_mesh": (ctypes.c_int, [_H, _vp, ctypes.POINTER(ctypes.c_int64), _vp, _vp]),
    "scvt_refine_noalloc": (ctypes.c_int, [_H, _vp, ctypes.POINTER(ctypes.c_int64)]),
    "scvt_multilevel": (ctypes.c_int, [ctypes.POINTER(Config), _vp, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int64, ctypes.c_double, ctypes.POINTER(Info),
                                       ctypes.POINTER(_H)]),
    "scvt_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "scvt_footprint": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_size_t)]),
    "scvt_server_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int, _vp, ctypes.POINTER(_H)]),
    "scvt_server_submit": (ctypes.c_int, [_H, ctypes.POINTER(Config), _vp, ctypes.c_double,
                                          ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "scvt_server_poll": (ctypes.c_int, [_H, ctypes.c_int64, _vp, ctypes.POINTER(Info), _dp]),
    "scvt_server_release": (ctypes.c_int, [_H, ctypes.c_int64]),
    "scvt_server_stats": (ctypes.c_int, [_H, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_size_t)]),
    "scvt_server_destroy": (None, [_H]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class ScvtError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, _lib.scvt_strerror(code).decode(), code))


def _check(rc, what):
    if rc < 0:
        raise ScvtError(rc, what)
    return rc


def exported_symbols():
    return list(_sig)


def density_struct(d):
    s = Density()
    s.kind = KIND[d["kind"]]
    s.geodesic = 1 if d.get("geodesic") else 0
    xcs = d.get("xc", [])
    s.nbumps = len(xcs)
    for k, xc in enumerate(xcs[:2]):
        for j in range(3):
            s.xc[3 * k + j] = float(xc[j])
    for name in ("beta", "alpha", "amp"):
        for k, v in enumerate(d.get(name, [])[:2]):
            getattr(s, name)[k] = float(v)
    s.gamma = float(d.get("gamma", 0.0))
    s.w_lon = float(d.get("w_lon", 1.0))
    s.w_lat = float(d.get("w_lat", 1.0))
    return s


METHODS = {"plbfgs": 0, "lloyd": 1, "lbfgs": 2}


def make_config(n, density=None, m_hist=7, precision="fp64", quad_levels=2, ls_max_evals=10,
                ls_c1=1e-4, curv_eps=1e-10, keep_cells=False, stream=None, ls_noise=-1.0,
                method="plbfgs", quad_rule=7, k_max=0):
    c = Config()
    _check(_lib.scvt_config_init(ctypes.byref(c), int(n)), "scvt_config_init")
    c.m_hist = int(m_hist)
    c.precision = MIXED if precision in ("mixed", MIXED) else FP64
    c.rho = density_struct(density or {"kind": "const"})
    c.quad_levels = int(quad_levels)
    c.ls_max_evals = int(ls_max_evals)
    c.ls_c1 = float(ls_c1)
    c.curv_eps = float(curv_eps)
    c.ls_noise = float(ls_noise)
    c.keep_cells = 1 if keep_cells else 0
    c.method = METHODS[method] if isinstance(method, str) else int(method)
    c.quad_rule = int(quad_rule)
    c.k_max = int(k_max)
    c.hip_stream = stream
    return c


def multilevel(z0, density=None, levels=1, max_iter=100, tol=1e-8, **kw):
    """Optimisation-bisection (scvt_multilevel): solve at z0, then `levels`
    times refine and solve again.  Returns (Solver of the last level, list
    of per-level info dicts)."""
    z0 = np.ascontiguousarray(z0, dtype=np.float64)
    cfg = make_config(z0.shape[0], density, **kw)
    infos = (Info * (levels + 1))()
    h = _H()
    rc = _lib.scvt_multilevel(ctypes.byref(cfg), z0.ctypes.data_as(ctypes.c_void_p), 0, int(levels),
                              int(max_iter), float(tol), infos, ctypes.byref(h))
    _check(rc, "scvt_multilevel")
    return Solver._adopt(h, cfg), [infos[k].as_dict() for k in range(levels + 1)]


def _ptr(x, n_expected=None):
    """(pointer, on_device) for a numpy array or a torch tensor."""
    if isinstance(x, np.ndarray):
        assert x.flags["C_CONTIGUOUS"]
        if n_expected is not None:
            assert x.size == n_expected
        return x.ctypes.data_as(ctypes.c_void_p), 0
    # torch tensor
    assert x.is_contiguous()
    if n_expected is not None:
        assert x.numel() == n_expected
    return ctypes.c_void_p(x.data_ptr()), 1 if x.is_cuda else 0


class Solver:
    """One SCVT problem resident on the device (scvt_handle)."""

    def __init__(self, z0, density=None, **kw):
        n = z0.shape[0]
        self.n = n
        self.cfg = make_config(n, density, **kw)
        if isinstance(z0, np.ndarray):
            z0 = np.ascontiguousarray(z0, dtype=np.float64)
        p, dev = _ptr(z0, 3 * n)
        self._z0 = z0
        h = _H()
        _check(_lib.scvt_create(ctypes.byref(self.cfg), p, dev, ctypes.byref(h)), "scvt_create")
        self.h = h
        self.info = Info()

    @classmethod
    def _adopt(cls, h, cfg):
        """Wrap a handle the library created (scvt_multilevel)."""
        self = cls.__new__(cls)
        n = ctypes.c_int64()
        _check(_lib.scvt_num_generators(h, ctypes.byref(n)), "scvt_num_generators")
        self.n = n.value
        self.cfg = cfg
        self.cfg.n = n.value
        self._z0 = None
        self.h = h
        self.info = Info()
        return self

    def refine(self):
        """Bisection: the generators followed by the normalised midpoints of
        all Delaunay edges (scvt_refine), as an (m, 3) array."""
        m = ctypes.c_int64()
        _check(_lib.scvt_refine(self.h, None, 0, ctypes.byref(m)), "scvt_refine")
        out = np.zeros((m.value, 3))
        _check(_lib.scvt_refine(self.h, out.ctypes.data_as(ctypes.c_void_p), 0, ctypes.byref(m)),
               "scvt_refine")
        return out

    def mesh(self):
        """(triangles (ntri, 3) int32, cellQ (n,), triQ (ntri,)) at the
        current generators (scvt_mesh)."""
        nt = ctypes.c_int64()
        _check(_lib.scvt_mesh(self.h, None, ctypes.byref(nt), None, None), "scvt_mesh")
        tri = np.zeros((nt.value, 3), np.int32)
        cq = np.zeros(self.n)
        tq = np.zeros(nt.value)
        _check(_lib.scvt_mesh(self.h, tri.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nt),
                              cq.ctypes.data_as(ctypes.c_void_p), tq.ctypes.data_as(ctypes.c_void_p)),
               "scvt_mesh")
        return tri, cq, tq

    def close(self):
        if getattr(self, "h", None) and _lib is not None:  # _lib is None at interpreter exit
            _lib.scvt_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def step(self):
        _check(_lib.scvt_step(self.h, ctypes.byref(self.info)), "scvt_step")
        return self.info.as_dict()

    def records(self, max_records=RECORD_RING):
        """The last per-iteration records (the initial evaluation's and one
        after every iteration, at most RECORD_RING), oldest first, as dicts."""
        buf = (Info * max_records)()
        cnt = ctypes.c_int64()
        _check(_lib.scvt_get_records(self.h, int(max_records), buf, ctypes.byref(cnt)),
               "scvt_get_records")
        return [buf[k].as_dict() for k in range(cnt.value)]

    def solve(self, max_iter, tol):
        rc = _check(_lib.scvt_solve(self.h, int(max_iter), float(tol), ctypes.byref(self.info)),
                    "scvt_solve")
        d = self.info.as_dict()
        d["converged"] = rc == SCVT_OK
        return d

    def solve_rel(self, max_iter, step_tol=0.0, grad_rel_tol=0.0, f_rel_tol=0.0):
        """Stopping tests of the paper's method comparison (scvt_solve_rel)."""
        rc = _check(_lib.scvt_solve_rel(self.h, int(max_iter), float(step_tol),
                                        float(grad_rel_tol), float(f_rel_tol),
                                        ctypes.byref(self.info)), "scvt_solve_rel")
        d = self.info.as_dict()
        d["converged"] = rc == SCVT_OK
        return d

    def energy(self):
        F = ctypes.c_double()
        m = np.zeros(self.n)
        c = np.zeros((self.n, 3))
        e = np.zeros(self.n)
        _check(_lib.scvt_energy(self.h, ctypes.byref(F), m.ctypes.data_as(ctypes.c_void_p),
                                c.ctypes.data_as(ctypes.c_void_p),
                                e.ctypes.data_as(ctypes.c_void_p), 0), "scvt_energy")
        return F.value, m, c, e

    def generators(self, out=None):
        if out is None:
            out = np.zeros((self.n, 3))
        p, dev = _ptr(out, 3 * self.n)
        _check(_lib.scvt_get_generators(self.h, p, dev), "scvt_get_generators")
        return out

    def vector(self, which):
        names = {"g": 0, "h": 1, "lloyd": 2, "mu": 3, "q": 4, "R": 5}
        w = names.get(which, which)
        out = np.zeros(self.n) if w in (1, 5) else np.zeros((self.n, 3))
        _check(_lib.scvt_get_vectors(self.h, w, out.ctypes.data_as(ctypes.c_void_p), 0),
               "scvt_get_vectors")
        return out

    def direction(self):
        q = np.zeros((self.n, 3))
        gq = ctypes.c_double()
        _check(_lib.scvt_direction(self.h, q.ctypes.data_as(ctypes.c_void_p), 0, ctypes.byref(gq)),
               "scvt_direction")
        return q, gq.value

    def cells(self):
        nbr = np.zeros((self.n, VMAX), np.int32)
        deg = np.zeros(self.n, np.int32)
        verts = np.zeros((self.n, VMAX, 6))
        flags = np.zeros(self.n, np.uint8)
        _check(_lib.scvt_get_cells(self.h, VMAX, nbr.ctypes.data_as(ctypes.c_void_p),
                                   deg.ctypes.data_as(ctypes.c_void_p),
                                   verts.ctypes.data_as(ctypes.c_void_p),
                                   flags.ctypes.data_as(ctypes.c_void_p)), "scvt_get_cells")
        return nbr, deg, verts, flags

    def neighbours(self):
        """Neighbour lists (n, 32; -1 padded) and degrees of the current
        cells (scvt_get_cells without vertices; needs keep_cells)."""
        nbr = np.zeros((self.n, VMAX), np.int32)
        deg = np.zeros(self.n, np.int32)
        _check(_lib.scvt_get_cells(self.h, VMAX, nbr.ctypes.data_as(ctypes.c_void_p),
                                   deg.ctypes.data_as(ctypes.c_void_p), None, None),
               "scvt_get_cells")
        return nbr, deg

    def degrees(self):
        """Voronoi degree of every cell at the current generators."""
        deg = np.zeros(self.n, np.int32)
        _check(_lib.scvt_get_cells(self.h, VMAX, None, deg.ctypes.data_as(ctypes.c_void_p), None,
                                   None), "scvt_get_cells")
        return deg

    def get_state(self):
        nb = ctypes.c_size_t()
        _check(_lib.scvt_get_state(self.h, None, ctypes.byref(nb)), "scvt_get_state")
        buf = ctypes.create_string_buffer(nb.value)
        _check(_lib.scvt_get_state(self.h, buf, ctypes.byref(nb)), "scvt_get_state")
        return buf.raw

    def set_state(self, blob):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(_lib.scvt_set_state(self.h, buf, len(blob)), "scvt_set_state")

    def set_timing(self, on=True, quad_only=False):
        """Kernel timers: all of them, or (quad_only) only the quadrature
        kernel's (two events per evaluation); on=False turns them off."""
        level = 0 if not on else (2 if quad_only else 1)
        _check(_lib.scvt_set_timing(self.h, level), "scvt_set_timing")

    def kernel_time(self, kernel):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check(_lib.scvt_kernel_time(self.h, int(kernel), ctypes.byref(ms), ctypes.byref(cnt)),
               "scvt_kernel_time")
        return ms.value, cnt.value


def footprint(n, density=None, **kw):
    """Device bytes a solver with this configuration allocates."""
    c = make_config(n, density, **kw)
    b = ctypes.c_size_t()
    _check(_lib.scvt_footprint(ctypes.byref(c), ctypes.byref(b)), "scvt_footprint")
    return b.value


class Server:
    """Continuous-batching request loop (scvt_server): submit requests at any
    time, poll for results.  Admission by slots and HBM footprint; all
    admitted requests advance together in rounds of segmented launches on
    `stream` (a hipStream_t as an int, or None for the server's own)."""

    def __init__(self, hbm_budget, max_slots=8, stream=None):
        h = _H()
        _check(_lib.scvt_server_create(int(hbm_budget), int(max_slots), stream, ctypes.byref(h)),
               "scvt_server_create")
        self.h = h
        self.n_of = {}

    def submit(self, z0, density, tol, max_iter, **kw):
        z0 = np.ascontiguousarray(z0, dtype=np.float64)
        c = make_config(len(z0), density, **kw)
        rid = ctypes.c_int64()
        _check(_lib.scvt_server_submit(self.h, ctypes.byref(c), z0.ctypes.data_as(ctypes.c_void_p),
                                       float(tol), int(max_iter), ctypes.byref(rid)),
               "scvt_server_submit")
        self.n_of[rid.value] = len(z0)
        return rid.value

    def poll(self, rid, want_z=True):
        """None while pending, else a dict with status, info, times, z."""
        n = self.n_of[rid]
        z = np.zeros((n, 3)) if want_z else None
        info = Info()
        times = np.zeros(3)
        rc = _lib.scvt_server_poll(self.h, int(rid),
                                   z.ctypes.data_as(ctypes.c_void_p) if want_z else None,
                                   ctypes.byref(info), times.ctypes.data_as(_dp))
        if rc == SCVT_PENDING:
            return None
        return {"status": rc, "info": info.as_dict(), "t_submit": times[0], "t_start": times[1],
                "t_done": times[2], "z": z}

    def release(self, rid):
        _check(_lib.scvt_server_release(self.h, int(rid)), "scvt_server_release")
        self.n_of.pop(rid, None)

    def stats(self):
        w, r, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
        _check(_lib.scvt_server_stats(self.h, ctypes.byref(w), ctypes.byref(r), ctypes.byref(b)),
               "scvt_server_stats")
        return {"waiting": w.value, "running": r.value, "bytes_used": b.value}

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.scvt_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()
