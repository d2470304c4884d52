"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke
check.  This module holds no arithmetic of the method: it draws generators,
spells out density parameters and the serving request stream.

Workloads (the paper's experiments use analytic densities and Monte-Carlo or
uniform starts, section 4; these synthetic stand-ins keep that structure):
  C1  n=2,562      rho = 1                          M=7   seed 1
  C2  n=163,842    tanh bump, lat 30 lon 90, beta pi/6, alpha 0.2, 8x
  C3  n=1,048,576  tanh bump, lat 30 lon 90, beta pi/9, alpha 0.15, 16x, M=10
  C4  serving stream: Poisson 20 req/s, n log-uniform in [10242, 655362]
  C5  n=4,194,304  two bumps at lat +-45, 16x and 8x, M=10
Densities are dicts understood by both the HIP binding and the oracle:
  {"kind": "const"}
  {"kind": "tanh", "xc": [[x,y,z],...], "beta": [...], "alpha": [...],
   "amp": [...], "gamma": g, "geodesic": bool}
     rho = gamma + sum_k amp_k * (tanh((beta_k - d_k)/alpha_k) + 1) / 2
  {"kind": "x3", "gamma": g}            rho = (1-gamma) z^4 + gamma
  {"kind": "x16", ...}                  anisotropic bump of section 4
"""
import math

import numpy as np


def uniform_sphere(n, seed):
    """n points uniform on the unit sphere: rows of default_rng(seed)
    standard normals, each scaled to unit length."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((int(n), 3))
    Z /= np.linalg.norm(Z, axis=1)[:, None]
    return np.ascontiguousarray(Z)


def cap_points(u, theta, m, seed):
    """m points within angle ~theta of the unit vector u: tangent-plane
    offsets uniform in a disc of radius theta (default_rng(seed)), then
    projected to the sphere (a dense cluster of generators)."""
    rng = np.random.default_rng(seed)
    u = np.asarray(u, float) / np.linalg.norm(u)
    e1 = np.cross(u, [0.3, 0.5, 0.8])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(u, e1)
    r = theta * np.sqrt(rng.uniform(size=m))
    ph = rng.uniform(0.0, 2 * math.pi, m)
    P = u + (r * np.cos(ph))[:, None] * e1 + (r * np.sin(ph))[:, None] * e2
    return np.ascontiguousarray(P / np.linalg.norm(P, axis=1)[:, None])


def toward(xc, chord, seed):
    """A unit vector at the given chord distance from the unit vector xc
    (in a direction drawn from default_rng(seed))."""
    rng = np.random.default_rng(seed)
    xc = np.asarray(xc, float)
    w = np.cross(xc, rng.standard_normal(3))
    w /= np.linalg.norm(w)
    a = 2.0 * math.asin(chord / 2.0)
    return math.cos(a) * xc + math.sin(a) * w


def latlon(lat_deg, lon_deg):
    la, lo = math.radians(lat_deg), math.radians(lon_deg)
    return [math.cos(la) * math.cos(lo), math.cos(la) * math.sin(lo), math.sin(la)]


def density_const():
    return {"kind": "const"}


def density_tanh(xc, beta, alpha, ratio, geodesic=False):
    """One tanh bump; gamma = ratio**-4 so that the spacing ratio is `ratio`
    (mesh spacing scales as rho**-1/4, section 4)."""
    gamma = float(ratio) ** -4
    return {"kind": "tanh", "xc": [list(map(float, xc))], "beta": [float(beta)],
            "alpha": [float(alpha)], "amp": [1.0 - gamma], "gamma": gamma,
            "geodesic": bool(geodesic)}


def density_two_centre():
    """Two bumps at lat +45 / -45 (lon 0): 16x and 8x finer than the floor."""
    gamma = 16.0 ** -4
    return {"kind": "tanh", "xc": [latlon(45, 0), latlon(-45, 0)],
            "beta": [math.pi / 6, math.pi / 6], "alpha": [0.2, 0.2],
            "amp": [1.0 - gamma, 2.0 ** -4 - gamma], "gamma": gamma, "geodesic": False}


def density_x3():
    return {"kind": "x3", "gamma": 3.0 ** -4}


def density_x16():
    return {"kind": "x16", "xc": [[1.0, 0.0, 0.0]], "beta": [math.pi / 6], "alpha": [0.3],
            "amp": [1.0 - 16.0 ** -4], "gamma": 16.0 ** -4, "w_lon": 0.3, "w_lat": 1.2}


def density_x64():
    gamma = 64.0 ** -4
    return {"kind": "tanh", "xc": [[0.0, -0.866, 0.5]], "beta": [math.pi / 6], "alpha": [0.15],
            "amp": [1.0 - gamma], "gamma": gamma, "geodesic": True}


CONFIGS = {
    "C1": dict(name="n2562_const_fp64", n=2562, density=density_const(), m_hist=7,
               max_iter=100, tol=1e-10, seed=1),
    "C2": dict(name="n163842_tanh8x_fp64", n=163842,
               density=density_tanh(latlon(30, 90), math.pi / 6, 0.2, 8), m_hist=7,
               max_iter=20000, tol=1e-8, seed=2),
    "C3": dict(name="n1048576_tanh16x", n=1048576,
               density=density_tanh(latlon(30, 90), math.pi / 9, 0.15, 16), m_hist=10,
               max_iter=200, tol=0.0, seed=3),
    "C5": dict(name="n4194304_twocentre", n=4194304, density=density_two_centre(), m_hist=10,
               max_iter=100, tol=0.0, seed=5),
}


def serving_stream(seed=4, rate=20.0, count=200, n_lo=10242, n_hi=655362):
    """Open-loop Poisson arrivals; every request gets its own tanh density.
    Returns dicts with arrival time (s), n, density, z0 seed."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        c = rng.standard_normal(3)
        c /= np.linalg.norm(c)
        beta = rng.uniform(math.pi / 12, math.pi / 4)
        alpha = rng.uniform(0.1, 0.3)
        ratio = rng.uniform(4.0, 16.0)
        out.append(dict(id=rid, t=t, n=n, density=density_tanh(c, beta, alpha, ratio),
                        z0_seed=seed * 10**6 + rid))
    return out


def platonic(name):
    """Vertices of a Platonic solid (tetra, octa, icosa, cube, dodeca) or of
    the icosidodecahedron, on the unit sphere."""
    if name == "tetra":
        P = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=float)
    elif name == "octa":
        P = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                     dtype=float)
    elif name == "icosa":
        p = (1 + 5 ** 0.5) / 2
        P = []
        for a in (-1, 1):
            for b in (-p, p):
                P += [[0, a, b], [a, b, 0], [b, 0, a]]
        P = np.array(P, dtype=float)
    elif name == "cube":
        P = np.array([[a, b, c] for a in (-1, 1) for b in (-1, 1) for c in (-1, 1)], dtype=float)
    elif name == "dodeca":  # 20 vertices; its pentagonal faces put 5 points on a circle
        p = (1 + 5 ** 0.5) / 2
        P = [[a, b, c] for a in (-1, 1) for b in (-1, 1) for c in (-1, 1)]
        for a in (-1, 1):
            for b in (-1, 1):
                P += [[0, a / p, b * p], [a / p, b * p, 0], [b * p, 0, a / p]]
        P = np.array(P, dtype=float)
    elif name == "icosidodeca":  # 30 vertices (edge midpoints of the icosahedron)
        p = (1 + 5 ** 0.5) / 2
        P = []
        for a in (-1, 1):
            P += [[0, 0, a * p], [0, a * p, 0], [a * p, 0, 0]]
            for b in (-1, 1):
                for c in (-1, 1):
                    v = [a * 0.5, b * p / 2, c * p * p / 2]
                    P += [v, [v[2], v[0], v[1]], [v[1], v[2], v[0]]]
        P = np.array(P, dtype=float)
    else:
        raise ValueError(name)
    return np.ascontiguousarray(P / np.linalg.norm(P, axis=1)[:, None])
