"""Triangle rules of the oracle, built from their definitions (test
infrastructure only).

    rule(7) -- Radon's 7-point degree-5 rule (Stroud T2:5-1), as the C oracle
               computes it from sqrt(15);
    rule(4), rule(9) -- the conical product rules (Stroud) of 2 x 2 and 3 x 3
               points, degrees 3 and 5: on the triangle (0,0), (1,0), (0,1)
               substitute (x, y) = (u, v (1 - u)), dx dy = (1 - u) du dv, and
               take Gauss-Jacobi points in u (weight 1 - u) times
               Gauss-Legendre points in v.  The paper integrates with unnamed
               4- and 9-point rules (section 4.1); these are rules of those
               sizes.

Returned as (lam (nq, 3) barycentric for (A, B, C), w (nq,) summing to 1).
"""
import numpy as np
from scipy.special import roots_jacobi, roots_legendre

from . import _clib


def radon7():
    lam = np.zeros(21)
    w = np.zeros(7)
    _clib.lib().oracle_rule7(_clib.ptr(lam), _clib.ptr(w))
    return lam.reshape(7, 3), w


def conical(k):
    tj, wj = roots_jacobi(k, 1.0, 0.0)   # on [-1, 1], weight (1 - t)
    tl, wl = roots_legendre(k)
    u = (1.0 + tj) / 2.0                   # int_0^1 (1-u) f = sum wj/4 f(u)
    v = (1.0 + tl) / 2.0                   # int_0^1 g = sum wl/2 g(v)
    lam, w = [], []
    for ui, wi in zip(u, wj):
        for vj, wk in zip(v, wl):
            x, y = ui, vj * (1.0 - ui)
            lam.append((1.0 - x - y, x, y))
            w.append(wi * wk / 4.0)        # (wi/4)(wk/2) over the area 1/2
    return np.array(lam), np.array(w)


def rule(nq):
    if nq == 7:
        return radon7()
    if nq == 4:
        return conical(2)
    if nq == 9:
        return conical(3)
    raise ValueError("rules: 4, 7 or 9 points")


def crule(nq):
    lam, w = rule(nq)
    return _clib.crule(lam, w)
