"""SCVT energy, gradient, Lloyd preconditioner and the preconditioned LBFGS
loop (oracle).

Test infrastructure only.

Per generator (sections 2.2.1 and 3.1):
    m_i  = int rho,  mu_i = int y rho  (the paper's c_i),  e_i = int |y-z_i|^2 rho
    F    = sum_i e_i                                             (CCVT energy)
    g_i  = 2 (mu_i . z_i) z_i - 2 mu_i          tangential gradient, section 3.1
    h_i  = 1 / (2 mu_i . z_i)                   spherical Lloyd preconditioner
    l_i  = mu_i/|mu_i| - z_i                    Lloyd step: the constrained
                                                centroid (radial projection of
                                                the mass centroid) minus z_i
The P-LBFGS direction is the LBFGS two-loop recursion (section 2.2.2) with
the initial inverse Hessian replaced by diag(h_i) applied to all three
coordinates of generator i (section 3.1, eq. precStep and the spherical form
of eq. loyInit).  The line search is the documented reading: Armijo
backtracking from alpha = 1 (the Lloyd step length, section 3.1), factor 1/2,
c1 = 1e-4, at most ten evaluations (section 4: ten evaluations, M = 7 by
default); every trial point is projected back to the sphere (section 3.1).
When no trial passes, the history is cleared and the Lloyd step itself is
taken (it decreases the exact F without a line search, section 2.2.1); if
the evaluated F rises beyond rounding (1e-13 relative) all the same,
LineSearchError is raised and the generators stay where they were.
"""
import numpy as np

from . import _clib
from .voronoi import cells as _cells


def dot(a, b):
    """Dot product of two flattened arrays with numpy's pairwise summation."""
    return float(np.sum(np.ravel(a) * np.ravel(b)))


def normalize_rows(X):
    return X / np.linalg.norm(X, axis=1)[:, None]


def cell_integrals(C, density, levels=2, rule=7):
    """m (n,), mu (n,3), e (n,) for the cells C (oracle.voronoi.Cells), with
    the triangle rule of `rule` points (oracle.rules)."""
    from .rules import crule
    L = _clib.lib()
    n = len(C.ptr) - 1
    Z = np.ascontiguousarray(C.Z, dtype=np.float64)
    V = np.ascontiguousarray(C.verts, dtype=np.float64)
    ptr = np.ascontiguousarray(C.ptr, dtype=np.int64)
    m = np.zeros(n)
    mu = np.zeros((n, 3))
    e = np.zeros(n)
    D = _clib.cdensity(density)
    import ctypes
    rc = L.oracle_cell_integrals(n, _clib.ptr(Z), ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 _clib.ptr(V), ctypes.byref(D), int(levels),
                                 ctypes.byref(crule(rule)), _clib.ptr(m),
                                 _clib.ptr(mu), _clib.ptr(e))
    assert rc == 0
    return m, mu, e


class Evaluation:
    """Everything one evaluation at Z produces."""

    def __init__(self, Z, C, m, mu, e):
        self.Z, self.cells, self.m, self.mu, self.e = Z, C, m, mu, e
        mz = np.einsum("ij,ij->i", mu, Z)
        self.F = float(np.sum(e))
        self.g = 2.0 * mz[:, None] * Z - 2.0 * mu
        self.h = 1.0 / (2.0 * mz)
        self.lloyd = mu / np.linalg.norm(mu, axis=1)[:, None] - Z
        self.step_inf = float(np.max(np.abs(self.lloyd)))
        self.centroid = mu / m[:, None]


def evaluate(Z, density, levels=2, rule=7):
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    C = _cells(Z)
    m, mu, e = cell_integrals(C, density, levels, rule)
    return Evaluation(Z, C, m, mu, e)


def two_loop(g, h, hist):
    """P-LBFGS direction q = -H g (section 2.2.2 two-loop recursion with the
    initial inverse Hessian replaced by diag(h), section 3.1).

    hist: list of (s, y, r) oldest first, r = 1/(y.s)."""
    q = -np.array(g, dtype=np.float64)
    a = [0.0] * len(hist)
    for j in range(len(hist) - 1, -1, -1):       # backward: newest to oldest
        s, y, r = hist[j]
        a[j] = r * dot(s, q)
        q = q - a[j] * y
    q = h[:, None] * q                            # q <- H0 q, H0 = diag(h)
    for j in range(len(hist)):                    # forward: oldest to newest
        s, y, r = hist[j]
        b = r * dot(y, q)
        q = q + (a[j] - b) * s
    return q


class LineSearchError(RuntimeError):
    """No sufficient decrease along the direction, and the Lloyd step did
    not lower F either (beyond the evaluation's rounding)."""


# relative rise of F the Lloyd fallback may show and still count as a
# decrease (the evaluation's rounding in FP64)
LLOYD_ALLOWANCE = 1e-13


class Solver:
    """Lloyd-preconditioned LBFGS (state machine written out plainly).

    method: "plbfgs" (section 3.1, initial inverse Hessian diag(h)),
    "lloyd" (section 2.2.1: every generator moves to its constrained mass
    centroid mu/|mu|), "lbfgs" (section 2.2.2: initial inverse Hessian
    gamma_n I with gamma_n = y.s / y.y of the newest stored pair, the
    identity while none is stored)."""

    def __init__(self, Z0, density, m_hist=7, levels=2, ls_max_evals=10, c1=1e-4,
                 curv_eps=1e-10, method="plbfgs", rule=7):
        assert method in ("plbfgs", "lloyd", "lbfgs")
        self.method = method
        self.rule = rule
        self.density, self.M, self.levels = density, int(m_hist), levels
        self.ls_max_evals, self.c1, self.curv_eps = ls_max_evals, c1, curv_eps
        self.cur = evaluate(normalize_rows(np.asarray(Z0, dtype=np.float64)), density, levels, rule)
        self.hist = []
        self.iter = 0
        self.n_evals = 1
        self.last_alpha = 0.0
        self.n_lloyd_fallback = 0
        self.history_F = [self.cur.F]

    @property
    def Z(self):
        return self.cur.Z

    def initial_diag(self):
        if self.method != "lbfgs":
            return self.cur.h
        if not self.hist:
            return np.ones(len(self.cur.h))
        s, y, r = self.hist[-1]
        return np.full(len(self.cur.h), dot(y, s) / dot(y, y))

    def direction(self):
        return two_loop(self.cur.g, self.initial_diag(), self.hist)

    def _line_search(self, q, gq):
        alpha = 1.0
        for _ in range(self.ls_max_evals):
            Zt = normalize_rows(self.cur.Z + alpha * q)
            ev = evaluate(Zt, self.density, self.levels, self.rule)
            self.n_evals += 1
            if ev.F <= self.cur.F + self.c1 * alpha * gq:
                return alpha, ev
            alpha *= 0.5
        return None, None

    def step(self):
        cur = self.cur
        if self.method == "lloyd":
            ev = evaluate(normalize_rows(cur.mu), self.density, self.levels, self.rule)
            self.n_evals += 1
            self.cur = ev
            self.iter += 1
            self.last_alpha = 1.0
            self.history_F.append(ev.F)
            return ev
        q = self.direction()
        gq = dot(cur.g, q)
        if gq >= 0.0:                                  # not a descent direction
            self.hist = []
            q = -self.initial_diag()[:, None] * cur.g
            gq = dot(cur.g, q)
        alpha, ev = self._line_search(q, gq)
        if ev is None:
            # no sufficient decrease within the evaluation budget: take the
            # Lloyd step (alpha = 1 along -h g), which decreases F without a
            # line search (section 2.2.1), and restart the history
            self.hist = []
            q = -cur.h[:, None] * cur.g
            ev = evaluate(normalize_rows(cur.Z + q), self.density, self.levels, self.rule)
            self.n_evals += 1
            # section 2.2.1: Lloyd's step lowers the exact energy; a rise of
            # the evaluated energy (coarse quadrature of very large cells)
            # ends the iteration, the generators staying where they are
            if not ev.F <= cur.F + LLOYD_ALLOWANCE * abs(cur.F):
                raise LineSearchError("Lloyd step raised F from %.17g to %.17g" % (cur.F, ev.F))
            alpha = 1.0
            self.n_lloyd_fallback += 1
        s = ev.Z - cur.Z
        y = ev.g - cur.g
        ys = dot(y, s)
        if ys > self.curv_eps * np.sqrt(dot(y, y) * dot(s, s)):
            self.hist.append((s, y, 1.0 / ys))
            if len(self.hist) > self.M:
                self.hist.pop(0)
        self.cur = ev
        self.iter += 1
        self.last_alpha = alpha
        self.history_F.append(ev.F)
        return ev

    def solve(self, max_iter, tol):
        while self.cur.step_inf >= tol and self.iter < max_iter:
            self.step()
        return self.cur

    def solve_rel(self, max_iter, step_tol=0.0, grad_rel_tol=0.0, f_rel_tol=0.0):
        """Stopping tests of the method comparison (section 4.1): point
        movement (the Lloyd step) below step_tol; for the quasi-Newton
        methods also |g|/F <= grad_rel_tol or |dF|/F < f_rel_tol.  Returns
        True when a test (not the iteration cap) stopped it."""
        qn = self.method != "lloyd"
        F_prev = None
        while True:
            c = self.cur
            if step_tol > 0 and c.step_inf < step_tol:
                return True
            if qn and grad_rel_tol > 0 and np.sqrt(dot(c.g, c.g)) / c.F <= grad_rel_tol:
                return True
            if qn and f_rel_tol > 0 and F_prev is not None and abs(F_prev - c.F) / F_prev < f_rel_tol:
                return True
            if self.iter >= max_iter:
                return False
            F_prev = c.F
            self.step()


def local_cell(Z, i, density, radius, levels=2):
    """Cell i and its integrals from the generators within chord `radius` of
    z_i only (for sampled checks at sizes where the global hull is slow).

    The cell of z_i is decided by the generators closer than 2R_i (R_i its
    circumradius): a generator farther than that cannot be nearer than z_i
    to any point of the cell.  Raises if 2R_i >= radius.  Returns
    (neighbour ids, vertices (deg,3) counter-clockwise, m, mu, e)."""
    from .voronoi import cells as _c
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    d = np.linalg.norm(Z - Z[i], axis=1)
    sub = np.where(d < radius)[0]
    C = _c(Z[sub])
    k = int(np.where(sub == i)[0][0])
    verts = C.verts[C.ptr[k]:C.ptr[k + 1]]
    R = np.max(np.linalg.norm(verts - Z[i], axis=1))
    if not 2 * R < radius:
        raise ValueError("radius too small for cell %d" % i)
    # neighbour on the edge from vertex t to t+1: the facet pair's common index
    fac = C.fac[C.ptr[k]:C.ptr[k + 1]]
    nb = []
    for t in range(len(fac)):
        common = (set(C.F[fac[t]]) & set(C.F[fac[(t + 1) % len(fac)]])) - {k}
        nb.append(int(sub[common.pop()]))
    one = type(C).__new__(type(C))
    one.Z = Z[i:i + 1]
    one.ptr = np.array([0, len(verts)], dtype=np.int64)
    one.verts = np.ascontiguousarray(verts)
    m, mu, e = cell_integrals(one, density, levels)
    return nb, verts, m[0], mu[0], e[0]
