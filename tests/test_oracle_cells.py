"""Pins for the oracle's Voronoi cells and cell integrals (not the GPU path).

  * brute-force definition at tiny n: every Voronoi vertex of cell i is a
    point equidistant from z_i and two others with no generator closer
    (section 2.1, eq. viInS), enumerated over all triples;
  * nearest-generator sampling: random points fall in the oracle cell of
    their brute-force nearest generator, and sampled areas agree within 4 sigma;
  * Euler counts of a triangulated sphere: 2n-4 triangles, 3n-6 edges;
  * empty circumcircle (section 3.2.1): the nearest generators of every
    Voronoi vertex (kd-tree, independent of the hull) are its three own;
  * Platonic configurations at rho = 1: closed-form cell area, moment and
    energy, and the exact Lloyd fixed point;
  * total area 4 pi, total mass and total moment against 1-D quadrature of
    the tanh density (scipy quad), and the X3 closed-form total mass.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.spatial import cKDTree

import oracle
import paper_1709_06924_amd.inputs as I


def vos_area(a, b, c):
    num = np.dot(a, np.cross(b, c))
    den = 1 + np.dot(a, b) + np.dot(b, c) + np.dot(c, a)
    return 2 * math.atan2(num, den)


def stokes_moment(verts):
    mu = np.zeros(3)
    k = len(verts)
    for t in range(k):
        p, q = verts[t], verts[(t + 1) % k]
        cr = np.cross(p, q)
        theta = math.atan2(np.linalg.norm(cr), np.dot(p, q))
        mu += 0.5 * theta * cr / np.linalg.norm(cr)
    return mu


def hemisphere_points(n, seed):
    """n points all inside one open hemisphere (origin outside the hull)."""
    Z = I.uniform_sphere(n, seed)
    Z[:, 2] = np.abs(Z[:, 2]) + 0.05
    return Z / np.linalg.norm(Z, axis=1)[:, None]


@pytest.mark.parametrize("n,seed,hemi", [(5, 0, False), (9, 1, False), (17, 2, False),
                                         (31, 3, False), (5, 1, False), (6, 4, True),
                                         (10, 5, True)])
def test_cells_match_bruteforce_definition(n, seed, hemi):
    Z = hemisphere_points(n, seed) if hemi else I.uniform_sphere(n, seed)
    C = oracle.cells(Z)
    for i in range(n):
        found = []
        for j in range(n):
            for l in range(j + 1, n):
                if i in (j, l):
                    continue
                w = np.cross(Z[j] - Z[i], Z[l] - Z[i])
                w /= np.linalg.norm(w)
                for v in (w, -w):
                    d = np.linalg.norm(Z - v, axis=1)
                    if np.all(d >= d[i] - 1e-12):
                        found.append(v)
        verts = C.verts[C.ptr[i]:C.ptr[i + 1]]
        assert len(found) == len(verts)
        for v in found:
            assert np.min(np.linalg.norm(verts - v, axis=1)) < 1e-12


def point_in_cell(C, i, x):
    verts = C.verts[C.ptr[i]:C.ptr[i + 1]]
    k = len(verts)
    return all(np.dot(x, np.cross(verts[t], verts[(t + 1) % k])) >= -1e-14 for t in range(k))


def test_cells_match_nearest_generator_sampling():
    n = 60
    Z = I.uniform_sphere(n, 11)
    C = oracle.cells(Z)
    ev = oracle.evaluate(Z, {"kind": "const"})
    X = I.uniform_sphere(200000, 12)
    near = np.argmax(X @ Z.T, axis=1)
    for x, i in zip(X[:2000], near[:2000]):
        assert point_in_cell(C, i, x)
    counts = np.bincount(near, minlength=n)
    p = ev.m / (4 * np.pi)
    sigma = np.sqrt(len(X) * p * (1 - p))
    assert np.all(np.abs(counts - len(X) * p) < 4.5 * sigma)


@pytest.mark.parametrize("n", [4, 7, 100, 2562, 40962])
def test_euler_counts(n):
    Z = I.uniform_sphere(n, n)
    C = oracle.cells(Z)
    assert len(C.F) == 2 * n - 4
    i, j, fl = oracle.neighbour_sets(Z, C)
    assert len(i) == 3 * n - 6
    assert C.deg().sum() == 6 * n - 12
    assert not fl.any()


def test_empty_circumcircle_kdtree():
    n = 20000
    Z = I.uniform_sphere(n, 5)
    C = oracle.cells(Z)
    tree = cKDTree(Z)
    d, idx = tree.query(C.V, k=4)
    own = np.sort(C.F, axis=1)
    assert np.array_equal(np.sort(idx[:, :3], axis=1), own)
    r = np.linalg.norm(C.V - Z[C.F[:, 0]], axis=1)
    assert np.allclose(d[:, 0], r, rtol=0, atol=1e-12)
    assert np.all(d[:, 3] > r)


def platonic_cells(P):
    """Cells of a Platonic configuration built without the hull: faces are
    the triples of mutually nearest vertices; the cell of a vertex is the
    polygon of the normalised centroids of its faces, ordered by azimuth."""
    n = len(P)
    D = np.linalg.norm(P[:, None] - P[None], axis=2)
    edge = np.min(D[D > 1e-9])
    faces = [(a, b, c) for a in range(n) for b in range(a + 1, n) for c in range(b + 1, n)
             if max(D[a, b], D[b, c], D[a, c]) < edge * (1 + 1e-9)]
    cells = []
    for i in range(n):
        cen = [P[list(f)].sum(0) for f in faces if i in f]
        cen = [c / np.linalg.norm(c) for c in cen]
        e1 = np.cross(P[i], [0.3, 0.5, 0.8])
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(P[i], e1)
        cen.sort(key=lambda v: math.atan2(np.dot(v, e2), np.dot(v, e1)))
        cells.append(cen)
    return cells


@pytest.mark.parametrize("name", ["tetra", "octa", "icosa"])
def test_platonic_closed_forms_and_fixed_point(name):
    P = I.platonic(name)
    cells = platonic_cells(P)
    F_closed = 0.0
    for i, verts in enumerate(cells):
        area = sum(vos_area(P[i], verts[k], verts[(k + 1) % len(verts)]) for k in range(len(verts)))
        mu = stokes_moment(verts)
        F_closed += 2 * area - 2 * np.dot(P[i], mu)
    F = {}
    for L in (2, 4):
        ev = oracle.evaluate(P, {"kind": "const"}, levels=L)
        # cells of these solids span up to 109 degrees: the 2-level rule is
        # good to ~1e-5 there and each further level gains ~2^6
        assert np.isclose(ev.m.sum(), 4 * np.pi, rtol=1e-5 if L == 2 else 1e-8)
        assert ev.step_inf < 1e-14          # exact Lloyd fixed point by symmetry
        F[L] = ev.F
    assert abs(F[2] - F_closed) / F_closed < 1e-5
    assert abs(F[4] - F_closed) / F_closed < 1e-8
    assert abs(F[4] - F_closed) < abs(F[2] - F_closed) / 30


def test_cube_is_flagged_degenerate():
    P = I.platonic("cube")
    C = oracle.cells(P)
    i, j, fl = oracle.neighbour_sets(P, C)
    assert fl.sum() == 6       # one diagonal of each square face
    ev = oracle.evaluate(P, {"kind": "const"})
    assert abs(ev.m.sum() - 4 * np.pi) < 1e-4
    assert ev.step_inf < 1e-14


def test_total_area_and_moment_rho1():
    Z = I.uniform_sphere(2562, 1)
    ev = oracle.evaluate(Z, {"kind": "const"})
    assert abs(ev.m.sum() - 4 * np.pi) < 1e-11
    assert np.linalg.norm(ev.mu.sum(0)) < 1e-12
    # per-cell closed forms on the oracle's own cells
    C = ev.cells
    worst = 0.0
    for i in range(0, 2562, 37):
        verts = C.verts[C.ptr[i]:C.ptr[i + 1]]
        area = sum(vos_area(Z[i], verts[k], verts[(k + 1) % len(verts)]) for k in range(len(verts)))
        worst = max(worst, abs(ev.m[i] - area) / area)
        mu = stokes_moment(list(verts))
        assert np.linalg.norm(ev.mu[i] - mu) < 1e-11 * area
    assert worst < 1e-11


def tanh_totals(d):
    """Total mass and first moment of the tanh family by linearity: the floor
    gamma contributes 4 pi gamma and no moment; bump k is axially symmetric
    about its own centre x_c,k, so with theta the angle from x_c,k its mass
    is 2 pi amp_k int sigma_k(theta) sin(theta) and its moment is x_c,k times
    2 pi amp_k int sigma_k(theta) cos(theta) sin(theta)  (1-D scipy quad)."""
    g = d["gamma"]
    M = 4 * math.pi * g
    MU = np.zeros(3)
    for k in range(len(d["xc"])):
        xc = np.array(d["xc"][k])
        a, b, amp = d["alpha"][k], d["beta"][k], d["amp"][k]

        def bump(theta):
            dist = theta if d.get("geodesic") else 2 * math.sin(theta / 2)
            return amp * 0.5 * (math.tanh((b - dist) / a) + 1)

        M += 2 * math.pi * integrate.quad(lambda t: bump(t) * math.sin(t), 0, math.pi, epsabs=0,
                                          epsrel=1e-13, limit=400)[0]
        m1 = 2 * math.pi * integrate.quad(lambda t: bump(t) * math.cos(t) * math.sin(t), 0,
                                          math.pi, epsabs=0, epsrel=1e-13, limit=400)[0]
        MU += m1 * xc
    return M, MU


@pytest.mark.parametrize("geodesic", [False, True])
def test_total_mass_tanh(geodesic):
    d = I.density_tanh(I.latlon(30, 90), math.pi / 6, 0.2, 8, geodesic=geodesic)
    Z = I.uniform_sphere(10242, 2)
    ev = oracle.evaluate(Z, d)
    M, MU = tanh_totals(d)
    assert abs(ev.m.sum() - M) / M < 1e-9
    assert np.linalg.norm(ev.mu.sum(0) - MU) / np.linalg.norm(MU) < 1e-8


def test_total_mass_two_centre():
    """The two-bump density (sum over bumps with their own heights) against
    the per-bump 1-D integrals; dropping the second bump moves the mass by
    ~5% and the moment's direction by tens of degrees."""
    d = I.density_two_centre()
    Z = I.uniform_sphere(10242, 5)
    ev = oracle.evaluate(Z, d)
    M, MU = tanh_totals(d)
    assert abs(ev.m.sum() - M) / M < 1e-9
    assert np.linalg.norm(ev.mu.sum(0) - MU) / np.linalg.norm(MU) < 1e-8
    M1, _ = tanh_totals(dict(d, xc=d["xc"][:1], beta=d["beta"][:1], alpha=d["alpha"][:1],
                             amp=d["amp"][:1]))
    assert (M - M1) / M > 0.01


def x16_totals(d):
    """Mass and first moment of the X16 density by 2-D scipy quadrature over
    latitude and longitude (area element cos(lat)), the distance in spherical
    trigonometry (see test_oracle_rule._x16_closed_form), the ranges split
    at the centre's parallel and meridian where the distance has kinks."""
    xc = np.array(d["xc"][0])
    lat_c, lon_c = math.asin(xc[2]), math.atan2(xc[1], xc[0])

    def rho(la, lo):
        d_lon = 2.0 * math.asin(math.cos(la) * abs(math.sin((lo - lon_c) / 2.0)))
        dist = math.hypot(d_lon / d["w_lon"], (la - lat_c) / d["w_lat"])
        return d["gamma"] + d["amp"][0] * 0.5 * (math.tanh((d["beta"][0] - dist) / d["alpha"][0]) + 1)

    def integral(f):
        tot = 0.0
        for lo0, lo1 in ((lon_c - math.pi, lon_c), (lon_c, lon_c + math.pi)):
            for la0, la1 in ((-math.pi / 2, lat_c), (lat_c, math.pi / 2)):
                tot += integrate.dblquad(lambda la, lo: f(la, lo) * math.cos(la), lo0, lo1,
                                         la0, la1, epsabs=1e-13, epsrel=1e-12)[0]
        return tot

    M = integral(rho)
    MU = np.array([integral(lambda la, lo: rho(la, lo) * math.cos(la) * math.cos(lo)),
                   integral(lambda la, lo: rho(la, lo) * math.cos(la) * math.sin(lo)),
                   integral(lambda la, lo: rho(la, lo) * math.sin(la))])
    return M, MU


def test_total_mass_x16():
    """X16 totals against 2-D quadrature of its closed form.  The density has
    kinks along the centre's parallel and meridian (|lat - lat_c| and the arc
    of the parallel), which the cells' degree-5 rule resolves only to about
    1.3e-9 relative at n = 10,242 (measured), so the tolerance is 1e-8; a
    swap of the two widths moves the mass by 1.5e-3."""
    d = I.density_x16()
    Z = I.uniform_sphere(10242, 6)
    ev = oracle.evaluate(Z, d)
    M, MU = x16_totals(d)
    assert abs(ev.m.sum() - M) / M < 1e-8, (ev.m.sum(), M)
    assert np.linalg.norm(ev.mu.sum(0) - MU) / np.linalg.norm(MU) < 1e-8


def test_total_mass_x3():
    Z = I.uniform_sphere(2562, 3)
    ev = oracle.evaluate(Z, I.density_x3())
    g = 3.0 ** -4
    exact = (1 - g) * 4 * math.pi / 5 + 4 * math.pi * g
    assert abs(ev.m.sum() - exact) / exact < 1e-10


def test_local_cell_equals_global():
    """The neighbourhood-only cell (used for sampled checks at full size)
    equals the global one."""
    n = 5000
    Z = I.uniform_sphere(n, 21)
    d = I.density_tanh(I.latlon(30, 90), math.pi / 6, 0.2, 8)
    ev = oracle.evaluate(Z, d)
    h = math.sqrt(4 * math.pi / n)
    for i in range(0, n, 499):
        nb, verts, m, mu, e = oracle.local_cell(Z, i, d, 6 * h)
        assert abs(m - ev.m[i]) <= 1e-14 * ev.m[i]
        assert np.max(np.abs(mu - ev.mu[i])) <= 1e-15
        assert abs(e - ev.e[i]) <= 1e-14 * ev.e[i]
        assert len(nb) == ev.cells.deg()[i]


def test_one_ulp_generator_change_conditioning():
    """The limit of per-cell parity: renormalising the rows once more (a
    change of at most an ulp or two in ~a third of the generators) moves the
    masses of a few ill-conditioned cells (near-cocircular generators, whose
    Voronoi vertices move by ~ulp / angle) by a few 1e-12 relative, while the
    median cell moves by ~1e-13.  So the GPU and the oracle must evaluate the
    very same generators (the library's renormalised rows) before their
    cells are compared at 1e-12."""
    n = 2562
    Z0 = I.uniform_sphere(n, 1)
    d = I.density_tanh(I.latlon(30, 90), math.pi / 6, 0.2, 8)
    Z1 = oracle.normalize_rows(Z0)
    changed = np.any(Z1 != Z0, axis=1)
    assert 0.1 * n < changed.sum() < 0.6 * n
    assert np.max(np.abs(Z1 - Z0)) <= 2 * np.finfo(float).eps
    a, b = oracle.evaluate(Z0, d), oracle.evaluate(Z1, d)
    rel = np.abs(a.m - b.m) / a.m
    assert 1e-12 < rel.max() < 2e-11, rel.max()
    assert np.median(rel) < 2e-13
    assert abs(a.F - b.F) < 1e-14 * a.F
