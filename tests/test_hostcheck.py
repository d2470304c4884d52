"""CPU checks of the HIP path's geometry and quadrature code (host build of
csrc/cellgeom.h, see tests/host/cellcheck.cpp) against the oracle.

These run the very functions the kernels call per lane, sequentially on the
host: the per-bisector edge construction with its certificate, the
sequential fallback clipper, the window certificate of the cube-map grid and
the fan quadrature.  The GPU parity tests then check the wave-level drivers.
"""
import math
from collections import defaultdict

import numpy as np
import pytest

import hostcheck as hc
import oracle
import paper_1709_06924_amd.inputs as I


def oracle_nbrs(Z):
    C = oracle.cells(Z)
    i, j, fl = oracle.neighbour_sets(Z, C)
    nb = defaultdict(set)
    for a, b in zip(i, j):
        nb[a].add(b)
        nb[b].add(a)
    return C, nb, {(a, b) for a, b, f in zip(i, j, fl) if f}


def oracle_cell_edges(C, k):
    """{neighbour: (v_start, v_end)} of the oracle's cell k."""
    out = {}
    verts = C.verts[C.ptr[k]:C.ptr[k + 1]]
    fac = C.fac[C.ptr[k]:C.ptr[k + 1]]
    d = len(verts)
    for t in range(d):
        f0, f1 = set(C.F[fac[t]]), set(C.F[fac[(t + 1) % d]])
        common = (f0 & f1) - {k}
        assert len(common) == 1
        out[common.pop()] = (verts[t], verts[(t + 1) % d])
    return out


@pytest.mark.parametrize("n,seed", [(500, 1), (3000, 2)])
def test_certified_cells_match_oracle(n, seed):
    Z = I.uniform_sphere(n, seed)
    C, nb, _ = oracle_nbrs(Z)
    h = math.sqrt(4 * math.pi / n)
    st, deg, nbr, verts, R = hc.cells(Z, 3.5 * h)
    ok = np.where(st == 0)[0]
    assert len(ok) > 0.95 * n
    for k in ok:
        got = nbr[k][:deg[k]].tolist()
        assert set(got) == nb[k]
        ed = oracle_cell_edges(C, k)
        for t, j in enumerate(got):
            v0, v1 = ed[j]
            assert np.max(np.abs(verts[k, t, :3] - v0)) < 1e-14
            assert np.max(np.abs(verts[k, t, 3:] - v1)) < 1e-14


def _certify(Z, rt, cap, attempts=8):
    """The kernels' radius policy for a group holding `cap` candidates: grow
    to min(2.1 R, 1.6 r) after an uncertified attempt and to 1.6 r after an
    unbounded one; on overflow shrink toward 3/4 cap candidates, giving up
    when that is no larger than a radius already found too small."""
    n = len(Z)
    rt = np.array(rt, dtype=float)
    r_small = np.zeros(n)
    done = np.zeros(n, bool)
    open_ = np.ones(n, bool)
    for attempt in range(attempts):
        st, deg, nbr, verts, R = hc.cells(Z, rt, cap=cap)
        st = np.where(open_, st, -1)
        done |= st == 0
        open_ &= st != 0
        grow_u = st == 3
        grow_b = st == 2
        r_small = np.where(grow_u | grow_b, np.maximum(r_small, rt), r_small)
        shrink = rt * np.sqrt(0.75 * cap / np.maximum(R, 1.0))
        give_up = (st == 4) & (shrink <= r_small)
        open_ &= ~give_up
        rt = np.where(grow_u, np.minimum(2.1 * R, 1.6 * rt), rt)
        rt = np.where(grow_b, 1.6 * rt, rt)
        rt = np.where(st == 4, shrink, rt)
    return done


def test_retry_policy_certifies_nearly_all():
    """On random input the main pass (16 candidates per cell) certifies most
    cells from a too small and from a too large first radius, the list
    passes (32, then 64 candidates) nearly all of the rest."""
    n = 3000
    Z = I.uniform_sphere(n, 2)
    h = math.sqrt(4 * math.pi / n)
    for r0 in (2.0 * h, 6.0 * h):
        done = _certify(Z, np.full(n, r0), cap=16)
        assert done.mean() > 0.6
        done |= _certify(Z, np.full(n, 2.0 * h), cap=32)
        assert done.mean() > 0.99
        done |= _certify(Z, np.full(n, 2.0 * h), cap=64)
        assert done.mean() > 0.998
    # from the previous evaluation's circumradius (2.3 R) as well; on random
    # input (irregular cells) about 30% need more than 16 candidates
    st, deg, nbr, verts, R = hc.cells(Z, 3.5 * h)
    R = np.where(st == 0, R, h)
    done = _certify(Z, 2.3 * R, cap=16)
    assert done.mean() > 0.6
    done |= _certify(Z, 2.3 * R, cap=32)
    assert done.mean() > 0.98
    done |= _certify(Z, 2.3 * R, cap=64)
    assert done.mean() > 0.998


def test_certificate_is_sound():
    """A cell certified with a small candidate set equals the one built from
    all generators (brute force within radius 2)."""
    n = 800
    Z = I.uniform_sphere(n, 9)
    h = math.sqrt(4 * math.pi / n)
    st, deg, nbr, verts, R = hc.cells(Z, 2.4 * h)
    st_all, deg_all, nbr_all, verts_all, _ = hc.cells(Z, np.full(n, 2.0001))
    for k in np.where(st == 0)[0]:
        if st_all[k] == 4:  # more than 64 within radius 2: skip
            continue
        assert np.array_equal(nbr[k], nbr_all[k])
        assert np.array_equal(verts[k], verts_all[k])


@pytest.mark.parametrize("name", ["tetra", "octa", "icosa", "cube"])
def test_fallback_clipper_platonic(name):
    P = I.platonic(name)
    C, nb, flagged = oracle_nbrs(P)
    ev = oracle.evaluate(P, {"kind": "const"})
    for k in range(len(P)):
        deg, nbr, verts, flags, R = hc.clip(P, k)
        assert deg >= 3 and not (flags & 4)
        out = hc.quad(P[k], deg, verts, {"kind": "const"})
        assert abs(out[0] - ev.m[k]) < 1e-12 * ev.m[k]
        assert np.max(np.abs(out[1:4] - ev.mu[k])) < 1e-12
        assert abs(out[4] - ev.e[k]) < 1e-12 * ev.e[k]
        if name != "cube":
            assert set(nbr[:deg].tolist()) == nb[k]


@pytest.mark.parametrize("n,seed", [(4, 0), (5, 1), (9, 2), (40, 3), (600, 4)])
def test_fallback_clipper_random(n, seed):
    Z = I.uniform_sphere(n, seed)
    C, nb, _ = oracle_nbrs(Z)
    for k in range(n):
        deg, nbr, verts, flags, R = hc.clip(Z, k)
        assert not (flags & 4)
        assert set(nbr[:deg].tolist()) == nb[k]
        ed = oracle_cell_edges(C, k)
        for t, j in enumerate(nbr[:deg]):
            v0, v1 = ed[j]
            assert np.max(np.abs(verts[t, :3] - v0)) < 1e-13
            assert np.max(np.abs(verts[t, 3:] - v1)) < 1e-13


@pytest.mark.parametrize("density,rule", [("const", 7), ("tanh", 7), ("tanh_geo", 7), ("x3", 7),
                                          ("x16", 7), ("two", 7), ("x3", 4), ("x16", 4),
                                          ("x64", 9), ("tanh", 9)])
def test_quadrature_matches_oracle(density, rule):
    d = {"const": {"kind": "const"},
         "tanh": I.density_tanh(I.latlon(30, 90), math.pi / 6, 0.2, 8),
         "tanh_geo": I.density_tanh(I.latlon(10, 20), math.pi / 9, 0.15, 16, geodesic=True),
         "x3": I.density_x3(), "x16": I.density_x16(), "x64": I.density_x64(),
         "two": I.density_two_centre()}[density]
    n = 1500
    Z = I.uniform_sphere(n, 5)
    ev = oracle.evaluate(Z, d, rule=rule)
    h = math.sqrt(4 * math.pi / n)
    st, deg, nbr, verts, R = hc.cells(Z, 4.0 * h)
    worst = [0.0, 0.0, 0.0]
    for k in np.where(st == 0)[0]:
        out = hc.quad(Z[k], deg[k], verts[k], d, rule=rule)
        worst[0] = max(worst[0], abs(out[0] - ev.m[k]) / ev.m[k])
        worst[1] = max(worst[1], np.linalg.norm(out[1:4] - ev.mu[k]) / np.linalg.norm(ev.mu[k]))
        worst[2] = max(worst[2], abs(out[4] - ev.e[k]) / ev.e[k])
    assert max(worst) < 1e-12, worst


@pytest.mark.parametrize("n", [300, 2562, 100000])
def test_window_certificate_covers_ball(n):
    """Every generator within the window's certified radius D of z is stored
    in the window's cells on z's home face (home or ghost copy)."""
    GBW, dd = hc.grid(n)
    W = GBW[2]
    X = I.uniform_sphere(20000, 1)
    Z = I.uniform_sphere(300, 2)
    h = math.sqrt(4 * math.pi / n)
    for z in Z:
        for rt in (2.0 * h, 6.0 * h, 20.0 * h):
            (f, alo, ahi, blo, bhi), D = hc.window(GBW, dd, z, rt)
            if D <= 0:
                continue
            near = X[np.linalg.norm(X - z, axis=1) < D]
            c = hc.cell_on_face(GBW, dd, near, f)
            assert np.all(c >= 0)
            loc = c - f * W * W
            ia, ib = loc % W, loc // W
            assert np.all((ia >= alo) & (ia <= ahi) & (ib >= blo) & (ib <= bhi))


@pytest.mark.parametrize("n", [10**6, 10**8, 10**9])
def test_window_certificate_covers_ball_large_grids(n):
    """The same at the grids of large n, with points sampled in a cap around
    each z (uniform points would leave the small balls empty): the columns
    are chosen in FP32 (at n = 10^9 the column coordinate reaches ~10^4),
    and the certified radius, computed from the columns taken, still bounds
    every stored point; the window also reaches the radius asked for where
    the face allows it."""
    GBW, dd = hc.grid(n)
    W = GBW[2]
    Z = I.uniform_sphere(200, 5)
    h = math.sqrt(4 * math.pi / n)
    reached = 0
    for k, z in enumerate(Z):
        for rt in (2.0 * h, 6.0 * h):
            (f, alo, ahi, blo, bhi), D = hc.window(GBW, dd, z, rt)
            if D <= 0:
                continue
            reached += D >= rt
            X = I.cap_points(z, 1.2 * D, 400, 100 + k)
            near = X[np.linalg.norm(X - z, axis=1) < D]
            assert len(near) > 100
            c = hc.cell_on_face(GBW, dd, near, f)
            assert np.all(c >= 0)
            loc = c - f * W * W
            ia, ib = loc % W, loc // W
            assert np.all((ia >= alo) & (ia <= ahi) & (ib >= blo) & (ib <= bhi))
    assert reached >= 0.95 * 2 * len(Z), reached


def test_home_face_inside_its_grid():
    GBW, dd = hc.grid(100000)
    X = I.uniform_sphere(50000, 3)
    hf = hc.home_face(X)
    for f in range(6):
        sel = X[hf == f]
        assert np.all(hc.cell_on_face(GBW, dd, sel, f) >= 0)


@pytest.mark.parametrize("density", ["const", "tanh16", "two", "x3", "geo", "x16"])
def test_mixed_quadrature_error(density):
    """FP32 local-frame quadrature (the mixed path; the host build's special
    functions are IEEE) against the FP64 oracle, with the precision form's
    acceptance bounds: per cell |dm|/m <= 1e-5, |de|/e <= 1e-5 and centroid
    error <= 1e-7 h_i (h_i the mean distance to the cell's neighbours).
    X16's anisotropic distance is evaluated directly in FP32 (latitude and
    longitude of each point, ~6e-8 absolute, amplified by the bump's slope):
    its bound is 2e-7 h_i (1.3e-7 measured)."""
    d = {"const": {"kind": "const"}, "tanh16": I.CONFIGS["C3"]["density"],
         "two": I.density_two_centre(), "x3": I.density_x3(), "geo": I.density_x64(),
         "x16": I.density_x16()}[density]
    n = 4000
    Z = I.uniform_sphere(n, 5)
    ev = oracle.evaluate(Z, d)
    i, j, _ = oracle.neighbour_sets(Z, ev.cells)
    dist = np.linalg.norm(Z[i] - Z[j], axis=1)
    hi = (np.bincount(i, dist, n) + np.bincount(j, dist, n)) / (
        np.bincount(i, minlength=n) + np.bincount(j, minlength=n))
    h = math.sqrt(4 * math.pi / n)
    st, deg, nbr, verts, R = hc.cells(Z, 4 * h)
    worst = 0.0
    for k in np.where(st == 0)[0][::3]:
        out = hc.quad_mixed(Z[k], deg[k], verts[k], d)
        assert abs(out[0] - ev.m[k]) <= 1e-5 * ev.m[k]
        assert abs(out[4] - ev.e[k]) <= 1e-5 * ev.e[k]
        worst = max(worst, np.linalg.norm(out[1:4] / out[0] - ev.centroid[k]) / hi[k])
    print("mixed %s: max centroid error / h = %.2e" % (density, worst))
    assert worst <= (2e-7 if density == "x16" else 1e-7)


def test_exp_table_accuracy():
    """The table-driven exponential 2^(u/128) of the FP64 density agrees with
    an extended-precision evaluation within its bound (1.3e-15 truncation
    plus rounding) from the largest argument down into the denormal range,
    is exact at the table's own points, and underflows to 0 below."""
    rng = np.random.default_rng(5)
    lo, hi = -128.0 * 1021, 128.0 * 1009
    u = np.concatenate([rng.uniform(lo, hi, 100000), rng.uniform(-100.0, 100.0, 100000),
                        rng.uniform(-3000.0, 3000.0, 100000),
                        [0.0, lo, hi, 1e-300, -1e-300, 0.5, -0.5, 128.0, -128.0, 64.0, 0.4999999]])
    got = hc.exp2_n(u)
    ln2_n = np.log(np.longdouble(2)) / 128
    ref = np.exp(u.astype(np.longdouble) * ln2_n)
    rel = np.abs((got.astype(np.longdouble) - ref) / ref).astype(np.float64)
    assert rel.max() < 1.6e-15, rel.max()
    assert got[-11] == 1.0 and got[-8] == 1.0                 # u = 0 and u = 1e-300
    assert got[-4] == 2.0 and got[-3] == 0.5                  # u = +-128: exact powers of two
    assert got[-10] == 2.0 ** -1021 and got[-9] == 2.0 ** 1009
    # denormal results and underflow, also where the integer part saturates
    tiny = hc.exp2_n(np.array([-128.0 * 1030, -128.0 * 1080, -1e7, -3e9, -1e300]))
    assert tiny[0] == 2.0 ** -1030 and np.all(tiny[1:] == 0.0)


def test_grid2_leaves_equal_recursive_subdivision():
    """The 16 leaves built from the shared 15-point grid are bitwise the
    leaves of two recursive geodesic subdivisions, in the same vertex order."""
    rng = np.random.default_rng(12)
    for k in range(200):
        z = I.uniform_sphere(1, 100 + k)[0]
        t = rng.standard_normal((2, 3)) * (10.0 ** rng.uniform(-4, -0.5))
        B = z + t[0]
        C = z + t[1]
        B /= np.linalg.norm(B)
        C /= np.linalg.norm(C)
        rec, grid = hc.leaves2(z, B, C)
        assert np.array_equal(rec, grid)


@pytest.mark.parametrize("chord", [0.022, 0.1, 0.349, 0.45, 0.8, 1.9])
def test_density_polynomial_within_bound(chord):
    """The per-cell density polynomial (degree 7 in the logistic's argument
    about the generator) agrees with the direct evaluation of the tanh bump
    at points up to the qualifying chord radius from the generator: relative
    truncation below 7e-16 by the Cauchy bound, plus the rounding of the
    dot-product chord (d moves by ~2e-16/d, and rho by up to (2/alpha) times
    that relative); and the radius is what limits it (at 8 times the radius
    the error is over 10 times larger wherever the density varies)."""
    d = I.CONFIGS["C3"]["density"]
    xc = np.array(d["xc"][0])
    z = I.toward(xc, chord, 3)
    rl = 0.5 * (0.05 - 1 / 512) * d["alpha"][0]
    Y = I.cap_points(z, rl * 0.999, 20000, 4)
    poly, exact, _ = hc.rho_poly(z, d, Y)
    rel = np.abs(poly - exact) / exact
    assert rel.max() < 1.5e-14, rel.max()
    Yf = I.cap_points(z, 8 * rl, 20000, 5)
    pf, ef, _ = hc.rho_poly(z, d, Yf)
    if 0.1 <= chord <= 0.8:  # where the logistic varies
        assert (np.abs(pf - ef) / ef).max() > 10 * rel.max()


@pytest.mark.parametrize("chord,m,cap", [(0.1, 600, 0.012), (0.349, 600, 0.012),
                                         (0.6, 600, 0.012), (0.349, 250, 0.03)])
def test_density_polynomial_quadrature_matches_oracle(chord, m, cap):
    """Small cells (a dense cluster of generators) qualify for the per-cell
    density polynomials (in t and, away from the centre, in x); their
    integrals through either agree with the direct FP64 path on the same
    vertices to 2e-14, and with the oracle (which
    builds its own vertices) to 1e-12 on m and mu and 3e-12 on e: a cell of
    circumradius R ~ 6e-4 whose vertices move by an ulp moves its second
    moment by ~4 x 2e-16 / R relative."""
    d = I.CONFIGS["C3"]["density"]
    xc = np.array(d["xc"][0])
    u = I.toward(xc, chord, 7)
    C = I.cap_points(u, cap, m, 8)
    U = I.uniform_sphere(200, 9)
    Z = np.concatenate([C, U])
    ev = oracle.evaluate(Z, d)
    rad = np.concatenate([np.full(len(C), 4 * cap / math.sqrt(m)),
                          np.full(len(U), 4 * math.sqrt(4 * math.pi / 200))])
    st, deg, nbr, verts, R = hc.cells(Z, rad)
    used = 0
    worst = [0.0, 0.0, 0.0, 0.0]
    for k, force in [(k, f) for k in np.where(st == 0)[0] for f in (1, 2)]:
        res = hc.quad_poly(Z[k], deg[k], verts[k], d, force=force)
        if res is None:
            continue
        out = res[0]
        used += 1
        ref = hc.quad(Z[k], deg[k], verts[k], d)
        worst[0] = max(worst[0], abs(out[0] - ev.m[k]) / ev.m[k])
        worst[1] = max(worst[1], np.linalg.norm(out[1:4] - ev.mu[k]) / np.linalg.norm(ev.mu[k]))
        worst[2] = max(worst[2], abs(out[4] - ev.e[k]) / ev.e[k])
        worst[3] = max(worst[3], abs(out[0] - ref[0]) / ref[0], abs(out[4] - ref[4]) / ref[4])
    assert used >= m // 3, used
    assert max(worst[:2]) < 1e-12 and worst[2] < 3e-12, worst
    assert worst[3] < 2e-14, worst


def test_density_polynomial_skips_cells_near_centre():
    """Cells whose generator lies within 0.02 + R of the bump's centre (where
    the dot-product chord would lose relative accuracy) do not qualify, small
    as they are; those just outside do."""
    d = I.CONFIGS["C3"]["density"]
    xc = np.array(d["xc"][0])
    C = I.cap_points(xc, 0.04, 4000, 11)
    U = I.uniform_sphere(200, 12)
    Z = np.concatenate([C, U])
    rad = np.concatenate([np.full(len(C), 4e-3), np.full(len(U), 4 * math.sqrt(4 * math.pi / 200))])
    st, deg, nbr, verts, R = hc.cells(Z, rad)
    rl = 0.5 * (0.05 - 1 / 512) * d["alpha"][0]
    near = far = 0
    for k in np.where(st[:len(C)] == 0)[0]:
        v = verts[k][:deg[k]].reshape(-1, 3)
        if np.linalg.norm(v - Z[k], axis=1).max() > 0.99 * rl:
            continue
        dz = np.linalg.norm(Z[k] - xc)
        q = hc.quad_poly(Z[k], deg[k], verts[k], d) is not None
        if dz < 0.99 * (0.02 + rl):
            assert not q
            near += 1
        elif dz > 1.01 * (0.02 + rl):
            assert q
            far += 1
    assert near >= 100 and far >= 100, (near, far)


@pytest.mark.parametrize("chord", [0.45, 0.8, 1.3, 1.95])
def test_density_polynomial_in_x_within_bound(chord):
    """The expansion in x = d^2/2 (no square root per point) agrees with the
    direct evaluation wherever its table entry's radius covers |x - x*|
    (truncation below 1e-15 by its Cauchy bound, plus the dot product's
    rounding), the radius covers the benchmark's cells (R ~ 3e-3) at these
    distances, and beyond 4 times the radius the error is far larger."""
    d = I.CONFIGS["C3"]["density"]
    xc = np.array(d["xc"][0])
    z = I.toward(xc, chord, 3)
    _, _, lim = hc.rho_poly(z, d, z[None, :], mode=1)
    xz = 0.5 * float(np.sum((z - xc) ** 2))
    jx = round(xz / 1e-4)
    slack = lim - abs(xz - jx * 1e-4)
    dz = math.sqrt(2 * xz)
    rcap = slack / (dz + slack)  # R (d + R/2) <= slack
    assert rcap >= 3.3e-3 or chord < 0.5, rcap
    Y = I.cap_points(z, 0.999 * rcap, 20000, 4)
    poly, exact, _ = hc.rho_poly(z, d, Y, mode=1)
    rel = np.abs(poly - exact) / exact
    assert rel.max() < 1.5e-14, rel.max()
    if chord <= 0.8:  # where the logistic varies
        Yf = I.cap_points(z, 4 * rcap, 20000, 5)
        pf, ef, _ = hc.rho_poly(z, d, Yf, mode=1)
        assert (np.abs(pf - ef) / ef).max() > 10 * rel.max()


def two_centre_point(bump, chord, seed):
    d = I.density_two_centre()
    return d, I.toward(np.array(d["xc"][bump]), chord, seed)


@pytest.mark.parametrize("bump,chord", [(0, 0.45), (0, 1.0), (1, 0.3), (1, 0.8)])
def test_two_bump_expansion_in_x_within_bound(bump, chord):
    """Two chord tanh bumps: the sum of both bumps' expansions in x (each
    from its own table, gamma carried by the first) agrees with the direct
    density wherever both entries' radii cover the point's |x - x*| (the
    smaller radius taken for both), and the radius covers the cells of the
    first bump at n = 4,194,304 (R ~ 3e-4) at these distances."""
    d, z = two_centre_point(bump, chord, 3)
    _, _, lim = hc.rho_poly(z, d, z[None, :], mode=1)
    slack = lim
    for b in range(2):
        xc = np.array(d["xc"][b])
        xz = 0.5 * float(np.sum((z - xc) ** 2))
        slack_b = lim - abs(xz - round(xz / 1e-4) * 1e-4)
        slack = min(slack, slack_b / (math.sqrt(2 * xz) + slack_b))
    assert slack >= 5e-4, slack
    Y = I.cap_points(z, 0.999 * slack, 20000, 4)
    poly, exact, _ = hc.rho_poly(z, d, Y, mode=1)
    rel = np.abs(poly - exact) / exact
    assert rel.max() < 1.5e-14, rel.max()


def two_centre_clusters():
    """Generators of the two-centre density: dense clusters at chord 0.35
    from each bump's centre (cells small enough for both expansions in x),
    one at the first centre (too close to it), and a uniform background."""
    d = I.density_two_centre()
    x0, x1 = np.array(d["xc"][0]), np.array(d["xc"][1])
    Z = np.concatenate([I.cap_points(I.toward(x0, 0.35, 7), 0.012, 600, 8),
                        I.cap_points(I.toward(x1, 0.35, 9), 0.012, 400, 10),
                        I.cap_points(x0, 0.004, 100, 11), I.uniform_sphere(300, 12)])
    rad = np.concatenate([np.full(1000, 4 * 0.012 / math.sqrt(400)), np.full(100, 4e-3),
                          np.full(300, 4 * math.sqrt(4 * math.pi / 300))])
    return d, Z, rad


def test_two_bump_polynomial_quadrature_matches_oracle():
    """Cells of the two-centre density inside both bumps' expansion radii:
    their integrals through the two expansions in x agree with the direct
    FP64 path on the same vertices to 2e-14 and with the oracle to 1e-12 on
    m and mu and 3e-12 on e (as for one bump); cells at the first bump's
    centre do not qualify."""
    d, Z, rad = two_centre_clusters()
    ev = oracle.evaluate(Z, d)
    st, deg, nbr, verts, R = hc.cells(Z, rad)
    used = 0
    worst = [0.0, 0.0, 0.0, 0.0]
    for k in np.where(st == 0)[0]:
        res = hc.quad_poly(Z[k], deg[k], verts[k], d, force=2)
        if 1000 <= k < 1100:
            assert res is None  # at the centre: the entry radius shrinks to nothing
        if res is None:
            continue
        out = res[0]
        used += 1
        ref = hc.quad(Z[k], deg[k], verts[k], d)
        worst[0] = max(worst[0], abs(out[0] - ev.m[k]) / ev.m[k])
        worst[1] = max(worst[1], np.linalg.norm(out[1:4] - ev.mu[k]) / np.linalg.norm(ev.mu[k]))
        worst[2] = max(worst[2], abs(out[4] - ev.e[k]) / ev.e[k])
        worst[3] = max(worst[3], abs(out[0] - ref[0]) / ref[0], abs(out[4] - ref[4]) / ref[4])
    assert used >= 700, used
    assert max(worst[:2]) < 1e-12 and worst[2] < 3e-12, worst
    assert worst[3] < 2e-14, worst


@pytest.mark.parametrize("density", ["tanh16", "two"])
def test_mixed_expansion_in_x_error(density):
    """The mixed path's FP32 copies of the expansions in x (degree 5, one or
    two bumps) on cells inside the entries' radii, against the FP64 oracle:
    per cell |dm|/m and |de|/e <= 1e-5 and centroid error <= 1e-7 h_i."""
    if density == "two":
        d, Z, rad = two_centre_clusters()
    else:
        d = I.CONFIGS["C3"]["density"]
        xc = np.array(d["xc"][0])
        Z = np.concatenate([I.cap_points(I.toward(xc, 0.349, 7), 0.012, 600, 8),
                            I.uniform_sphere(200, 9)])
        rad = np.concatenate([np.full(600, 4 * 0.012 / math.sqrt(600)),
                              np.full(200, 4 * math.sqrt(4 * math.pi / 200))])
    n = len(Z)
    ev = oracle.evaluate(Z, d)
    i, j, _ = oracle.neighbour_sets(Z, ev.cells)
    dist = np.linalg.norm(Z[i] - Z[j], axis=1)
    hi = (np.bincount(i, dist, n) + np.bincount(j, dist, n)) / (
        np.bincount(i, minlength=n) + np.bincount(j, minlength=n))
    st, deg, nbr, verts, R = hc.cells(Z, rad)
    used = 0
    worst = 0.0
    for k in np.where(st == 0)[0]:
        out = hc.quad_mixed_poly(Z[k], deg[k], verts[k], d)
        if out is None:
            continue
        used += 1
        assert abs(out[0] - ev.m[k]) <= 1e-5 * ev.m[k]
        assert abs(out[4] - ev.e[k]) <= 1e-5 * ev.e[k]
        worst = max(worst, np.linalg.norm(out[1:4] / out[0] - ev.centroid[k]) / hi[k])
    print("mixed expansion in x, %s: %d cells, max centroid error / h = %.2e" % (density, used, worst))
    assert used >= 400, used
    assert worst <= 1e-7
