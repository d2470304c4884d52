"""Pins for the oracle's quadrature (not the GPU path).

The rule is the documented reading of the configurations' "7-point rule on
each spherical triangle with 2 levels of subdivision"; the paper names no rule
for these runs (section 4 uses unnamed 4- and 9-point rules).  Pins:
  * the planar 7-point rule integrates every monomial of degree <= 5 exactly
    and is not exact at degree 6 (so it is a degree-5 rule with these nodes);
  * on spherical triangles at rho = 1 the radial-projection rule converges to
    the closed-form area (Van Oosterom-Strackee) and first moment (Stokes on
    the cone: 1/2 sum over edges of arc angle times unit edge-plane normal)
    at the order of a degree-5 rule (error ratio near 2^6 per level).
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
from oracle import _clib


def rule7():
    lam = np.zeros(21)
    w = np.zeros(7)
    _clib.lib().oracle_rule7(_clib.ptr(lam), _clib.ptr(w))
    return lam.reshape(7, 3), w


def test_rule7_weights_and_nodes():
    lam, w = rule7()
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(lam.sum(axis=1), 1.0, atol=1e-15)
    assert np.all(lam > 0) and np.all(w > 0)


@pytest.mark.parametrize("deg", range(0, 7))
def test_rule7_planar_monomials(deg):
    lam, w = rule7()
    # reference triangle (0,0),(1,0),(0,1): x = lam1, y = lam2, area 1/2
    x, y = lam[:, 1], lam[:, 2]
    worst = 0.0
    for a in range(deg + 1):
        b = deg - a
        exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
        approx = 0.5 * np.sum(w * x ** a * y ** b)
        worst = max(worst, abs(approx - exact) / exact)
    if deg <= 5:
        assert worst < 5e-15
    else:
        assert worst > 1e-6


def vos_area(a, b, c):
    """Van Oosterom-Strackee solid angle of the spherical triangle (a,b,c)."""
    num = np.dot(a, np.cross(b, c))
    den = 1 + np.dot(a, b) + np.dot(b, c) + np.dot(c, a)
    return 2 * math.atan2(num, den)


def stokes_moment(verts):
    """int y dsigma over a CCW spherical polygon = 1/2 sum theta_e n_e."""
    mu = np.zeros(3)
    k = len(verts)
    for t in range(k):
        p, q = verts[t], verts[(t + 1) % k]
        cr = np.cross(p, q)
        theta = math.atan2(np.linalg.norm(cr), np.dot(p, q))
        mu += 0.5 * theta * cr / np.linalg.norm(cr)
    return mu


def tri_integrals(z, A, B, C, levels, density=None, rule=7):
    from oracle.rules import crule
    D = _clib.cdensity(density or {"kind": "const"})
    out = np.zeros(5)
    arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (z, A, B, C)]
    _clib.lib().oracle_triangle_integrals(ctypes.byref(D), *[_clib.ptr(v) for v in arrs],
                                          int(levels), ctypes.byref(crule(rule)), _clib.ptr(out))
    return out


def unit(v):
    v = np.asarray(v, dtype=float)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("size", [0.05, 0.3, 1.0])
def test_spherical_triangle_closed_forms_converge(size):
    rng = np.random.default_rng(7)
    z = unit(rng.standard_normal(3))
    t = [unit(z + size * unit(rng.standard_normal(3))) for _ in range(3)]
    A, B, C = t
    if np.dot(A, np.cross(B, C)) < 0:
        B, C = C, B
    area = vos_area(A, B, C)
    mu = stokes_moment([A, B, C])
    e = 2 * area - 2 * np.dot(z, mu)  # |y-z|^2 = 2 - 2 y.z on the unit sphere
    # the closed-form energy 2m - 2 z.mu cancels digits on small triangles, so
    # its own rounding floor is about 1e-15 * 2m / e (relative to e)
    e_floor = 1e-15 * 2 * area / e
    errs = []
    for L in range(0, 5):
        r = tri_integrals(z, A, B, C, L)
        errs.append(max(abs(r[0] - area) / area, np.linalg.norm(r[1:4] - mu) / np.linalg.norm(mu)))
        assert abs(r[4] - e) / e < max(10 * errs[-1] * 2 * area / e, 100 * e_floor) + 1e-2 * (L == 0)
    assert errs[-1] < 1e-10
    # degree-5 rule: the error falls by about 2^6 per level once resolved
    for L in range(1, 5):
        if errs[L] > 1e-13:
            assert errs[L - 1] / errs[L] > 30.0

def test_density_values():
    import paper_1709_06924_amd.inputs as I
    L = _clib.lib()
    d = I.density_tanh(I.latlon(30, 90), math.pi / 6, 0.2, 8)
    D = _clib.cdensity(d)
    xc = np.array(d["xc"][0])
    far = -xc
    rho_c = L.oracle_rho(ctypes.byref(D), _clib.ptr(np.ascontiguousarray(xc)))
    rho_f = L.oracle_rho(ctypes.byref(D), _clib.ptr(np.ascontiguousarray(far)))
    g = d["gamma"]
    exact_c = g + (1 - g) * 0.5 * (math.tanh((math.pi / 6) / 0.2) + 1)
    exact_f = g + (1 - g) * 0.5 * (math.tanh((math.pi / 6 - 2.0) / 0.2) + 1)
    assert abs(rho_c - exact_c) < 1e-15 and abs(rho_f - exact_f) < 1e-15
    assert rho_f / rho_c < 8.0 ** -4 * 1.01  # 8x spacing ratio, section 4
    x3 = _clib.cdensity(I.density_x3())
    p = np.array([0.0, 0.6, 0.8])
    assert abs(L.oracle_rho(ctypes.byref(x3), _clib.ptr(p)) - ((1 - 3.0 ** -4) * 0.8 ** 4 + 3.0 ** -4)) < 1e-15


# ---- the conical product rules of 4 and 9 points (the sizes of section 4.1)

@pytest.mark.parametrize("nq,degree", [(4, 3), (9, 5)])
def test_conical_rules_exactness(nq, degree):
    """Exact on every planar monomial up to the rule's degree, not beyond;
    positive weights summing to one, points inside the triangle."""
    from oracle.rules import rule
    lam, w = rule(nq)
    assert len(w) == nq and abs(w.sum() - 1.0) < 1e-15 and np.all(w > 0)
    assert np.all(lam > 0) and np.allclose(lam.sum(axis=1), 1.0, atol=1e-15)
    x, y = lam[:, 1], lam[:, 2]
    for deg in range(degree + 2):
        worst = 0.0
        for a in range(deg + 1):
            b = deg - a
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            worst = max(worst, abs(0.5 * np.sum(w * x ** a * y ** b) - exact) / exact)
        if deg <= degree:
            assert worst < 5e-15, (deg, worst)
        else:
            assert worst > 1e-6


@pytest.mark.parametrize("nq,ratio", [(4, 12.0), (9, 30.0)])
def test_conical_rules_converge_on_spherical_triangles(nq, ratio):
    """Through the radial projection the 4-point (degree 3) rule's error
    falls by about 2^4 per subdivision level, the 9-point (degree 5) rule's
    by about 2^6, toward the closed-form area and first moment."""
    rng = np.random.default_rng(8)
    z = unit(rng.standard_normal(3))
    A, B, C = [unit(z + 0.3 * unit(rng.standard_normal(3))) for _ in range(3)]
    if np.dot(A, np.cross(B, C)) < 0:
        B, C = C, B
    area = vos_area(A, B, C)
    mu = stokes_moment([A, B, C])
    errs = []
    for L in range(0, 5):
        r = tri_integrals(z, A, B, C, L, rule=nq)
        errs.append(max(abs(r[0] - area) / area, np.linalg.norm(r[1:4] - mu) / np.linalg.norm(mu)))
    for L in range(1, 5):
        if errs[L] > 1e-13:
            assert errs[L - 1] / errs[L] > ratio, errs


# ---- the anisotropic X16 density of section 4 --------------------------------

def _x16_closed_form(d, lat, lon):
    """rho at (lat, lon) from the section-4 definition written with spherical
    trigonometry instead of points: z_ic shares the point's latitude and the
    centre's longitude, so |z - z_ic| is the arc between two points of one
    parallel, 2 asin(cos(lat) |sin(dlon/2)|); z_ci shares the centre's
    latitude and the point's longitude, so |z - z_ci| = |lat - lat_c| along
    one meridian.  (tanh(x) + 1)/2 in its tanh form."""
    xc = np.array(d["xc"][0])
    lat_c = math.asin(xc[2])
    lon_c = math.atan2(xc[1], xc[0])
    dlon = lon - lon_c
    d_lon = 2.0 * math.asin(math.cos(lat) * abs(math.sin(dlon / 2.0)))
    d_lat = abs(lat - lat_c)
    dist = math.sqrt((d_lon / d["w_lon"]) ** 2 + (d_lat / d["w_lat"]) ** 2)
    t = (d["beta"][0] - dist) / d["alpha"][0]
    return d["gamma"] + d["amp"][0] * 0.5 * (math.tanh(t) + 1.0), dist


def _x16_at(d, lat, lon):
    L = _clib.lib()
    D = _clib.cdensity(d)
    p = np.array([math.cos(lat) * math.cos(lon), math.cos(lat) * math.sin(lon), math.sin(lat)])
    return L.oracle_rho(ctypes.byref(D), _clib.ptr(p))


@pytest.mark.parametrize("centre", [(0.0, 0.0), (20.0, 40.0), (-35.0, -120.0)])
def test_x16_density_closed_forms(centre):
    """X16 (section 4) at points on the centre's parallel (distance = the
    parallel's arc over w_lon), on its meridian (distance = latitude offset
    over w_lat) and anywhere (both terms), against the closed form; a swap of
    the widths or of the two auxiliary points fails the first two families."""
    import paper_1709_06924_amd.inputs as I
    d = I.density_x16()
    lat_c, lon_c = map(math.radians, centre)
    d["xc"] = [I.latlon(*centre)]
    worst = 0.0
    # on the centre's parallel: only the longitude term
    for dl in np.linspace(-3.0, 3.0, 25):
        rho, dist = _x16_closed_form(d, lat_c, lon_c + dl)
        assert abs(dist - 2 * math.asin(math.cos(lat_c) * abs(math.sin(dl / 2))) / d["w_lon"]) < 1e-15
        worst = max(worst, abs(_x16_at(d, lat_c, lon_c + dl) - rho))
    # on the centre's meridian: only the latitude term
    for la in np.linspace(-1.5, 1.5, 25):
        rho, dist = _x16_closed_form(d, la, lon_c)
        assert abs(dist - abs(la - lat_c) / d["w_lat"]) < 1e-15
        worst = max(worst, abs(_x16_at(d, la, lon_c) - rho))
    # general points
    rng = np.random.default_rng(16)
    for _ in range(200):
        la, lo = rng.uniform(-1.5, 1.5), rng.uniform(-math.pi, math.pi)
        rho, _ = _x16_closed_form(d, la, lo)
        worst = max(worst, abs(_x16_at(d, la, lo) - rho))
    assert worst < 2e-15, worst
    # the anisotropy: the same angular offset costs w_lat/w_lon = 4 times more
    # distance along the parallel than along the meridian
    if centre == (0.0, 0.0):
        r_lon = _x16_at(d, 0.0, 0.3)
        r_lat = _x16_at(d, 1.2, 0.0)
        exact = d["gamma"] + d["amp"][0] * 0.5 * (math.tanh((d["beta"][0] - 1.0) / d["alpha"][0]) + 1)
        assert abs(r_lon - exact) < 1e-15 and abs(r_lat - exact) < 1e-15
        assert abs(_x16_at(d, 0.0, 0.0) - (d["gamma"] + d["amp"][0] * 0.5 * (
            math.tanh(d["beta"][0] / d["alpha"][0]) + 1))) < 1e-15


def test_oracle_c_under_address_and_ub_sanitizers(tmp_path):
    """The oracle's C integrals built with AddressSanitizer and
    UndefinedBehaviorSanitizer (gcc, host code) run every density kind, both
    rule kinds and several subdivision levels without a report."""
    import os
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    here = os.path.dirname(os.path.abspath(__file__))
    exe = str(tmp_path / "oracle_sanitize")
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-ffp-contract=off",
                           "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-o", exe,
                           os.path.join(here, "host", "oracle_sanitize.c"), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr
    assert "0 failures" in p.stdout
