"""Pins for the oracle's optimizer (not the GPU path).

  * the two-loop recursion with H0 = diag(h) equals the dense BFGS matrix
    built by the product-form update (section 2.2.2; the printed factor
    S_i = I - rho_i s_i s_i^T is read as the standard I - rho_i y_i s_i^T,
    the only form that satisfies the secant equation also printed there);
  * the secant equation H y_newest = s_newest holds;
  * with no history (M = 0, or the first step) the step is exactly the
    Lloyd step mu/|mu| (section 3.1: Lloyd direction with step 1);
  * the analytic gradient 2 m z - 2 mu matches central differences of F
    along tangent directions (section 2.2.1, dF/dV = 0);
  * F decreases monotonically under the Armijo line search;
  * converged uniform-density energy matches the hexagonal (Gersho) constant
    5/(18 sqrt 3) (int rho^1/2)^2 / n, and the X3 energy matches the paper's
    Table 1 value within the spread of local minima.
"""
import math
import os

import numpy as np
import pytest

import oracle
import paper_1709_06924_amd.inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_bfgs(h3, hist):
    H = np.diag(h3)
    for s, y, r in hist:                       # oldest to newest
        V = np.eye(len(s)) - r * np.outer(y, s)
        H = V.T @ H @ V + r * np.outer(s, s)
    return H


@pytest.mark.parametrize("ngen,M,seed", [(4, 3, 0), (17, 7, 1), (50, 10, 2)])
def test_two_loop_equals_dense_bfgs(ngen, M, seed):
    rng = np.random.default_rng(seed)
    d = 3 * ngen
    A = rng.standard_normal((d, d))
    A = A @ A.T + d * np.eye(d)                # SPD model Hessian
    hist = []
    for _ in range(M):
        s = rng.standard_normal(d)
        y = A @ s
        hist.append((s.reshape(ngen, 3), y.reshape(ngen, 3), 1.0 / np.dot(y, s)))
    h = rng.uniform(0.5, 2.0, ngen)
    g = rng.standard_normal((ngen, 3))
    q = oracle.two_loop(g, h, hist)
    H = dense_bfgs(np.repeat(h, 3), [(s.ravel(), y.ravel(), r) for s, y, r in hist])
    ref = -(H @ g.ravel())
    assert np.linalg.norm(q.ravel() - ref) <= 1e-13 * np.linalg.norm(ref) * d
    s, y, r = hist[-1]
    assert np.allclose(H @ y.ravel(), s.ravel(), rtol=1e-10, atol=1e-12)


def test_no_history_is_lloyd_step():
    d = I.density_tanh(I.latlon(30, 90), math.pi / 6, 0.2, 8)
    Z = I.uniform_sphere(500, 4)
    for M in (0, 7):
        S = oracle.Solver(Z, d, m_hist=M)
        ev0 = S.cur
        S.step()
        assert S.last_alpha == 1.0
        target = ev0.mu / np.linalg.norm(ev0.mu, axis=1)[:, None]
        assert np.max(np.abs(S.Z - target)) < 1e-14
        assert np.max(np.abs(S.Z - (ev0.Z + ev0.lloyd))) < 1e-14


def test_gradient_matches_finite_differences():
    d = I.density_tanh(I.latlon(30, 90), math.pi / 4, 0.4, 4)
    Z = I.uniform_sphere(80, 6)
    ev = oracle.evaluate(Z, d)
    rng = np.random.default_rng(0)
    eps = 1e-5
    for i in rng.choice(80, 6, replace=False):
        t = np.cross(Z[i], rng.standard_normal(3))
        t /= np.linalg.norm(t)
        Fp = oracle.evaluate(np.vstack([Z[:i], (Z[i] + eps * t) / np.linalg.norm(Z[i] + eps * t), Z[i + 1:]]), d).F
        Fm = oracle.evaluate(np.vstack([Z[:i], (Z[i] - eps * t) / np.linalg.norm(Z[i] - eps * t), Z[i + 1:]]), d).F
        fd = (Fp - Fm) / (2 * eps)
        an = np.dot(ev.g[i], t)
        assert abs(fd - an) <= 1e-6 * np.linalg.norm(ev.g[i]) + 1e-9 * ev.F


def test_tangential_gradient_and_preconditioner_algebra():
    Z = I.uniform_sphere(300, 8)
    ev = oracle.evaluate(Z, I.density_x3())
    # tangential: g_i . z_i = 0; ambient gradient 2 m z - 2 mu projected
    assert np.max(np.abs(np.einsum("ij,ij->i", ev.g, Z))) < 1e-15
    G = 2 * ev.m[:, None] * Z - 2 * ev.mu
    Gt = G - np.einsum("ij,ij->i", G, Z)[:, None] * Z
    assert np.max(np.abs(Gt - ev.g)) < 1e-15
    # z - h g = mu / (mu.z), whose projection is the constrained centroid
    d = Z - ev.h[:, None] * ev.g
    mz = np.einsum("ij,ij->i", ev.mu, Z)
    assert np.max(np.abs(d - ev.mu / mz[:, None])) < 1e-12


@pytest.mark.parametrize("density", ["const", "tanh"])
def test_energy_monotone(density):
    d = {"kind": "const"} if density == "const" else I.density_tanh(I.latlon(30, 90), math.pi / 6, 0.2, 8)
    S = oracle.Solver(I.uniform_sphere(400, 9), d, m_hist=7)
    for _ in range(25):
        S.step()
    F = np.array(S.history_F)
    assert np.all(np.diff(F) <= 0)
    assert F[-1] < F[0]
    assert S.n_evals >= S.iter + 1


@pytest.mark.slow
def test_gersho_magnitude_uniform():
    n = 2562
    S = oracle.Solver(I.uniform_sphere(n, 1), {"kind": "const"}, m_hist=7)
    ev = S.solve(250, 1e-10)
    gersho = 5 / (18 * math.sqrt(3)) * (4 * math.pi) ** 2 / n
    # Fejes Toth's bound: no n-point configuration beats the hexagonal
    # constant; a converged SCVT (12 pentagons) sits a little above it
    assert 1.0 <= ev.F / gersho < 1.012
    assert ev.step_inf < 1e-3


@pytest.mark.slow
def test_x3_energy_near_paper_table():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_table1_x3.txt"))
            if l.strip() and not l.startswith("#")][1:]
    paper = {int(a): float(b) for a, b in rows}
    n = 2562
    S = oracle.Solver(I.uniform_sphere(n, 1), I.density_x3(), m_hist=7)
    ev = S.solve(200, 5e-6)
    # The printed value sits 2.6% below the hexagonal bound
    # 5/(18 sqrt 3) (int rho^1/2)^2 / n (a systematic offset of the paper's
    # numbers, same ratio at both n); our converged energy sits 0.8% above
    # that bound, as for rho = 1.  The pin is therefore a 5% band.
    assert abs(ev.F - paper[n]) / paper[n] < 0.05
    sqrt_mass = 2 * math.pi * sum(  # int rho^1/2 over the sphere, z = cos(theta)
        math.sqrt((1 - 3.0 ** -4) * z ** 4 + 3.0 ** -4) * w
        for z, w in zip(*np.polynomial.legendre.leggauss(200)))
    bound = 5 / (18 * math.sqrt(3)) * sqrt_mass ** 2 / n
    assert 1.0 <= ev.F / bound < 1.015


def test_line_search_failure_takes_lloyd_step():
    """With one evaluation per line search and c1 close to 1 the Armijo test
    fails; the iteration then takes the Lloyd step mu/|mu| (section 2.2.1)
    and clears the history."""
    d = I.density_tanh(I.latlon(30, 90), math.pi / 6, 0.2, 8)
    S = oracle.Solver(I.uniform_sphere(300, 14), d, m_hist=7, ls_max_evals=1, c1=0.9999)
    for _ in range(6):
        ev0 = S.cur
        n0 = S.n_lloyd_fallback
        S.step()
        if S.n_lloyd_fallback > n0:
            target = ev0.mu / np.linalg.norm(ev0.mu, axis=1)[:, None]
            assert np.max(np.abs(S.Z - target)) < 1e-14
            assert len(S.hist) <= 1
    assert S.n_lloyd_fallback >= 1
    assert S.history_F[-1] < S.history_F[0]


# ---- the compared methods of section 4.1: Lloyd and plain LBFGS ----

@pytest.mark.parametrize("density", [I.density_x3(),
                                     I.density_tanh(I.latlon(30, 90), math.pi / 6, 0.2, 8)])
def test_lloyd_method_is_the_centroid_map_and_descends(density):
    """Lloyd's method (section 2.2.1): each iteration moves every generator to
    its constrained mass centroid mu/|mu| = z + l, and F never increases."""
    Z = I.uniform_sphere(600, 21)
    S = oracle.Solver(Z, density, method="lloyd")
    F = [S.cur.F]
    for _ in range(5):
        ev0 = S.cur
        S.step()
        target = ev0.mu / np.linalg.norm(ev0.mu, axis=1)[:, None]
        assert np.array_equal(S.Z, target)
        assert np.max(np.abs(S.Z - (ev0.Z + ev0.lloyd))) < 1e-15
        F.append(S.cur.F)
    assert np.all(np.diff(F) <= 0.0)
    assert S.n_evals == 6 and S.hist == []


@pytest.mark.parametrize("name", ["tetra", "octa", "icosa"])
def test_platonic_sets_are_lloyd_fixed_points(name):
    P = I.platonic(name)
    S = oracle.Solver(P, {"kind": "const"}, method="lloyd")
    S.step()
    assert np.max(np.abs(S.Z - P)) < 1e-15


def test_plain_lbfgs_scaling_and_first_direction():
    """Plain LBFGS (section 2.2.2): with no stored pair the direction is -g;
    afterwards the initial inverse Hessian is gamma_n I with gamma_n =
    y.s / y.y of the newest pair, and the direction is the dense BFGS
    product with that H0."""
    d = I.density_tanh(I.latlon(30, 90), math.pi / 6, 0.2, 8)
    S = oracle.Solver(I.uniform_sphere(400, 22), d, method="lbfgs", m_hist=5)
    q0 = S.direction()
    assert np.array_equal(q0, -S.cur.g)
    for _ in range(4):
        S.step()
    assert len(S.hist) >= 1
    s, y, r = S.hist[-1]
    gam = np.sum(y * s) / np.sum(y * y)
    H = dense_bfgs(np.full(3 * len(S.Z), gam), [(a.ravel(), b.ravel(), c) for a, b, c in S.hist])
    ref = -(H @ S.cur.g.ravel())
    q = S.direction()
    assert np.linalg.norm(q.ravel() - ref) <= 1e-11 * np.linalg.norm(ref)
    # the Lloyd-preconditioned direction differs (diag(h) is not a multiple of I)
    P = oracle.two_loop(S.cur.g, S.cur.h, S.hist)
    assert np.linalg.norm(P - q) > 1e-3 * np.linalg.norm(q)


def test_solve_rel_stopping_tests():
    d = I.density_x3()
    Z = I.uniform_sphere(300, 23)
    S = oracle.Solver(Z, d, method="plbfgs")
    assert S.solve_rel(10, grad_rel_tol=1e30) and S.iter == 0        # gradient test first
    S = oracle.Solver(Z, d, method="plbfgs")
    assert S.solve_rel(10, f_rel_tol=1.0) and S.iter == 1            # |dF|/F < 1 after one step
    S = oracle.Solver(Z, d, method="lloyd")
    assert not S.solve_rel(3, grad_rel_tol=1e30, f_rel_tol=1.0)      # Lloyd: movement test only
    assert S.iter == 3
    S = oracle.Solver(Z, d, method="lloyd")
    assert S.solve_rel(50, step_tol=1.0) and S.iter == 0


def test_lloyd_fallback_that_raises_energy_is_an_error():
    """Lloyd's step lowers the exact energy (section 2.2.1), not necessarily
    a coarse quadrature of it: eight generators under the X64 density with
    the 4-point rule and no subdivision (cells a quarter of the sphere wide)
    find no decrease along the first direction in ten evaluations, and the
    Lloyd step raises the evaluated F by a third.  The iteration ends with
    LineSearchError, the generators and F where they were."""
    d = I.density_x64()
    O = oracle.Solver(I.uniform_sphere(8, 205), d, m_hist=7, levels=0, rule=4)
    Z, F = O.Z.copy(), O.cur.F
    with pytest.raises(oracle.LineSearchError):
        O.step()
    assert np.array_equal(O.Z, Z) and O.cur.F == F and O.iter == 0
    assert O.n_evals == 1 + 10 + 1 and O.hist == []
    # the same start with the default rule (7 points, 2 levels) descends
    P = oracle.Solver(I.uniform_sphere(8, 205), d, m_hist=7)
    P.step()
    assert P.cur.F < P.history_F[0]
