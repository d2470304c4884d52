"""Bisection, the optimisation-bisection driver and the mesh export /
quality measures on the device, against the oracle's definitions."""
import math

import numpy as np
import pytest

import oracle
import paper_1709_06924_amd.inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def scvt():
    from paper_1709_06924_amd import scvt as s
    return s


@pytest.mark.parametrize("n,seed", [(12, None), (200, 41), (5000, 42)])
def test_refine_matches_oracle(scvt, n, seed):
    Z = I.platonic("icosa") if seed is None else I.uniform_sphere(n, seed)
    S = scvt.Solver(Z, {"kind": "const"})
    Zg = S.generators()
    R = S.refine()
    ref = oracle.mesh.refine(Zg)
    assert R.shape == ref.shape == (4 * n - 6, 3)
    assert np.max(np.abs(R - ref)) <= 1e-15


def test_multilevel_from_icosahedron(scvt):
    """Optimisation-bisection from the icosahedron: 12 -> 42 -> 162 -> 642
    -> 2,562 generators (the paper's coarse sizes), each level solved; the
    final uniform SCVT sits just above the hexagonal energy bound."""
    S, infos = scvt.multilevel(I.platonic("icosa"), {"kind": "const"}, levels=4, max_iter=300,
                               tol=1e-9, m_hist=7)
    sizes = [12, 42, 162, 642, 2562]
    assert S.n == 2562
    for info, n in zip(infos, sizes):
        assert info["status"] >= 0
    assert infos[-1]["step_inf"] < 1e-9
    gersho = 5 / (18 * math.sqrt(3)) * (4 * math.pi) ** 2 / 2562
    assert 1.0 <= infos[-1]["F"] / gersho < 1.012
    # the last level's generators against the oracle's evaluation
    ev = oracle.evaluate(S.generators(), {"kind": "const"})
    assert abs(S.energy()[0] - ev.F) <= 1e-12 * ev.F


def test_multilevel_tanh_warm_start(scvt):
    """A bisected converged mesh is a better start than a uniform one: after
    the same number of iterations at 10,242 generators the warm start's
    Lloyd step and energy are smaller."""
    d = I.density_tanh(I.latlon(30, 90), math.pi / 6, 0.2, 8)
    S, infos = scvt.multilevel(I.uniform_sphere(2562, 43), d, levels=1, max_iter=150, tol=1e-9)
    assert S.n == 4 * 2562 - 6
    cold = scvt.Solver(I.uniform_sphere(S.n, 44), d).solve(150, 1e-9)
    print("warm", infos[1], "cold", cold)
    assert infos[1]["step_inf"] < cold["step_inf"]
    assert infos[1]["F"] < cold["F"]


@pytest.mark.parametrize("n,seed", [(200, 45), (3000, 46)])
def test_mesh_export_and_quality_match_oracle(scvt, n, seed):
    d = I.density_tanh(I.latlon(30, 90), math.pi / 6, 0.2, 8)
    S = scvt.Solver(I.uniform_sphere(n, seed), d)
    for _ in range(3):
        S.step()
    Zg = S.generators()
    tri, cq, tq = S.mesh()
    T = oracle.mesh.triangles(Zg)
    assert len(tri) == 2 * n - 4
    assert np.array_equal(tri.astype(np.int64), T)
    assert np.max(np.abs(cq - oracle.mesh.cell_quality(Zg))) < 1e-12
    assert np.max(np.abs(tq - oracle.mesh.tri_quality(Zg, T))) < 1e-12


def test_mesh_at_full_size(scvt):
    """n = 1,048,576: Euler's count of triangles, every edge in exactly two
    triangles with opposite orientations, quality measures in (0, 1]."""
    n = 1048576
    S = scvt.Solver(I.uniform_sphere(n, 3), I.CONFIGS["C3"]["density"], m_hist=10)
    tri, cq, tq = S.mesh()
    assert len(tri) == 2 * n - 4
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]]).astype(np.int64)
    key_fwd = e[:, 0] * n + e[:, 1]
    key_rev = e[:, 1] * n + e[:, 0]
    assert len(np.unique(key_fwd)) == len(key_fwd)             # each directed edge once
    assert np.array_equal(np.sort(key_fwd), np.sort(key_rev))  # and its reverse too
    assert np.all((cq > 0) & (cq <= 1)) and np.all((tq > 0) & (tq <= 1 + 1e-12))
