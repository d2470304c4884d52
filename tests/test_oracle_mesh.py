"""Pins of the oracle's mesh operations: bisection, triangle list, quality
measures."""
import itertools
import math

import numpy as np
import pytest

import oracle
import paper_1709_06924_amd.inputs as I


def test_bisected_icosahedron_is_the_42_point_geodesic_grid():
    """The icosahedron's 30 edges are exactly its pairs at the minimal
    distance; bisection appends their normalised midpoints (12 -> 42)."""
    P = I.platonic("icosa")
    R = oracle.mesh.refine(P)
    assert len(R) == 42 == 4 * 12 - 6
    assert np.array_equal(R[:12], P)
    d = np.linalg.norm(P[:, None] - P[None], axis=2)
    dmin = d[d > 0].min()
    pairs = [(i, j) for i, j in itertools.combinations(range(12), 2) if d[i, j] < dmin * (1 + 1e-9)]
    assert len(pairs) == 30
    mids = np.array([(P[i] + P[j]) / np.linalg.norm(P[i] + P[j]) for i, j in pairs])
    assert np.max(np.abs(R[12:] - mids)) < 1e-15       # same (i, j) order
    # all 42 points are unit and the new ones equidistant from their parents
    assert np.max(np.abs(np.linalg.norm(R, axis=1) - 1)) < 1e-15
    assert np.max(np.abs(np.linalg.norm(R[12:] - P[[p[0] for p in pairs]], axis=1) -
                         np.linalg.norm(R[12:] - P[[p[1] for p in pairs]], axis=1))) < 1e-15


@pytest.mark.parametrize("n,seed", [(100, 1), (2000, 2)])
def test_bisection_counts_and_midpoints(n, seed):
    """A spherical triangulation has 3n - 6 edges (Euler), so n -> 4n - 6;
    each new point is the normalised midpoint of two generators that share a
    Voronoi edge, listed once, in (i, j) order."""
    Z = I.uniform_sphere(n, seed)
    R = oracle.mesh.refine(Z)
    assert len(R) == 4 * n - 6
    C = oracle.cells(Z)
    nbr = [set() for _ in range(n)]
    for a, b, c in C.F:
        nbr[a] |= {b, c}
        nbr[b] |= {a, c}
        nbr[c] |= {a, b}
    pairs = sorted((i, j) for i in range(n) for j in nbr[i] if j > i)
    assert len(pairs) == 3 * n - 6
    i = np.array([p[0] for p in pairs])
    j = np.array([p[1] for p in pairs])
    M = Z[i] + Z[j]
    assert np.array_equal(R[n:], M / np.linalg.norm(M, axis=1)[:, None])


def test_triangles_are_the_delaunay_facets():
    """2n - 4 triangles, counter-clockwise seen from outside (positive
    orientation), each with an empty circumcircle (brute force)."""
    n = 300
    Z = I.uniform_sphere(n, 3)
    T = oracle.mesh.triangles(Z)
    assert len(T) == 2 * n - 4
    assert np.all(T[:, 0] < T[:, 1]) and np.all(T[:, 0] < T[:, 2])
    A, B, C = Z[T[:, 0]], Z[T[:, 1]], Z[T[:, 2]]
    nrm = np.cross(B - A, C - A)
    assert np.all(np.einsum("ij,ij->i", nrm, A) > 0)           # outward
    s = np.einsum("tj,tkj->tk", nrm, Z[None, :, :] - A[:, None, :])
    assert np.all(s <= 1e-12)                                  # empty circle


def test_quality_measures_closed_forms():
    """triQ is 1 for an equilateral triangle and 0 for a degenerate one; the
    octahedron's cells are squares (cellQ = 1) and its triangles equilateral;
    a cube's cells are triangles (cellQ = 1)."""
    Z = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0], [-1.0, 0, 0], [0, -1.0, 0], [0, 0, -1.0]])
    T = oracle.mesh.triangles(Z)
    assert len(T) == 8
    assert np.allclose(oracle.mesh.tri_quality(Z, T), 1.0, atol=1e-15)
    assert np.allclose(oracle.mesh.cell_quality(Z), 1.0, atol=1e-15)
    flat = np.array([[0.0, 0, 0], [1.0, 0, 0], [3.0, 0, 0]])     # collinear
    assert abs(oracle.mesh.tri_quality(flat, np.array([[0, 1, 2]]))[0]) < 1e-15
    # a right isosceles triangle: a = b = 1, c = sqrt 2
    R = np.array([[0.0, 0, 0], [1.0, 0, 0], [0, 1.0, 0]])
    q = oracle.mesh.tri_quality(R, np.array([[0, 1, 2]]))[0]
    s2 = math.sqrt(2)
    assert abs(q - (2 - s2) * s2 * s2 / s2) < 1e-15
    Q = oracle.mesh.cell_quality(I.platonic("icosa"))
    assert np.allclose(Q, 1.0, atol=1e-14)                     # regular pentagons
