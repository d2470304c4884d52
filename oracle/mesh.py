"""Mesh operations of the method, written from their definitions (test
infrastructure only, like the rest of the oracle).

    refine       -- the bisection step of the optimisation-bisection
                    initialisation (section 3.3; section 4.3 bisects a
                    converged 2,562-generator SCVT up to 655,362): every
                    Delaunay edge (i, j) gets the normalised midpoint of its
                    generators, appended in the order of (i, j), i < j.
    triangles    -- the Delaunay triangulation (the convex hull's facets,
                    counter-clockwise seen from outside), the mesh the paper
                    exports at the end of its algorithm (section 3.3).
    cell_quality -- cellQ(V) = min edge / max edge of each Voronoi cell
                    (section 4), with chord lengths between consecutive
                    Voronoi vertices.
    tri_quality  -- triQ = (a+b-c)(b+c-a)(c+a-b)/(abc) of each triangle
                    (section 4, eq. Qdef), with chord edge lengths.
"""
import numpy as np

from .voronoi import cells, delaunay, delaunay_edges


def refine(Z):
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    F = delaunay(Z)
    i, j, _, _ = delaunay_edges(Z, F)          # unique edges, sorted by (i, j)
    M = Z[i] + Z[j]
    M = M / np.linalg.norm(M, axis=1)[:, None]
    return np.vstack([Z, M])


def canonical_triangles(T):
    """Rotate each triangle so that its smallest index comes first (the
    orientation is kept) and sort the rows: a form two lists of the same
    triangulation share."""
    T = np.asarray(T, dtype=np.int64)
    r = np.argmin(T, axis=1)
    idx = (r[:, None] + np.arange(3)[None, :]) % 3
    R = np.take_along_axis(T, idx, axis=1)
    return R[np.lexsort((R[:, 2], R[:, 1], R[:, 0]))]


def triangles(Z):
    return canonical_triangles(delaunay(np.ascontiguousarray(Z, dtype=np.float64)))


def cell_quality(Z, C=None):
    if C is None:
        C = cells(Z)
    q = np.zeros(C.n)
    for k in range(C.n):
        v = C.verts[C.ptr[k]:C.ptr[k + 1]]
        e = np.linalg.norm(np.roll(v, -1, axis=0) - v, axis=1)
        q[k] = e.min() / e.max()
    return q


def tri_quality(Z, T):
    Z = np.asarray(Z, dtype=np.float64)
    T = np.asarray(T)
    a = np.linalg.norm(Z[T[:, 1]] - Z[T[:, 2]], axis=1)
    b = np.linalg.norm(Z[T[:, 2]] - Z[T[:, 0]], axis=1)
    c = np.linalg.norm(Z[T[:, 0]] - Z[T[:, 1]], axis=1)
    return (a + b - c) * (b + c - a) * (c + a - b) / (a * b * c)
