"""Spherical Voronoi cells from the 3-D convex hull (oracle).

Test infrastructure only.

Definition followed: the spherical Voronoi region of z_i is the set of points
of the sphere closer (Euclidean distance) to z_i than to every other generator
(section 2.1, eq. viInS; the paper stresses the metric stays Euclidean).  Its
dual is the Delaunay triangulation (section 2.1), which for points on the unit
sphere is exactly the convex hull: a hull facet's plane leaves every other
generator on the origin's side, i.e. no generator lies inside its circumcircle
(section 3.2.1, the empty-circle criterion).  The hull is taken from Qhull
through scipy (a library primitive); everything after it is written out here.

Voronoi vertex of facet {a,b,c}: the circumcentre on the sphere, computed from
the sorted triple a<b<c as normalize((z_b-z_a) x (z_c-z_a)), signed so that it
lies on z_a's side (it is equidistant from the three generators).
"""
import numpy as np
from scipy.spatial import ConvexHull

EPS = np.finfo(np.float64).eps


def delaunay(Z):
    """Facets (T,3) of the hull, each oriented counter-clockwise seen from
    outside the hull: (z_b - z_a) x (z_c - z_a) is the facet's outward normal
    (Qhull's facet equations give the outward direction)."""
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    hull = ConvexHull(Z)
    F = hull.simplices.astype(np.int64)
    nrm = np.cross(Z[F[:, 1]] - Z[F[:, 0]], Z[F[:, 2]] - Z[F[:, 0]])
    swap = np.einsum("ij,ij->i", nrm, hull.equations[:, :3]) < 0
    F[swap, 1], F[swap, 2] = F[swap, 2].copy(), F[swap, 1].copy()
    return F


def circumcentres(Z, F):
    """Voronoi vertex of every facet: the circumcentre on the sphere on the
    empty side of the facet, i.e. along its outward normal.  Computed from the
    sorted index triple, normalize((z_b-z_a) x (z_c-z_a)) with a<b<c, and
    signed to agree with the oriented facet's outward normal.  (When the origin
    is inside the hull this is the sign with v . z_a > 0; when all generators
    lie in one hemisphere the vertex of the far facet is more than 90 degrees
    from its generators.)"""
    S = np.sort(F, axis=1)
    za, zb, zc = Z[S[:, 0]], Z[S[:, 1]], Z[S[:, 2]]
    w = np.cross(zb - za, zc - za)
    w /= np.linalg.norm(w, axis=1)[:, None]
    out = np.cross(Z[F[:, 1]] - Z[F[:, 0]], Z[F[:, 2]] - Z[F[:, 0]])
    sgn = np.sign(np.einsum("ij,ij->i", w, out))
    sgn[sgn == 0] = 1.0
    return w * sgn[:, None]


def tangent_frame(Z):
    """Orthonormal (e1, e2) with (e1, e2, z) right-handed at every z."""
    a = np.zeros_like(Z)
    use_x = np.abs(Z[:, 0]) < 0.9
    a[use_x, 0] = 1.0
    a[~use_x, 1] = 1.0
    e1 = np.cross(Z, a)
    e1 /= np.linalg.norm(e1, axis=1)[:, None]
    e2 = np.cross(Z, e1)
    return e1, e2


class Cells:
    """Voronoi cells in CSR form.

    ptr (n+1,), fac (3T,) facet ids around each generator in counter-clockwise
    order seen from outside, verts (3T,3) the matching Voronoi vertices.
    """

    def __init__(self, Z, F, V, ptr, fac):
        self.Z, self.F, self.V, self.ptr, self.fac = Z, F, V, ptr, fac
        self.verts = np.ascontiguousarray(V[fac])

    @property
    def n(self):
        return len(self.ptr) - 1

    def deg(self):
        return np.diff(self.ptr)


def cells(Z, F=None):
    """Order the facets around each generator by azimuth in its tangent plane.
    A spherical Voronoi cell is convex and contains its generator, so it is
    star-shaped about it and azimuthal order is the boundary's cyclic order."""
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    if F is None:
        F = delaunay(Z)
    V = circumcentres(Z, F)
    n = len(Z)
    gen = F.reshape(-1)                      # generator of each incidence
    fac = np.repeat(np.arange(len(F)), 3)    # facet of each incidence
    e1, e2 = tangent_frame(Z)
    vv = V[fac]
    ang = np.arctan2(np.einsum("ij,ij->i", vv, e2[gen]), np.einsum("ij,ij->i", vv, e1[gen]))
    order = np.lexsort((ang, gen))
    gen, fac = gen[order], fac[order]
    counts = np.bincount(gen, minlength=n)
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    return Cells(Z, F, V, ptr, fac)


def orient3d_with_bound(a, b, c, d):
    """det(a-d, b-d, c-d) in FP64 and a forward-error bound for it.

    Derivation: each difference is rounded once (relative error u), each of
    the six 2x2 products once, each minor subtraction once, each of the three
    outer products once and the final two additions once; summing the first-
    order terms gives at most 7u times the permanent (the same expression
    with absolute values of the rounded differences).  We use 8u."""
    u = EPS / 2
    ad, bd, cd = a - d, b - d, c - d
    m1 = bd[:, 1] * cd[:, 2] - bd[:, 2] * cd[:, 1]
    m2 = bd[:, 2] * cd[:, 0] - bd[:, 0] * cd[:, 2]
    m3 = bd[:, 0] * cd[:, 1] - bd[:, 1] * cd[:, 0]
    det = ad[:, 0] * m1 + ad[:, 1] * m2 + ad[:, 2] * m3
    p1 = np.abs(bd[:, 1] * cd[:, 2]) + np.abs(bd[:, 2] * cd[:, 1])
    p2 = np.abs(bd[:, 2] * cd[:, 0]) + np.abs(bd[:, 0] * cd[:, 2])
    p3 = np.abs(bd[:, 0] * cd[:, 1]) + np.abs(bd[:, 1] * cd[:, 0])
    perm = np.abs(ad[:, 0]) * p1 + np.abs(ad[:, 1]) * p2 + np.abs(ad[:, 2]) * p3
    return det, 8.0 * u * perm


def delaunay_edges(Z, F):
    """Unique Delaunay edges (i<j) with the two opposite vertices (k, l)."""
    e = np.concatenate([F[:, [0, 1, 2]], F[:, [1, 2, 0]], F[:, [2, 0, 1]]])  # (i,j,opp)
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    key = lo * (len(Z) + 1) + hi
    order = np.argsort(key, kind="stable")
    key, lo, hi, opp = key[order], lo[order], hi[order], e[order, 2]
    # every edge of a closed triangulated sphere is shared by exactly two facets
    assert np.all(key[0::2] == key[1::2]), "hull is not a closed 2-manifold"
    return lo[0::2], hi[0::2], opp[0::2], opp[1::2]


def neighbour_sets(Z, C, flag_scale=8.0):
    """Voronoi neighbours of every generator plus near-degenerate edge flags.

    Returns (i, j, flagged) arrays over unique edges i<j whose dual Voronoi
    edge is an edge of both cells.  An edge is flagged when the four points of
    its two facets are co-circular within the orient3d error bound times
    `flag_scale`, or when the Voronoi edge is shorter than 1e-12 times the
    mean spacing."""
    Z = C.Z
    i, j, k, l = delaunay_edges(Z, C.F)
    det, bound = orient3d_with_bound(Z[i], Z[j], Z[k], Z[l])
    flagged = np.abs(det) <= flag_scale * bound
    # Voronoi edge = segment between the circumcentres of the two facets
    # sharing the Delaunay edge; find them by their sorted index triples.
    N = len(Z) + 1
    S = np.sort(C.F, axis=1)
    fkey = (S[:, 0] * N + S[:, 1]) * N + S[:, 2]
    forder = np.argsort(fkey)
    fsorted = fkey[forder]

    def facet_of(a, b, c):
        T = np.sort(np.stack([a, b, c], axis=1), axis=1)
        q = (T[:, 0] * N + T[:, 1]) * N + T[:, 2]
        pos = np.searchsorted(fsorted, q)
        assert np.all(fsorted[pos] == q)
        return forder[pos]

    t1 = facet_of(i, j, k)
    t2 = facet_of(i, j, l)
    elen = np.linalg.norm(C.V[t1] - C.V[t2], axis=1)
    h = np.sqrt(4 * np.pi / len(Z))
    flagged |= elen < 1e-12 * h
    return i, j, flagged
