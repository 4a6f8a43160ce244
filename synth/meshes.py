"""Closed triangle meshes with exact vertex counts.

All meshes are returned as ``xyz`` float32 ``[3][N]`` (structure-of-arrays)
and ``tri`` int32 ``[3][F]`` with counter-clockwise winding seen from outside,
so that ``(v1 - v0) x (v2 - v0)`` is an outward normal.
"""
import numpy as np
from scipy.spatial import ConvexHull


def _orient_outward(pts, tri):
    """Flip triangles whose normal points towards the centroid (convex input)."""
    c = pts.mean(axis=0)
    v0, v1, v2 = pts[tri[:, 0]], pts[tri[:, 1]], pts[tri[:, 2]]
    n = np.cross(v1 - v0, v2 - v0)
    flip = np.einsum("ij,ij->i", n, v0 - c) < 0
    tri = tri.copy()
    tri[flip, 1], tri[flip, 2] = tri[flip, 2].copy(), tri[flip, 1].copy()
    return tri


def icosphere(level):
    """Unit icosphere: 10*4**level + 2 vertices, 20*4**level faces (float64)."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
             (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
             (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in verts]
    for _ in range(level):
        cache = {}
        new_faces = []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    pts = np.array(verts)
    tri = _orient_outward(pts, np.array(faces, dtype=np.int64))
    return pts, tri


def _to_soa(pts, tri):
    return (np.ascontiguousarray(pts.T.astype(np.float32)),
            np.ascontiguousarray(tri.T.astype(np.int32)))


def ellipsoid_icosphere(level, semi_axes, centre):
    """Icosphere scaled to an ellipsoid with the given semi-axes and centre."""
    pts, tri = icosphere(level)
    pts = pts * np.asarray(semi_axes, dtype=np.float64) + np.asarray(centre, dtype=np.float64)
    return _to_soa(pts, tri)


def fibonacci_ellipsoid(n_vertices, semi_axes, centre):
    """Ellipsoid meshed with exactly ``n_vertices`` vertices.

    Points lie on a Fibonacci spiral over the unit sphere (near-uniform
    density); their convex hull gives a closed triangulation with
    2N - 4 faces, which is then scaled to the ellipsoid.
    """
    n = int(n_vertices)
    i = np.arange(n, dtype=np.float64) + 0.5
    phi = np.arccos(1.0 - 2.0 * i / n)
    golden = np.pi * (3.0 - 5.0 ** 0.5)
    theta = golden * i
    pts = np.stack([np.sin(phi) * np.cos(theta), np.cos(phi), np.sin(phi) * np.sin(theta)], axis=1)
    hull = ConvexHull(pts)
    tri = _orient_outward(pts, hull.simplices.astype(np.int64))
    pts = pts * np.asarray(semi_axes, dtype=np.float64) + np.asarray(centre, dtype=np.float64)
    return _to_soa(pts, tri)
