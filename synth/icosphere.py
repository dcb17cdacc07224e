"""Icosphere meshes: a regular icosahedron subdivided k times (each triangle
split into four through its edge midpoints) with every vertex projected onto
the sphere.  20 * 4**k triangles, outward (counter-clockwise seen from
outside) orientation."""

import numpy as np
from scipy.spatial import ConvexHull


def _orient_outward(verts, tris):
    v0, v1, v2 = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    n = np.cross(v1 - v0, v2 - v0)
    c = (v0 + v1 + v2) / 3.0
    flip = np.einsum("ij,ij->i", n, c) < 0
    tris = tris.copy()
    tris[flip] = tris[flip][:, [0, 2, 1]]
    return tris


def icosphere(subdiv, radius=4.0, center=(0.0, 0.0, 0.0)):
    """Return (verts float64 [Nv,3], tris int32 [20*4**subdiv, 3])."""
    g = (1.0 + 5.0 ** 0.5) / 2.0
    base = []
    for a in (-1.0, 1.0):
        for b in (-g, g):
            base += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    verts = np.array(base, dtype=np.float64)
    verts /= np.linalg.norm(verts, axis=1, keepdims=True)
    tris = _orient_outward(verts, ConvexHull(verts).simplices.astype(np.int64))
    for _ in range(subdiv):
        nv = len(verts)
        e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
        e.sort(axis=1)
        key = e[:, 0] * nv + e[:, 1]
        ukey, inv = np.unique(key, return_inverse=True)
        a, b = ukey // nv, ukey % nv
        mid = verts[a] + verts[b]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        verts = np.concatenate([verts, mid])
        nt = len(tris)
        m01, m12, m20 = (nv + inv[:nt], nv + inv[nt:2 * nt], nv + inv[2 * nt:])
        t0, t1, t2 = tris[:, 0], tris[:, 1], tris[:, 2]
        tris = np.concatenate([
            np.stack([t0, m01, m20], 1),
            np.stack([t1, m12, m01], 1),
            np.stack([t2, m20, m12], 1),
            np.stack([m01, m12, m20], 1),
        ])
    verts = verts * radius + np.asarray(center, dtype=np.float64)
    return np.ascontiguousarray(verts), np.ascontiguousarray(tris.astype(np.int32))
