"""Panel geometry for flat triangles (test infrastructure only).

Collocation point = centroid; unit normal n = (v1-v0)x(v2-v0)/|.| (outward
for counter-clockwise triangles seen from the solvent); area
A = |(v1-v0)x(v2-v0)|/2 (Algorithmic details, "boundary element method").
"""

import numpy as np


def panels(verts, tris):
    v = np.asarray(verts, dtype=np.float64)
    t = np.asarray(tris, dtype=np.int64)
    v0, v1, v2 = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    cr = np.cross(v1 - v0, v2 - v0)
    nn = np.linalg.norm(cr, axis=1)
    return dict(centroid=(v0 + v1 + v2) / 3.0, normal=cr / nn[:, None],
                area=0.5 * nn, v0=v0, v1=v1, v2=v2)


def quad_points(geo, bary):
    """Physical quadrature points [N, nq, 3] for barycentric nodes [nq, 3]."""
    b = np.asarray(bary)
    return (b[None, :, 0, None] * geo["v0"][:, None, :]
            + b[None, :, 1, None] * geo["v1"][:, None, :]
            + b[None, :, 2, None] * geo["v2"][:, None, :])
