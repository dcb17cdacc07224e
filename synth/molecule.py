"""Synthetic globular molecules and their closed surface meshes.

Atoms: a self-avoiding random walk with fixed step length, grown with a bias
toward the origin and then relaxed (bond springs, soft-sphere exclusion for
chain-separated pairs, and a radius-of-gyration restraint) until the radius
of gyration reaches the requested value.

Surface: the isosurface rho(x) = 1 of the sum of Gaussians
    rho(x) = sum_a exp(-beta (|x - r_a|^2 / R_a^2 - 1)),   beta = 1,
so an isolated atom's surface sits at its radius R_a.  It is triangulated by
marching tetrahedra on a regular grid, each crossing kept at least 0.2 of
a grid step from the grid points (bounded triangle shapes) (each cube split into six tetrahedra
around its main diagonal, identically in every cube, which makes the mesh
watertight).  Interior voids are filled before meshing so the result is a
single closed, outward-oriented surface.
"""

import numpy as np
from scipy.spatial import cKDTree
from scipy import ndimage


def saw_molecule(rng, n_atoms, step=1.5, excl=3.0, rg_target=14.0,
                 radius_range=(1.2, 2.0), n_cand=24, relax_iters=400):
    """Return (positions [n,3], radii [n]) of a compact self-avoiding walk."""
    pos = np.zeros((n_atoms, 3))
    bias = 1.0
    for i in range(1, n_atoms):
        best = None
        for attempt in range(4):
            u = rng.normal(size=(n_cand, 3))
            u /= np.linalg.norm(u, axis=1, keepdims=True)
            cand = pos[i - 1] + step * u
            if i >= 3:
                prev = pos[: i - 2]
                d2 = ((cand[:, None, :] - prev[None, :, :]) ** 2).sum(-1)
                viol = np.clip(excl * excl - d2, 0.0, None).sum(1)
            else:
                viol = np.zeros(n_cand)
            score = (cand ** 2).sum(1) * bias + 1e3 * viol \
                + rng.uniform(0, 4.0 * step * step, size=n_cand)
            k = int(np.argmin(score))
            if best is None or score[k] < best[1]:
                best = (cand[k], score[k], viol[k])
            if viol[k] == 0.0:
                break
        pos[i] = best[0]
    pos -= pos.mean(0)
    pos = _relax(pos, step, excl, rg_target, relax_iters)
    radii = rng.uniform(radius_range[0], radius_range[1], size=n_atoms)
    return pos, radii


def _rg(pos):
    c = pos - pos.mean(0)
    return float(np.sqrt((c ** 2).sum(1).mean()))


def _relax(pos, step, excl, rg_target, iters):
    n = len(pos)
    idx = np.arange(n)
    for it in range(iters):
        f = np.zeros_like(pos)
        b = pos[1:] - pos[:-1]
        bl = np.linalg.norm(b, axis=1, keepdims=True)
        fb = (bl - step) * b / np.maximum(bl, 1e-12)
        f[:-1] += fb
        f[1:] -= fb
        pairs = cKDTree(pos).query_pairs(excl, output_type="ndarray")
        if len(pairs):
            pairs = pairs[np.abs(idx[pairs[:, 0]] - idx[pairs[:, 1]]) >= 3]
            dv = pos[pairs[:, 0]] - pos[pairs[:, 1]]
            dl = np.linalg.norm(dv, axis=1, keepdims=True)
            fr = (excl - dl) * dv / np.maximum(dl, 1e-12)
            np.add.at(f, pairs[:, 0], fr)
            np.add.at(f, pairs[:, 1], -fr)
        c = pos.mean(0)
        rg = _rg(pos)
        f -= 0.05 * (1.0 - rg_target / rg) * (pos - c)
        pos = pos + 0.3 * f
    return pos - pos.mean(0)


def _density(pos, radii, origin, h, shape, beta=1.0, cutoff_sigma=3.2):
    rho = np.zeros(shape)
    for p, r in zip(pos, radii):
        ext = r * np.sqrt(1.0 + cutoff_sigma ** 2 / beta)
        lo = np.maximum(np.floor((p - ext - origin) / h).astype(int), 0)
        hi = np.minimum(np.ceil((p + ext - origin) / h).astype(int) + 1,
                        np.array(shape))
        xs = origin[0] + h * np.arange(lo[0], hi[0]) - p[0]
        ys = origin[1] + h * np.arange(lo[1], hi[1]) - p[1]
        zs = origin[2] + h * np.arange(lo[2], hi[2]) - p[2]
        d2 = xs[:, None, None] ** 2 + ys[None, :, None] ** 2 \
            + zs[None, None, :] ** 2
        rho[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += \
            np.exp(-beta * (d2 / (r * r) - 1.0))
    return rho


# Six tetrahedra of the Kuhn (Freudenthal) split of the unit cube: each is the
# path 000 -> (one axis) -> (two axes) -> 111, for the 6 axis orders.
def _kuhn_tets():
    tets = []
    for perm in ([0, 1, 2], [0, 2, 1], [1, 0, 2], [1, 2, 0], [2, 0, 1],
                 [2, 1, 0]):
        c = np.zeros(3, dtype=int)
        path = [c.copy()]
        for ax in perm:
            c[ax] = 1
            path.append(c.copy())
        tets.append(path)
    return np.array(tets)  # [6, 4, 3] corner offsets


def isosurface_mesh(rho, origin, h, iso=1.0):
    """Marching tetrahedra of {rho > iso} -> (verts [Nv,3], tris [N,3]),
    triangles oriented with normals pointing toward lower rho."""
    rho = np.asarray(rho, dtype=np.float64).copy()
    # keep grid values away from the isovalue so no vertex lands on a corner
    close = np.abs(rho - iso) < 1e-9
    rho[close] = iso + 1e-9
    # fill voids: outside = low-density region connected to the box boundary
    low = rho <= iso
    lab, nlab = ndimage.label(low)
    border = np.unique(np.concatenate([
        lab[0].ravel(), lab[-1].ravel(), lab[:, 0].ravel(), lab[:, -1].ravel(),
        lab[:, :, 0].ravel(), lab[:, :, -1].ravel()]))
    outside = np.isin(lab, border[border > 0])
    rho[low & ~outside] = iso + 1.0
    nx, ny, nz = rho.shape
    inside = rho > iso
    tets = _kuhn_tets()
    I, J, K = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1),
                          np.arange(nz - 1), indexing="ij")
    base = np.stack([I.ravel(), J.ravel(), K.ravel()], 1)
    # only cubes that straddle the isosurface
    corners = base[:, None, :] + np.array(
        [[a, b, c] for a in (0, 1) for b in (0, 1) for c in (0, 1)])[None]
    cin = inside[corners[..., 0], corners[..., 1], corners[..., 2]]
    mixed = cin.any(1) & ~cin.all(1)
    base = base[mixed]
    flat = lambda c: (c[..., 0] * ny + c[..., 1]) * nz + c[..., 2]
    tri_edges = []  # list of arrays [n, 3, 2] grid-point index pairs
    tri_dir = []    # inside point and outside point, for orientation
    for t in tets:
        c = base[:, None, :] + t[None]  # [n,4,3]
        gid = flat(c)
        tin = inside[c[..., 0], c[..., 1], c[..., 2]]
        cnt = tin.sum(1)
        for k in (1, 3):
            sel = cnt == k
            if not sel.any():
                continue
            g, ti = gid[sel], tin[sel]
            lone = ti if k == 1 else ~ti  # the single vertex on its own side
            a = np.argmax(lone, axis=1)
            others = np.array([[j for j in range(4) if j != x] for x in range(4)])[a]
            ga = g[np.arange(len(g)), a]
            go = np.take_along_axis(g, others, 1)
            e = np.stack([np.stack([ga, go[:, m]], 1) for m in range(3)], 1)
            tri_edges.append(e)
            ins = ga if k == 1 else go[:, 0]
            out = go[:, 0] if k == 1 else ga
            tri_dir.append(np.stack([ins, out], 1))
        sel = cnt == 2
        if sel.any():
            g, ti = gid[sel], tin[sel]
            order = np.argsort(~ti, axis=1, kind="stable")  # inside first
            gi = np.take_along_axis(g, order, 1)
            p0, p1, q0, q1 = gi[:, 0], gi[:, 1], gi[:, 2], gi[:, 3]
            # quad p0q0, p0q1, p1q1, p1q0 -> two triangles
            e1 = np.stack([np.stack([p0, q0], 1), np.stack([p0, q1], 1),
                           np.stack([p1, q1], 1)], 1)
            e2 = np.stack([np.stack([p0, q0], 1), np.stack([p1, q1], 1),
                           np.stack([p1, q0], 1)], 1)
            tri_edges += [e1, e2]
            d = np.stack([p0, q0], 1)
            tri_dir += [d, d]
    E = np.concatenate(tri_edges)       # [T,3,2]
    D = np.concatenate(tri_dir)         # [T,2]
    lo = np.minimum(E[..., 0], E[..., 1])
    hi = np.maximum(E[..., 0], E[..., 1])
    npts = nx * ny * nz
    key = lo.astype(np.int64) * npts + hi
    ukey, inv = np.unique(key.ravel(), return_inverse=True)
    a, b = ukey // npts, ukey % npts
    unflat = lambda g: np.stack([g // (ny * nz), (g // nz) % ny, g % nz], 1)
    ra, rb = rho.ravel()[a], rho.ravel()[b]
    # the crossing is kept within [0.2, 0.8] of its grid edge: vertices then
    # never crowd a grid point, which would leave slivers of area ~1e-10 A^2
    # and aspect ratios ~1e5; the surface moves by at most 0.2 h along
    # the grid edges and stays closed (every vertex keeps its edge)
    t = np.clip((iso - ra) / (rb - ra), 0.2, 0.8)
    pa = origin + h * unflat(a)
    pb = origin + h * unflat(b)
    verts = pa + t[:, None] * (pb - pa)
    tris = inv.reshape(-1, 3)
    # orientation: normal should point from the inside grid point outward
    v0, v1, v2 = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    n = np.cross(v1 - v0, v2 - v0)
    dirv = (origin + h * unflat(D[:, 1])) - (origin + h * unflat(D[:, 0]))
    flip = np.einsum("ij,ij->i", n, dirv) < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    # drop exactly degenerate triangles only if their removal keeps the mesh
    # closed is not attempted: the isovalue nudge above prevents them.
    return np.ascontiguousarray(verts), np.ascontiguousarray(tris.astype(np.int32))


def molecule_mesh(pos, radii, h, pad=4.0):
    lo = pos.min(0) - radii.max() - pad
    hi = pos.max(0) + radii.max() + pad
    shape = tuple(np.ceil((hi - lo) / h).astype(int) + 1)
    rho = _density(pos, radii, lo, h, shape)
    return isosurface_mesh(rho, lo, h)
