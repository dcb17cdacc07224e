"""Named synthetic workloads, shaped like the paper's test cases.

  sphere_<N>     icosphere of radius 4 A with N = 1280 / 5120 / 20480 / 81920
                 triangles, holding the same 8 polarisable multipole sites
                 (seed 0) uniform within 2.5 A of the centre.
  globule_1000   1000-atom compact self-avoiding walk, radius of gyration
                 ~14 A, radii U[1.2, 2.0] A, isosurface mesh of ~30k
                 triangles (seed 2).  Size class of a small protein.
  globule_5000   same recipe, 5000 atoms, R_g ~24 A, ~150k triangles (seed 3).
  binding_*      receptor (3000 atoms, ~90k triangles), ligand (200 atoms,
                 ~8k triangles) placed at a 3.5 A surface gap along a seeded
                 direction, and the complex meshed from the union density
                 (seed 4).

Each workload is a dict with verts, tris, xyz, q, d, Q9, alpha and the
solver parameters the case is defined with.  Results are cached as .npz
under ``.synth_cache/`` at the repository root (or ``$SYNTH_CACHE``).
"""

import os
import numpy as np

from .icosphere import icosphere
from .sites import random_multipoles, sites_in_ball
from .molecule import saw_molecule, molecule_mesh

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CACHE = os.environ.get("SYNTH_CACHE", os.path.join(_ROOT, ".synth_cache"))

BASE_PARAMS = dict(eps_in=1.0, eps_out=80.0, kappa=0.125, thole_a=0.39,
                   near_eta=2.0, gauss_far=3, gmres_restart=50,
                   gmres_tol=1e-6, scf_tol_debye=1e-6, scf_omega=0.7)


def _sphere(n_tri):
    level = {1280: 3, 5120: 4, 20480: 5, 81920: 6}[n_tri]
    verts, tris = icosphere(level, radius=4.0)
    rng = np.random.default_rng(0)
    xyz = sites_in_ball(rng, 8, radius=2.5, min_sep=1.0)
    q, d, Q9, alpha = random_multipoles(rng, 8)
    params = dict(BASE_PARAMS)
    params["mode"] = "direct" if n_tri < 20000 else "treecode"
    params.update(theta=0.5, order_P=4, leaf_panels=300)
    return dict(verts=verts, tris=tris, xyz=xyz, q=q, d=d, Q9=Q9,
                alpha=alpha, params=params)


def _calibrated_mesh(pos, radii, n_target, h0=1.0, rounds=3):
    h = h0
    verts = tris = None
    for _ in range(rounds):
        verts, tris = molecule_mesh(pos, radii, h)
        ratio = len(tris) / float(n_target)
        if abs(ratio - 1.0) < 0.04:
            break
        h *= np.sqrt(ratio)
    return verts, tris, h


def _globule(n_atoms, rg, n_tri, seed, order_P):
    rng = np.random.default_rng(seed)
    pos, radii = saw_molecule(rng, n_atoms, rg_target=rg)
    q, d, Q9, alpha = random_multipoles(rng, n_atoms)
    verts, tris, h = _calibrated_mesh(pos, radii, n_tri)
    params = dict(BASE_PARAMS)
    # GMRES(200) on molecular surfaces: restarts at 50 stagnate on their
    # crevices (4x more iterations on the 5000-atom globule), and the
    # basis of the largest one is 233 MB
    params.update(mode="treecode", theta=0.5, order_P=order_P,
                  leaf_panels=300, grid_h=h, gmres_restart=200)
    return dict(verts=verts, tris=tris, xyz=pos, q=q, d=d, Q9=Q9,
                alpha=alpha, radii=radii, params=params)


def _binding(part):
    rngR = np.random.default_rng([4, 0])
    rngL = np.random.default_rng([4, 1])
    rngP = np.random.default_rng([4, 2])
    posR, radR = saw_molecule(rngR, 3000, rg_target=20.2)
    mR = random_multipoles(rngR, 3000)
    posL, radL = saw_molecule(rngL, 200, rg_target=8.2)
    mL = random_multipoles(rngL, 200)
    u = rngP.normal(size=3)
    u /= np.linalg.norm(u)

    def gap(t):
        dd = np.linalg.norm(posR[:, None, :] - (posL[None] + t * u), axis=2)
        return float((dd - radR[:, None] - radL[None, :]).min())

    lo, hi = 0.0, 200.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if gap(mid) < 3.5:
            lo = mid
        else:
            hi = mid
    posL = posL + hi * u
    params = dict(BASE_PARAMS)
    params.update(mode="treecode", theta=0.5, order_P=4, leaf_panels=300, gmres_restart=200)
    if part == "receptor":
        pos, rad, m, n_tri = posR, radR, mR, 90000
    elif part == "ligand":
        pos, rad, m, n_tri = posL, radL, mL, 8000
    else:
        pos = np.concatenate([posR, posL])
        rad = np.concatenate([radR, radL])
        m = tuple(np.concatenate([a, b]) for a, b in zip(mR, mL))
        n_tri = 95000
    verts, tris, h = _calibrated_mesh(pos, rad, n_tri)
    params["grid_h"] = h
    q, d, Q9, alpha = m
    return dict(verts=verts, tris=tris, xyz=pos, q=q, d=d, Q9=Q9,
                alpha=alpha, radii=rad, params=params,
                ligand_shift=hi * u, n_receptor=3000)


WORKLOADS = {
    "sphere_1280": lambda: _sphere(1280),
    "sphere_5120": lambda: _sphere(5120),
    "sphere_20480": lambda: _sphere(20480),
    "sphere_81920": lambda: _sphere(81920),
    "globule_1000": lambda: _globule(1000, 14.0, 30000, 2, 4),
    "globule_5000": lambda: _globule(5000, 24.0, 150000, 3, 5),
    "binding_receptor": lambda: _binding("receptor"),
    "binding_ligand": lambda: _binding("ligand"),
    "binding_complex": lambda: _binding("complex"),
}


def workload(name, cache=True):
    """Return the named workload (see module docstring)."""
    path = os.path.join(CACHE, name + "_v3.npz")
    if cache and os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        out = {k: z[k] for k in z.files if k != "params_keys"}
        keys = list(z["params_keys"])
        vals = out.pop("params_vals")
        params = {}
        for k, v in zip(keys, vals):
            params[str(k)] = v
        for k in ("mode",):
            params[k] = str(out.pop("mode"))
        for k in ("gauss_far", "gmres_restart", "order_P", "leaf_panels"):
            if k in params:
                params[k] = int(params[k])
        for k in list(params):
            if isinstance(params[k], np.floating):
                params[k] = float(params[k])
        out["params"] = params
        return out
    w = WORKLOADS[name]()
    if cache:
        os.makedirs(CACHE, exist_ok=True)
        p = dict(w["params"])
        mode = p.pop("mode")
        keys = sorted(p)
        arrs = {k: v for k, v in w.items() if k != "params"}
        np.savez(path + ".tmp.npz", params_keys=np.array(keys),
                 params_vals=np.array([float(p[k]) for k in keys]),
                 mode=np.array(mode), **arrs)
        os.replace(path + ".tmp.npz", path)
    return w
