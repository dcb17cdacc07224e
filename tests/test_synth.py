"""Input generators: meshes are closed, consistently oriented and outward,
sites lie inside, distributions have the documented ranges, and every
generator is deterministic for its seed.  CPU only."""

import numpy as np
import pytest

from synth import icosphere, workload, saw_molecule, molecule_mesh, random_multipoles
from synth.sites import sites_in_ball


def _check_closed_outward(v, t):
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    key = e[:, 0].astype(np.int64) * len(v) + e[:, 1]
    rev = e[:, 1].astype(np.int64) * len(v) + e[:, 0]
    assert len(np.unique(key)) == len(key)          # each directed edge once
    assert np.isin(rev, key).all()                   # and its reverse present
    v0, v1, v2 = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    vol = np.einsum("ij,ij->i", v0, np.cross(v1, v2)).sum() / 6
    assert vol > 0
    area = 0.5 * np.linalg.norm(np.cross(v1 - v0, v2 - v0), axis=1)
    assert area.min() > 1e-12
    return vol


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_icosphere(k):
    v, t = icosphere(k, 4.0)
    assert len(t) == 20 * 4 ** k
    assert np.allclose(np.linalg.norm(v, axis=1), 4.0)
    vol = _check_closed_outward(v, t)
    assert vol < 4 / 3 * np.pi * 64


def test_sites_and_multipoles():
    rng = np.random.default_rng(0)
    xyz = sites_in_ball(rng, 8, 2.5, 1.0)
    q, d, Q9, a = random_multipoles(rng, 8)
    assert (np.linalg.norm(xyz, axis=1) < 2.5).all()
    dd = np.linalg.norm(xyz[:, None] - xyz[None], axis=2) + 10 * np.eye(8)
    assert dd.min() >= 1.0
    assert (np.abs(q) <= 0.5).all() and (np.linalg.norm(d, axis=1) <= 0.3).all()
    Q = Q9.reshape(-1, 3, 3)
    assert np.abs(Q - Q.transpose(0, 2, 1)).max() == 0.0
    assert np.abs(np.trace(Q, axis1=1, axis2=2)).max() < 1e-15
    assert ((a >= 0.3) & (a <= 1.5)).all()


def test_determinism():
    w1 = workload("sphere_1280", cache=False)
    w2 = workload("sphere_1280", cache=False)
    for k in ("verts", "tris", "xyz", "q", "d", "Q9", "alpha"):
        assert np.array_equal(w1[k], w2[k])


def test_small_molecule_mesh():
    rng = np.random.default_rng(3)
    pos, rad = saw_molecule(rng, 40, rg_target=5.0)
    v, t = molecule_mesh(pos, rad, 0.8)
    _check_closed_outward(v, t)
    # genus 0: V - E + F = 2
    assert len(v) - 3 * len(t) // 2 + len(t) == 2
    # every atom centre inside: winding number ~ 1
    for p in pos[:5]:
        a, b, c = v[t[:, 0]] - p, v[t[:, 1]] - p, v[t[:, 2]] - p
        na, nb, nc = (np.linalg.norm(u, axis=1) for u in (a, b, c))
        num = np.einsum("ij,ij->i", a, np.cross(b, c))
        den = na * nb * nc + np.einsum("ij,ij->i", a, b) * nc + \
            np.einsum("ij,ij->i", a, c) * nb + np.einsum("ij,ij->i", b, c) * na
        assert abs(2 * np.arctan2(num, den).sum() / (4 * np.pi) - 1) < 1e-9
    rg = np.sqrt(((pos - pos.mean(0)) ** 2).sum(1).mean())
    assert abs(rg - 5.0) < 0.5


def test_globule_recipe():
    """The 1000-atom globule as its workload states it: about 30k panels of a
    closed outward surface, radius of gyration about 14 A, radii in
    [1.2, 2.0] A, every site inside, multipole and polarisability ranges of
    the sphere workloads, treecode theta 0.5 and P 4."""
    w = workload("globule_1000", cache=False)
    assert len(w["xyz"]) == 1000 and 25000 <= len(w["tris"]) <= 35000
    _check_closed_outward(w["verts"], w["tris"])
    x = w["xyz"]
    rg = np.sqrt(((x - x.mean(0)) ** 2).sum(1).mean())
    assert abs(rg - 14.0) < 0.5
    assert w["radii"].min() >= 1.2 and w["radii"].max() <= 2.0
    assert (np.abs(w["q"]) <= 0.5).all() and (np.linalg.norm(w["d"], axis=1) <= 0.3).all()
    assert ((w["alpha"] >= 0.3) & (w["alpha"] <= 1.5)).all()
    p = w["params"]
    assert (p["mode"], p["theta"], int(p["order_P"])) == ("treecode", 0.5, 4)


def test_binding_triad_recipe():
    """The binding triad: the ligand sits at a 3.5 A gap between atom spheres
    from the receptor, the complex's sites are the receptor's followed by the
    ligand's, and the three surfaces have about 90k, 8k and 95k panels."""
    R, L, C = (workload(n, cache=False) for n in ("binding_receptor", "binding_ligand",
                                                   "binding_complex"))
    dd = np.linalg.norm(R["xyz"][:, None, :] - L["xyz"][None], axis=2)
    gap = (dd - R["radii"][:, None] - L["radii"][None, :]).min()
    assert abs(gap - 3.5) < 1e-6
    assert int(C["n_receptor"]) == len(R["xyz"]) == 3000 and len(L["xyz"]) == 200
    assert np.array_equal(C["xyz"], np.concatenate([R["xyz"], L["xyz"]]))
    for w, n in ((R, 90000), (L, 8000), (C, 95000)):
        assert abs(len(w["tris"]) - n) < 0.1 * n
