"""Binding energies of a complex AB from its parts (thermodynamic cycle of
the binding-energy section), three independent solves through the library:
  relative   ddG = dG_solv(AB) - dG_solv(A) - dG_solv(B)   (eq. rel_bind_energy)
  vacuum     dG_bind,vac = G_AB - G_A - G_B                  (eq. bind_vac)
  dissolved  dG_bind,diss = ddG + dG_bind,vac                (eq. bind_energy)
with G the vacuum-state Coulomb energy each solve reports, and the
derivative of ddG with respect to a rigid translation of the ligand B.

Translating B moves B's sites and the part of the complex surface that
belongs to B; the surface of B alone translates as a whole, which leaves
dG_solv(B) unchanged, and A does not move.  Hence
    d ddG / dt = sum_{sites of B in AB} dG_AB/dr + sum_{vertices of AB owned by B} dG_AB/dv.
A complex vertex belongs to the molecule whose atom minimises |v - r_a| - R_a.
"""

import numpy as np

from .pbmp import Solver


def vertex_owner(verts, xyz, radii, is_ligand):
    """True for complex-surface vertices closest (in |v - r| - R) to a ligand
    atom.  Chunked host computation (input preparation)."""
    owner = np.zeros(len(verts), dtype=bool)
    for a in range(0, len(verts), 4096):
        v = verts[a:a + 4096]
        d = np.linalg.norm(v[:, None, :] - xyz[None], axis=2) - radii[None]
        owner[a:a + 4096] = is_ligand[np.argmin(d, axis=1)]
    return owner


def _solve(w, opts, grad):
    s = Solver(**opts)
    s.set_mesh(w["verts"], w["tris"])
    s.set_sites(w["xyz"], w["q"], w["d"], w["Q9"], w["alpha"])
    r = s.solve(outputs=False)
    g = s.backward(1.0, verts=True) if grad else None
    s.close()
    return r, g


def relative_binding(complex_w, receptor_w, ligand_w, n_receptor, grad=True, **opts):
    """Returns dict(ddG, dG_bind_vac, dG_bind_diss, dG_complex, dG_receptor,
    dG_ligand, grad_t [3] or None, per-solve results).  Sites of the complex
    are the receptor's (first n_receptor) followed by the ligand's."""
    rAB, gAB = _solve(complex_w, opts, grad)
    rA, _ = _solve(receptor_w, opts, False)
    rB, _ = _solve(ligand_w, opts, False)
    ddG = rAB["dG"] - rA["dG"] - rB["dG"]
    vac = rAB["G_vac"] - rA["G_vac"] - rB["G_vac"]
    out = dict(ddG=ddG, dG_bind_vac=vac, dG_bind_diss=ddG + vac,
               dG_complex=rAB["dG"], dG_receptor=rA["dG"], dG_ligand=rB["dG"],
               grad_t=None, solves=dict(complex=rAB, receptor=rA, ligand=rB))
    if grad:
        is_lig = np.arange(len(complex_w["q"])) >= n_receptor
        own = vertex_owner(complex_w["verts"], complex_w["xyz"], complex_w["radii"], is_lig)
        out["grad_t"] = gAB["xyz"][is_lig].sum(0) + gAB["verts"][own].sum(0)
        out["ligand_vertices"] = int(own.sum())
    return out
