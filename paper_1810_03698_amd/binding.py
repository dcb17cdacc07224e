"""Binding energies of a complex AB from its parts (thermodynamic cycle of
the binding-energy section) through the library: three solves, then
pbmp_binding_energies (relative, vacuum and dissolved binding energies) and
pbmp_ligand_translation_gradient (derivative of the relative binding energy
with respect to a rigid translation of the ligand).  Argument marshalling
only: the cycle, the vertex ownership and the gradient sums run in the
library."""

from .pbmp import Solver, binding_energies


def _solve(w, opts):
    s = Solver(**opts)
    s.set_mesh(w["verts"], w["tris"])
    s.set_sites(w["xyz"], w["q"], w["d"], w["Q9"], w["alpha"])
    r = s.solve(outputs=False)
    return s, r


def relative_binding(complex_w, receptor_w, ligand_w, n_receptor, grad=True, **opts):
    """Returns dict(ddG, dG_bind_vac, dG_bind_diss, dG_complex, dG_receptor,
    dG_ligand, grad_t [3] or None, ligand_vertices, per-solve results).
    Sites of the complex are the receptor's (first n_receptor) followed by
    the ligand's; complex_w["radii"] holds the sites' atomic radii (vertex
    ownership for the gradient)."""
    sAB, rAB = _solve(complex_w, opts)
    sA, rA = _solve(receptor_w, opts)
    sB, rB = _solve(ligand_w, opts)
    ddG, vac, diss = binding_energies(sAB, sA, sB)
    out = dict(ddG=ddG, dG_bind_vac=vac, dG_bind_diss=diss,
               dG_complex=rAB["dG"], dG_receptor=rA["dG"], dG_ligand=rB["dG"],
               grad_t=None, solves=dict(complex=rAB, receptor=rA, ligand=rB))
    if grad:
        g, nlv, status = sAB.ligand_translation_gradient(n_receptor, complex_w["radii"])
        out.update(grad_t=g, ligand_vertices=nlv, grad_status=status)
    for s in (sAB, sA, sB):
        s.close()
    return out
