"""A structure read from files (an MSMS surface, Tinker coordinates and
multipole/polarize records) solves to the same energy as the arrays the
readers return, and to the FP64 oracle's: the ingestion path end to end on
the device.  The files are written here from a small synthetic molecule."""

import numpy as np
import pytest

from oracle import solver as osolver
from paper_1810_03698_amd import ingest
from synth import saw_molecule, molecule_mesh

pytestmark = pytest.mark.gpu


def _write_structure(tmp_path):
    rng = np.random.default_rng(41)
    pos, rad = saw_molecule(rng, 9, rg_target=2.5)
    verts, tris = molecule_mesh(pos, rad, 1.0)
    verts = verts + np.random.default_rng(42).normal(scale=1e-3, size=verts.shape)
    vp, fp = tmp_path / "mol.vert", tmp_path / "mol.face"
    ingest.write_msms(vp, fp, verts, tris)
    # a chain: atom i bonded to i-1 and i+1; types alternate between two
    # z-then-x frames along the chain (ends take a z-only frame; the atoms
    # next to the ends find their x atom through a second record)
    n = len(pos)
    lines = ["%6d  chain" % n]
    for a in range(n):
        nb = [b + 1 for b in (a - 1, a + 1) if 0 <= b < n]
        t = 1 if a in (0, n - 1) else 2 + a % 2
        lines.append("%6d  C  %12.6f %12.6f %12.6f %5d %s" % (
            a + 1, *pos[a], t, " ".join("%5d" % b for b in nb)))
    xp = tmp_path / "mol.xyz"
    xp.write_text("\n".join(lines) + "\n")
    prm = """
multipole     1    2                    0.20000
                                        0.00000    0.00000    0.10000
                                        0.05000
                                        0.00000    0.05000
                                        0.00000    0.00000   -0.10000
multipole     1    3                    0.20000
                                        0.00000    0.00000    0.10000
                                        0.05000
                                        0.00000    0.05000
                                        0.00000    0.00000   -0.10000
multipole     2    3    3              -0.10000
                                        0.05000    0.00000    0.08000
                                        0.10000
                                        0.00000   -0.04000
                                        0.02000    0.00000   -0.06000
multipole     3    2    2              -0.05000
                                       -0.03000    0.00000    0.06000
                                       -0.02000
                                        0.00000    0.07000
                                        0.01000    0.00000   -0.05000
multipole     3    2    1              -0.05000
                                       -0.03000    0.00000    0.06000
                                       -0.02000
                                        0.00000    0.07000
                                        0.01000    0.00000   -0.05000
polarize      1     1.3340     0.3900
polarize      2     1.0730     0.3900
polarize      3     0.8370     0.3900
"""
    pp = tmp_path / "mol.prm"
    pp.write_text(prm)
    return vp, fp, xp, pp


def test_structure_from_files_matches_arrays_and_oracle(tmp_path):
    from paper_1810_03698_amd import Solver
    vp, fp, xp, pp = _write_structure(tmp_path)
    opts = dict(mode="direct", precision="fp64", gmres_tol=1e-13, scf_tol_debye=1e-11,
                scf_maxit=500)
    got = ingest.solve_files(vp, fp, xp, pp, **opts)
    verts, tris, _, flipped = ingest.read_msms(vp, fp)
    sites = ingest.load_tinker(xp, pp)
    s = Solver(**opts)
    s.set_mesh(verts, tris)
    s.set_sites(sites["xyz"], sites["q"], sites["d"], sites["Q9"], sites["alpha"],
                group=sites["group"])
    ref_arrays = s.solve(outputs=False)["dG"]
    ref = osolver.solvation(sites["xyz"], sites["q"], sites["d"], sites["Q9"], sites["alpha"],
                            osolver.BemSolvent(verts, tris, 1.0, 80.0, 0.125),
                            group=sites["group"], tol_debye=1e-11)["dG"]
    print("from files", got["dG"], "arrays", ref_arrays, "oracle", ref, "flipped", flipped)
    assert got["status"] == 0
    assert got["dG"] == ref_arrays
    assert abs(got["dG"] - ref) < 1e-10 * abs(ref)
