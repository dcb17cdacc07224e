"""Binding energies from the thermodynamic cycle (binding-energy section)
on a small synthetic triad -- a receptor, a ligand at a 3.5 A surface gap
and the complex meshed from the union density -- through the library
against the FP64 oracle: relative (eq. rel_bind_energy), vacuum (eq.
bind_vac) and dissolved (eq. bind_energy) binding energies to 1e-10, and
the gradient of the relative binding energy with respect to a rigid
translation of the ligand against central differences of the library's
own FP64 solves (topology fixed, ligand-owned complex vertices moved)."""

import numpy as np
import pytest

from oracle import solver as osolver
from synth import saw_molecule, molecule_mesh, random_multipoles

pytestmark = pytest.mark.gpu

OPTS = dict(mode="direct", precision="fp64", gmres_tol=1e-13, scf_tol_debye=1e-11,
            scf_maxit=500)


def _triad():
    rngR, rngL, rngP = (np.random.default_rng([11, k]) for k in range(3))
    posR, radR = saw_molecule(rngR, 24, rg_target=4.0)
    mR = random_multipoles(rngR, 24)
    posL, radL = saw_molecule(rngL, 7, rg_target=2.0)
    mL = random_multipoles(rngL, 7)
    u = rngP.normal(size=3)
    u /= np.linalg.norm(u)

    def gap(t):
        dd = np.linalg.norm(posR[:, None, :] - (posL[None] + t * u), axis=2)
        return float((dd - radR[:, None] - radL[None, :]).min())

    lo, hi = 0.0, 60.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if gap(mid) < 3.5 else (lo, mid)
    posL = posL + hi * u
    h = 1.1

    def part(pos, rad, m):
        # 1e-3 A jitter: no centroid distance sits exactly on the near-field
        # threshold (the mesher's grid-aligned panels are congruent)
        v, t = molecule_mesh(pos, rad, h)
        v = v + np.random.default_rng([12, len(t)]).normal(scale=1e-3, size=v.shape)
        q, d, Q9, al = m
        return dict(verts=v, tris=t, xyz=pos, q=q, d=d, Q9=Q9, alpha=al, radii=rad)

    A = part(posR, radR, mR)
    B = part(posL, radL, mL)
    AB = part(np.concatenate([posR, posL]), np.concatenate([radR, radL]),
              tuple(np.concatenate([a, b]) for a, b in zip(mR, mL)))
    return A, B, AB


@pytest.fixture(scope="module")
def triad():
    return _triad()


def _oracle(w):
    return osolver.solvation(w["xyz"], w["q"], w["d"], w["Q9"], w["alpha"],
                             osolver.BemSolvent(w["verts"], w["tris"], 1.0, 80.0, 0.125),
                             tol_debye=1e-11)


def test_binding_energies_match_oracle(triad):
    from paper_1810_03698_amd.binding import relative_binding
    A, B, AB = triad
    print("panels", len(A["tris"]), len(B["tris"]), len(AB["tris"]), flush=True)
    got = relative_binding(AB, A, B, n_receptor=len(A["q"]), grad=False, **OPTS)
    rA, rB, rAB = _oracle(A), _oracle(B), _oracle(AB)
    ddG = rAB["dG"] - rA["dG"] - rB["dG"]
    vac = rAB["G_vac"] - rA["G_vac"] - rB["G_vac"]
    print("ddG", got["ddG"], ddG, "vac", got["dG_bind_vac"], vac)
    scale = max(abs(rAB["dG"]), abs(rAB["G_vac"]))
    assert abs(got["ddG"] - ddG) < 1e-10 * scale
    assert abs(got["dG_bind_vac"] - vac) < 1e-10 * scale
    assert abs(got["dG_bind_diss"] - (ddG + vac)) < 2e-10 * scale


def _vertex_owner(verts, xyz, radii, is_ligand):
    """Test-side statement of which complex vertices move with the ligand:
    those whose closest atom sphere (smallest |v - r_a| - R_a) is a ligand
    atom."""
    d = np.linalg.norm(verts[:, None, :] - xyz[None], axis=2) - radii[None]
    return is_ligand[np.argmin(d, axis=1)]


def test_binding_translation_gradient_fd(triad):
    from paper_1810_03698_amd import Solver
    from paper_1810_03698_amd.binding import relative_binding
    A, B, AB = triad
    nR = len(A["q"])
    got = relative_binding(AB, A, B, n_receptor=nR, grad=True, **OPTS)
    is_lig = np.arange(len(AB["q"])) >= nR
    own = _vertex_owner(AB["verts"], AB["xyz"], AB["radii"], is_lig)
    assert got["ligand_vertices"] == int(own.sum())

    def dG_complex(t):
        v = AB["verts"].copy()
        v[own] += t
        x = AB["xyz"].copy()
        x[is_lig] += t
        s = Solver(**OPTS)
        s.set_mesh(v, AB["tris"])
        s.set_sites(x, AB["q"], AB["d"], AB["Q9"], AB["alpha"])
        r = s.solve(outputs=False)["dG"]
        s.close()
        return r

    h = 1e-4
    fd = np.empty(3)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd[a] = (dG_complex(e) - dG_complex(-e)) / (2 * h)
    print("grad_t", got["grad_t"], "fd", fd, "ligand vertices", got["ligand_vertices"])
    assert np.abs(got["grad_t"] - fd).max() < 1e-4 * max(np.abs(fd).max(), 1e-3)


def test_binding_translation_gradient_vs_oracle_fd(triad):
    """The library's ligand-translation gradient (direct mode, FP64 adjoint)
    against central differences of the FP64 oracle's solvation energies of
    the displaced complex (dense LU, SCF 1e-11 D; h = 5e-4 A along each
    axis, the ligand's sites and the complex vertices it owns moved, the
    receptor's and ligand's own energies being translation invariant):
    relative 1e-4 of the largest component."""
    from paper_1810_03698_amd.binding import relative_binding
    A, B, AB = triad
    nR = len(A["q"])
    got = relative_binding(AB, A, B, n_receptor=nR, grad=True, **OPTS)
    is_lig = np.arange(len(AB["q"])) >= nR
    own = _vertex_owner(AB["verts"], AB["xyz"], AB["radii"], is_lig)
    h = 5e-4
    fd = np.empty(3)
    for a in range(3):
        e = []
        for sg in (1.0, -1.0):
            w = dict(AB)
            w["verts"] = AB["verts"].copy()
            w["verts"][own, a] += sg * h
            w["xyz"] = AB["xyz"].copy()
            w["xyz"][is_lig, a] += sg * h
            e.append(_oracle(w)["dG"])
        fd[a] = (e[0] - e[1]) / (2 * h)
    err = np.abs(got["grad_t"] - fd).max() / np.abs(fd).max()
    print("grad_t", got["grad_t"], "oracle fd", fd, "err", err)
    assert err < 1e-4


def test_binding_translation_gradient_treecode_converges(triad):
    """The treecode's translation gradient (adjoint with the treecode's
    transposed product and vertex terms) against the direct-mode one on the
    same triad, as the order grows (theta 0.5, leaf 16): the sum over the
    ligand's sites and vertices cancels strongly, so its relative error
    sits far above the energy's (measured 1.6e-2, 8.3e-3, 1.3e-3, 9.6e-4 of
    the gradient's norm at P 3 to 6, energies 1.6e-4 to 5e-7; at theta 0.3
    and P 6, 1.8e-5); bars: below 2.5e-2 at P 3, falling by more than 5x
    from P 3 to P 5, below 2e-3 at P 6, below 1e-4 at theta 0.3 and P 6."""
    from paper_1810_03698_amd import Solver
    A, B, AB = triad
    nR = len(A["q"])

    def grad(**kw):
        # GMRES 1e-11 / SCF 1e-9 D: far below the differences measured here
        s = Solver(**dict(OPTS, gmres_tol=1e-11, scf_tol_debye=1e-9, **kw))
        s.set_mesh(AB["verts"], AB["tris"])
        s.set_sites(AB["xyz"], AB["q"], AB["d"], AB["Q9"], AB["alpha"])
        s.solve(outputs=False)
        g, _, st = s.ligand_translation_gradient(nR, AB["radii"])
        s.close()
        assert st == 0
        return np.asarray(g)

    gd = grad()
    err = {}
    for theta, P in ((0.5, 3), (0.5, 5), (0.5, 6), (0.3, 6)):
        g = grad(mode="treecode", theta=theta, order_P=P, leaf_panels=16)
        err[theta, P] = np.abs(g - gd).max() / np.linalg.norm(gd)
        print("theta", theta, "P", P, "translation gradient", g, "direct", gd,
              "err/|g|", err[theta, P])
    assert err[0.5, 3] < 2.5e-2 and err[0.5, 5] < err[0.5, 3] / 5
    assert err[0.5, 6] < 2e-3 and err[0.3, 6] < 1e-4
