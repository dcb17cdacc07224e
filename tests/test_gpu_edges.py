"""Edge cases of the path through the C-ABI against the FP64 oracle: no
salt (kappa = 0, Yukawa -> Laplace), the one-node far rule, a single site,
a homogeneous dielectric (no reaction field), the treecode at its order
extremes and with tiny leaves (deep trees), and inputs the library must
refuse."""

import numpy as np
import pytest

from oracle import bie, solver as osolver
from synth import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfg0():
    return workload("sphere_1280")


def _solver(w, **kw):
    from paper_1810_03698_amd import Solver
    args = dict(eps_in=1.0, eps_out=80.0, kappa=0.125, mode="direct", precision="fp64")
    args.update(kw)
    s = Solver(**args)
    s.set_mesh(w["verts"], w["tris"])
    s.set_sites(w["xyz"], w["q"], w["d"], w["Q9"], w["alpha"])
    return s


def test_no_salt_matches_oracle(cfg0):
    w = cfg0
    kw = dict(gmres_tol=1e-13, scf_tol_debye=1e-12)
    got = _solver(w, kappa=0.0, **kw).solve()
    ref = osolver.solvation(w["xyz"], w["q"], w["d"], w["Q9"], w["alpha"],
                            osolver.BemSolvent(w["verts"], w["tris"], 1.0, 80.0, 0.0),
                            tol_debye=1e-12)
    rel = abs(got["dG"] - ref["dG"]) / abs(ref["dG"])
    print("kappa 0", got["dG"], ref["dG"], rel)
    assert rel < 1e-10


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 2e-5)])
def test_one_node_far_rule_matches_oracle(precision, tol, cfg0):
    """The one-node rule puts each panel's node on its own centroid (the
    self pair is the singular integral alone)."""
    w = cfg0
    s = _solver(w, gauss_far=1, precision=precision)
    m = bie.Mesh(w["verts"], w["tris"], 0.125, far=1)
    x = np.random.default_rng(2).normal(size=2 * m.N)
    ref = bie.matvec(m, x, 1.0, 80.0)
    err = np.abs(s.matvec(x) - ref).max() / np.abs(ref).max()
    print(precision, "one-node far rule", err)
    assert err < tol
    if precision == "fp64":
        z = np.random.default_rng(3).normal(size=2 * m.N)
        lhs = z @ s.matvec(x)
        rhs = x @ s.matvec(z, transpose=True)
        assert abs(lhs - rhs) < 1e-12 * np.abs(z).sum() * np.abs(ref).max()


def test_single_site(cfg0):
    w = dict(cfg0)
    for k in ("xyz", "q", "d", "Q9", "alpha"):
        w[k] = cfg0[k][:1]
    got = _solver(w, gmres_tol=1e-13, scf_tol_debye=1e-12).solve()
    ref = osolver.solvation(w["xyz"], w["q"], w["d"], w["Q9"], w["alpha"],
                            osolver.BemSolvent(w["verts"], w["tris"], 1.0, 80.0, 0.125),
                            tol_debye=1e-12)
    print("single site", got["dG"], ref["dG"], got["G_vac"])
    assert abs(got["dG"] - ref["dG"]) < 1e-10 * abs(ref["dG"])
    # one site: no Coulomb partner, so the vacuum energy vanishes
    assert abs(got["G_vac"]) < 1e-12


def test_homogeneous_dielectric(cfg0):
    """eps_out = eps_in without salt: the continuum has no reaction field, so
    the discrete energy is only discretisation error -- small next to the
    water value, and the same as the oracle's."""
    w = cfg0
    big = abs(_solver(w).solve(outputs=False)["dG"])
    got = _solver(w, eps_out=1.0, kappa=0.0, gmres_tol=1e-13,
                  scf_tol_debye=1e-12).solve(outputs=False)["dG"]
    ref = osolver.solvation(w["xyz"], w["q"], w["d"], w["Q9"], w["alpha"],
                            osolver.BemSolvent(w["verts"], w["tris"], 1.0, 1.0, 0.0),
                            tol_debye=1e-12)["dG"]
    print("homogeneous", got, ref, "water", big)
    assert abs(got - ref) < 1e-10 * big
    assert abs(got) < 2e-2 * big


@pytest.mark.parametrize("P,leaf,tol", [(1, 300, 5e-2), (4, 8, 5e-4)])
def test_treecode_extremes(P, leaf, tol):
    """Lowest Taylor order, and leaves of 8 panels (a deep tree)."""
    w = workload("sphere_5120")
    s = _solver(w, mode="treecode", order_P=P, leaf_panels=leaf)
    m = bie.Mesh(w["verts"], w["tris"], 0.125)
    x = np.random.default_rng(4).normal(size=2 * m.N)
    ref = bie.matvec(m, x, 1.0, 80.0)
    err = np.linalg.norm(s.matvec(x) - ref) / np.linalg.norm(ref)
    t = s.tree()
    print("P", P, "leaf", leaf, "error", err, "boxes", len(t["box_level"]),
          "depth", int(t["box_level"].max()))
    assert err < tol


def test_refused_inputs(cfg0):
    from paper_1810_03698_amd import Solver, PbmpError
    w = cfg0
    s = Solver(mode="direct")
    s.set_mesh(w["verts"], w["tris"])
    bad_alpha = -np.abs(w["alpha"])
    with pytest.raises(PbmpError) as e:
        s.set_sites(w["xyz"], w["q"], w["d"], w["Q9"], bad_alpha)
    assert e.value.code == -1
    twin = w["xyz"].copy()
    twin[1] = twin[0]
    with pytest.raises(PbmpError) as e:
        s.set_sites(twin, w["q"], w["d"], w["Q9"], w["alpha"])
    assert e.value.code == -1
    with pytest.raises(PbmpError) as e:
        s.solve()
    assert e.value.code == -6
    tiny = w["verts"].copy()
    t0 = w["tris"][0]
    tiny[t0[1]] = tiny[t0[0]] + 1e-14 * (tiny[t0[1]] - tiny[t0[0]])
    with pytest.raises(PbmpError) as e:
        s.set_mesh(tiny, w["tris"])
    assert e.value.code == -2
    with pytest.raises(PbmpError) as e:
        Solver(order_P=7)
    assert e.value.code == -1
    with pytest.raises(PbmpError) as e:
        s.set_options(gmres_restart=500)
    assert e.value.code == -1
    with pytest.raises(ValueError):
        s.set_options(theta=0.3)
