"""Adjoint gradients of the solvation energy (pbmp_backward) against
central finite differences of the FP64 CPU oracle, on the 1280-panel sphere
with 8 polarisable sites and on a small irregular molecule.

FD protocol: mesh fixed (site moves do not remesh), oracle with dense LU
and SCF tolerance 1e-12 D, step 1e-4 A for positions and 1e-5 for
multipole entries; quadrupole entries are perturbed along symmetric
directions (Q_ab and Q_ba together) and compared with the matching sum of
the independent-entry gradients.  Bar: 1e-4 relative (to the largest
gradient component of each kind)."""

import numpy as np
import pytest

from oracle import solver as osolver
from synth import workload

pytestmark = pytest.mark.gpu


def _gpu_grad(w, precision="fp64", mode="direct"):
    from paper_1810_03698_amd import Solver
    s = Solver(mode=mode, precision=precision, gmres_tol=1e-13,
               scf_tol_debye=1e-12, scf_maxit=500)
    s.set_mesh(w["verts"], w["tris"])
    s.set_sites(w["xyz"], w["q"], w["d"], w["Q9"], w["alpha"])
    r = s.solve(outputs=False)
    g = s.backward(1.0, verts=False)
    return r, g


def _oracle_fd(w, solvent, params, h):
    """Central differences of the oracle dG for a list of (kind, site,
    index/direction) parameters."""
    base = dict(xyz=w["xyz"].copy(), q=w["q"].copy(), d=w["d"].copy(),
                Q9=w["Q9"].copy())

    def energy(v):
        return osolver.solvation(v["xyz"], v["q"], v["d"], v["Q9"], w["alpha"],
                                 solvent, tol_debye=1e-12, maxit=2000)["dG"]

    out = []
    for kind, l, k in params:
        vals = []
        for sgn in (1.0, -1.0):
            v = {key: val.copy() for key, val in base.items()}
            if kind == "xyz":
                v["xyz"][l, k] += sgn * h
            elif kind == "q":
                v["q"][l] += sgn * h
            elif kind == "d":
                v["d"][l, k] += sgn * h
            else:
                a, b = k
                v["Q9"][l, 3 * a + b] += sgn * h
                if a != b:
                    v["Q9"][l, 3 * b + a] += sgn * h
            vals.append(energy(v))
        out.append((vals[0] - vals[1]) / (2 * h))
    return np.array(out)


def _pick(g, kind, l, k):
    if kind == "xyz":
        return g["xyz"][l, k]
    if kind == "q":
        return g["q"][l]
    if kind == "d":
        return g["d"][l, k]
    a, b = k
    return g["Q9"][l, 3 * a + b] + (g["Q9"][l, 3 * b + a] if a != b else 0.0)


@pytest.fixture(scope="module")
def cfg0():
    return workload("sphere_1280")


@pytest.fixture(scope="module")
def cfg0_solvent(cfg0):
    return osolver.BemSolvent(cfg0["verts"], cfg0["tris"], 1.0, 80.0, 0.125)


@pytest.fixture(scope="module")
def cfg0_grad(cfg0):
    return _gpu_grad(cfg0)


def test_backward_positions_vs_oracle_fd(cfg0, cfg0_solvent, cfg0_grad):
    r, g = cfg0_grad
    params = [("xyz", l, k) for l in range(8) for k in range(3)]
    fd = _oracle_fd(cfg0, cfg0_solvent, params, 1e-4)
    got = np.array([_pick(g, *p) for p in params])
    err = np.abs(got - fd).max() / np.abs(fd).max()
    print("xyz", err, np.c_[got, fd][:6])
    assert err < 1e-4


def test_backward_multipoles_vs_oracle_fd(cfg0, cfg0_solvent, cfg0_grad):
    r, g = cfg0_grad
    for kind, params in (
            ("q", [("q", l, 0) for l in range(8)]),
            ("d", [("d", l, k) for l in range(8) for k in range(3)]),
            ("Q", [("Q", l, (a, b)) for l in (0, 5) for a in range(3)
                   for b in range(a, 3)])):
        fd = _oracle_fd(cfg0, cfg0_solvent, params, 1e-5)
        got = np.array([_pick(g, *p) for p in params])
        err = np.abs(got - fd).max() / np.abs(fd).max()
        print(kind, err)
        assert err < 1e-4, kind


def test_backward_homogeneous_medium_is_flat(cfg0_grad):
    """eps_out = eps_in and kappa = 0: there is no reaction field, the
    dissolved and vacuum states coincide, dG = 0 and so is its gradient, up
    to the discretisation error of the surface."""
    from paper_1810_03698_amd import Solver
    w = workload("sphere_1280")
    s = Solver(mode="direct", precision="fp64", eps_out=1.0, kappa=0.0,
               gmres_tol=1e-13, scf_tol_debye=1e-12)
    s.set_mesh(w["verts"], w["tris"])
    s.set_sites(w["xyz"], w["q"], w["d"], w["Q9"], w["alpha"])
    r = s.solve(outputs=False)
    g = s.backward(1.0, verts=False)
    # the homogeneous medium leaves only the discretisation error
    assert abs(r["dG"]) < 5e-3 * 21.0
    gmax = max(np.abs(g[k]).max() for k in ("xyz", "q", "d", "Q9"))
    assert gmax < 0.1


def test_backward_mixed_matches_fp64(cfg0, cfg0_grad):
    r64, g64 = cfg0_grad
    rmx, gmx = _gpu_grad(cfg0, precision="mixed")
    for k in ("xyz", "q", "d", "Q9"):
        err = np.abs(gmx[k] - g64[k]).max() / np.abs(g64[k]).max()
        print(k, err)
        assert err < 1e-4, k


def test_backward_mixed_adjoint_of_fp64_state(cfg0, cfg0_grad):
    """An FP64 solve differentiated with mixed-precision adjoint solves (the
    precision switched between solve and backward): the FP64 refinement of
    the transposed solves keeps the gradient at FP64 quality.  Switching
    back to FP64 reproduces the FP64 solve exactly."""
    from paper_1810_03698_amd import Solver
    r64, g64 = cfg0_grad
    s = Solver(mode="direct", precision="fp64", gmres_tol=1e-13, scf_tol_debye=1e-12,
               scf_maxit=500)
    s.set_mesh(cfg0["verts"], cfg0["tris"])
    s.set_sites(cfg0["xyz"], cfg0["q"], cfg0["d"], cfg0["Q9"], cfg0["alpha"])
    r = s.solve(outputs=False)
    assert r["dG"] == r64["dG"]
    s.set_options(precision="mixed", gmres_tol=1e-12)
    g = s.backward(1.0, verts=False)
    for k in ("xyz", "q", "d", "Q9"):
        err = np.abs(g[k] - g64[k]).max() / np.abs(g64[k]).max()
        print("mixed adjoint of the fp64 state", k, err)
        assert err < 1e-9, k
    s.set_options(precision="fp64", gmres_tol=1e-13)
    assert s.solve(outputs=False)["dG"] == r64["dG"]


def test_backward_warm_start(cfg0, cfg0_grad):
    """A warm-started backward (multipliers of the previous call, rescaled
    to the new dG_bar) gives the cold gradient."""
    from paper_1810_03698_amd import Solver
    r64, g64 = cfg0_grad
    s = Solver(mode="direct", precision="fp64", gmres_tol=1e-13, scf_tol_debye=1e-12,
               scf_maxit=500, warm_start=True)
    s.set_mesh(cfg0["verts"], cfg0["tris"])
    s.set_sites(cfg0["xyz"], cfg0["q"], cfg0["d"], cfg0["Q9"], cfg0["alpha"])
    s.solve(outputs=False)
    s.backward(1.0, verts=False)
    g = s.backward(2.0, verts=False)
    for k in ("xyz", "q", "d", "Q9"):
        err = np.abs(g[k] - 2.0 * g64[k]).max() / np.abs(2.0 * g64[k]).max()
        print("warm backward", k, err)
        assert err < 1e-10, k


def test_backward_ragged_positions_fd():
    from tests.test_gpu_direct import _ragged
    w = _ragged()
    r, g = _gpu_grad(w)
    solvent = osolver.BemSolvent(w["verts"], w["tris"], 1.0, 80.0, 0.125)
    rng = np.random.default_rng(4)
    sites = rng.choice(len(w["q"]), 4, replace=False)
    params = [("xyz", int(l), k) for l in sites for k in range(3)] + \
             [("d", int(l), 1) for l in sites] + [("q", int(l), 0) for l in sites]
    fd = _oracle_fd(w, solvent, params, 1e-4)
    got = np.array([_pick(g, *p) for p in params])
    err = np.abs(got - fd).max() / np.abs(fd).max()
    print("ragged", err)
    assert err < 1e-4


def _gpu_grad_verts(w, precision="fp64"):
    from paper_1810_03698_amd import Solver
    s = Solver(mode="direct", precision=precision, gmres_tol=1e-13,
               scf_tol_debye=1e-12, scf_maxit=500)
    s.set_mesh(w["verts"], w["tris"])
    s.set_sites(w["xyz"], w["q"], w["d"], w["Q9"], w["alpha"])
    s.solve(outputs=False)
    return s.backward(1.0, verts=True)


@pytest.fixture(scope="module")
def cfg0_grad_verts(cfg0):
    return _gpu_grad_verts(cfg0)


def test_backward_vertices_vs_oracle_fd(cfg0, cfg0_grad_verts):
    """Vertex moves of 1e-5 A keep every near/far decision (smallest margin
    to the threshold on this mesh: 0.025 A)."""
    g = cfg0_grad_verts
    rng = np.random.default_rng(9)
    vids = rng.choice(len(cfg0["verts"]), 4, replace=False)
    h = 1e-5
    got, fd = [], []
    for v in vids:
        for k in range(3):
            vals = []
            for sgn in (1.0, -1.0):
                vv = cfg0["verts"].copy()
                vv[v, k] += sgn * h
                sol = osolver.BemSolvent(vv, cfg0["tris"], 1.0, 80.0, 0.125)
                vals.append(osolver.solvation(cfg0["xyz"], cfg0["q"], cfg0["d"],
                                              cfg0["Q9"], cfg0["alpha"], sol,
                                              tol_debye=1e-12, maxit=2000)["dG"])
            fd.append((vals[0] - vals[1]) / (2 * h))
            got.append(g["verts"][v, k])
    got, fd = np.array(got), np.array(fd)
    err = np.abs(got - fd).max() / np.abs(fd).max()
    print("verts", err, np.c_[got, fd][:6])
    assert err < 1e-4


def test_backward_rigid_translation_invariance(cfg0_grad_verts):
    """Moving every site and every vertex by the same vector changes
    nothing: the site and vertex gradients sum to zero."""
    g = cfg0_grad_verts
    tot = g["xyz"].sum(0) + g["verts"].sum(0)
    scale = np.abs(g["xyz"]).sum() + np.abs(g["verts"]).sum()
    print(tot, scale)
    assert np.abs(tot).max() < 1e-9 * scale


def test_autograd_function_matches_backward(cfg0, cfg0_grad_verts):
    import torch
    from paper_1810_03698_amd import solvation_energy
    dev = torch.device("cuda:0")
    t = lambda a, req=False: torch.tensor(a, dtype=torch.float64, device=dev,
                                          requires_grad=req)
    verts, xyz, q, d, Q9 = (t(cfg0[k], True) for k in ("verts", "xyz", "q", "d", "Q9"))
    tris = torch.tensor(cfg0["tris"], dtype=torch.int32, device=dev)
    alpha = t(cfg0["alpha"])
    dG = solvation_energy(verts, tris, xyz, q, d, Q9, alpha, mode="direct",
                          precision="fp64", gmres_tol=1e-13, scf_tol_debye=1e-12,
                          scf_maxit=500)
    (2.0 * dG).backward()
    g = cfg0_grad_verts
    for name, tens in (("xyz", xyz), ("q", q), ("d", d), ("Q9", Q9), ("verts", verts)):
        ref = 2.0 * g[name].reshape(tens.shape)
        got = tens.grad.cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max(), name
