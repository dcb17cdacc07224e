"""The GPU path at the full workload sizes, in the configuration the
benchmark times (mixed precision, each workload's own mode, theta, order and
leaf size), through the C-ABI.

The FP64 oracle cannot run a whole product at these sizes, so it evaluates
sampled rows one at a time: operator-product rows, right-hand-side entries
and site fields.  Whole-solve results are checked through properties that
hold at any size: the mixed path against the FP64 path of the same method
(relative 1e-4 on the energy), and the treecode energy against the direct
sum (relative 1e-5 at P = 5, 2e-5 at P = 4 -- the treecode's own accuracy,
measured against the oracle on the smaller cases).

Bars on sampled rows (max-norm error over the sample divided by the
sample's max-norm): direct mixed 2e-5 (FP32 far field); treecode 1e-3 at
P = 4 and 5e-4 at P = 5 (its 2-norm error is 2-4e-4 at P = 4 on the
5120-panel sphere against the full oracle product; a max-norm over a
sample sits above that)."""

import numpy as np
import pytest

from oracle import bie, multipoles as mp
from synth import workload

pytestmark = pytest.mark.gpu

FULL = ["sphere_81920", "globule_1000", "globule_5000", "binding_complex"]
ROWS = 40
SITES = 24


def _solver(w, precision="mixed", mode=None, **kw):
    from paper_1810_03698_amd import Solver
    p = w["params"]
    args = dict(eps_in=p["eps_in"], eps_out=p["eps_out"], kappa=p["kappa"],
                gauss_far=int(p["gauss_far"]), near_eta=p["near_eta"],
                mode=mode or p["mode"], theta=p.get("theta", 0.5),
                order_P=int(p.get("order_P", 4)), leaf_panels=int(p.get("leaf_panels", 300)),
                gmres_restart=int(p["gmres_restart"]), gmres_tol=p["gmres_tol"],
                scf_tol_debye=p["scf_tol_debye"], scf_omega=p["scf_omega"],
                thole_a=p["thole_a"], precision=precision)
    args.update(kw)
    s = Solver(**args)
    s.set_mesh(w["verts"], w["tris"])
    s.set_sites(w["xyz"], w["q"], w["d"], w["Q9"], w["alpha"])
    return s


_W = {}


def _work(name):
    if name not in _W:
        w = workload(name)
        m = bie.Mesh(w["verts"], w["tris"], w["params"]["kappa"])
        _W[name] = (w, m)
    return _W[name]


def _densities(m, seed):
    rng = np.random.default_rng(seed)
    c = m.cen - m.cen.mean(0)
    c = c / np.linalg.norm(c, axis=1, keepdims=True)
    smooth = np.concatenate([1 + 0.5 * c[:, 2] + c[:, 0] * c[:, 1], 0.3 - 0.7 * c[:, 1]])
    return {"random": rng.normal(size=2 * m.N), "smooth": smooth}


def _oracle_rows(m, x, rows, eps_in, eps_out):
    N = m.N
    yr = np.empty(2 * len(rows))
    for k, i in enumerate(rows):
        s = m.operator_sums(x[:N], x[N:], rows=(int(i), int(i) + 1))
        y = bie.system_apply(s, x[i:i + 1], eps_in, eps_out)
        yr[k], yr[len(rows) + k] = y[0], y[1]
    return yr


def _bar(w, mode, kind):
    if mode == "direct":
        return 2e-5
    P = int(w["params"].get("order_P", 4))
    return 1e-3 if P <= 4 else 5e-4


@pytest.mark.parametrize("name", FULL)
def test_fullsize_matvec_rows(name):
    w, m = _work(name)
    p = w["params"]
    print("case", name, "panels", m.N, flush=True)
    s = _solver(w)
    rows = np.sort(np.random.default_rng(7).choice(m.N, ROWS, replace=False))
    for kind, x in _densities(m, 3).items():
        y = s.matvec(x)
        got = np.concatenate([y[rows], y[m.N + rows]])
        ref = _oracle_rows(m, x, rows, p["eps_in"], p["eps_out"])
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(name, kind, p["mode"], "sampled-row error", err, flush=True)
        assert err < _bar(w, p["mode"], kind)
    s.close()


def test_fullsize_direct_matvec_rows():
    """The direct product at the largest sphere (the bench's direct mode)."""
    w, m = _work("sphere_81920")
    s = _solver(w, mode="direct")
    rows = np.sort(np.random.default_rng(8).choice(m.N, ROWS, replace=False))
    x = _densities(m, 4)["random"]
    y = s.matvec(x)
    got = np.concatenate([y[rows], y[m.N + rows]])
    ref = _oracle_rows(m, x, rows, 1.0, 80.0)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("direct sampled-row error", err)
    assert err < 2e-5


@pytest.mark.parametrize("name", ["globule_5000", "binding_complex"])
def test_fullsize_rhs_and_site_fields(name):
    w, m = _work(name)
    s = _solver(w)
    rng = np.random.default_rng(9)
    rows = np.sort(rng.choice(m.N, 256, replace=False))
    p_tot = w["d"] + 0.05 * rng.normal(size=w["d"].shape)
    f = s.rhs(p_tot)
    ref = mp.rhs(m.cen[rows], w["xyz"], w["q"], p_tot, w["Q9"], 1.0)
    err = np.abs(f[rows] - ref).max() / np.abs(ref).max()
    print(name, "rhs sampled error", err)
    assert err < 1e-6
    sites = np.sort(rng.choice(len(w["q"]), SITES, replace=False))
    x = _densities(m, 5)["smooth"]
    out = s.site_fields(x)[sites]
    ref = 4 * np.pi * m.readout(x, w["xyz"][sites])
    for k in range(10):
        e = np.abs(out[:, k] - ref[:, k]).max() / np.abs(ref[:, k]).max()
        print(name, "site field", k, e)
        assert e < 2e-5, (k, e)


@pytest.mark.parametrize("name", ["sphere_81920", "globule_1000", "globule_5000"])
def test_fullsize_energy_properties(name):
    """Mixed vs FP64 on the same method, and treecode vs direct."""
    w, m = _work(name)
    print(name, "mixed solve", flush=True)
    rm = _solver(w, gmres_restart=100, gmres_maxit=8000).solve(outputs=False)
    print(name, "status", rm["status"], "scf", rm["scf_iters"], "gmres", rm["gmres_iters"],
          "relres", rm["relres"], flush=True)
    print(name, "fp64 solve", flush=True)
    r64 = _solver(w, precision="fp64", gmres_restart=100, gmres_maxit=8000).solve(outputs=False)
    print(name, "status", r64["status"], "scf", r64["scf_iters"], "gmres", r64["gmres_iters"],
          "relres", r64["relres"], flush=True)
    rel = abs(rm["dG"] - r64["dG"]) / abs(r64["dG"])
    print(name, "dG mixed", rm["dG"], "fp64", r64["dG"], "rel", rel, flush=True)
    assert rm["status"] == 0 and r64["status"] == 0
    assert rel < 1e-4
    if w["params"]["mode"] == "treecode":
        print(name, "direct solve", flush=True)
        rd = _solver(w, precision="mixed", mode="direct", gmres_restart=100,
                     gmres_maxit=8000).solve(outputs=False)
        rel_t = abs(r64["dG"] - rd["dG"]) / abs(rd["dG"])
        P = int(w["params"]["order_P"])
        print(name, "dG tree fp64", r64["dG"], "direct mixed", rd["dG"], "rel", rel_t)
        assert rel_t < (2e-5 if P <= 4 else 1e-5) + 1e-6


def test_fullsize_gradients_fd_globule_5000(say):
    """The 5000-atom globule (treecode, P = 5): adjoint gradients of the
    solvation energy for 4 seeded atoms against central differences
    (h = 1e-4 A) along a random direction per atom.  FP64 state: the base
    solved in stages of tightening tolerance (each warm-started from the
    last), every displaced solve warm-started from the last one, all to a
    GMRES tolerance of 1e-14: the energy error of a solve is about the
    adjoint times the residual, and at 1e-12 it still moved these
    differences by ~5e-4 (1e-5 on the 1000-atom globule, where 1e-14 brings
    the agreement to 1e-8..1e-6).  The adjoint differentiates that FP64
    state with mixed-precision transposed solves at 1e-8 (precision switched
    after the solve; their FP64 refinement holds the tolerance)."""
    w, m = _work("globule_5000")
    s = _solver(w, precision="fp64", gmres_restart=100, gmres_maxit=20000, scf_maxit=500,
                warm_start=True)
    for gtol, stol in ((1e-6, 1e-6), (1e-9, 1e-8), (1e-12, 1e-11), (1e-14, 1e-12)):
        s.set_options(gmres_tol=gtol, scf_tol_debye=stol)
        base = s.solve(outputs=False)
        say("base stage", gtol, base["dG"], base["status"], base["scf_iters"],
            base["gmres_iters"])
        assert base["status"] == 0
    # the adjoint's operator is the exact transpose of the solve's
    rng0 = np.random.default_rng(21)
    x, z = rng0.normal(size=2 * m.N), rng0.normal(size=2 * m.N)
    lhs, rhs = z @ s.matvec(x), s.matvec(z, transpose=True) @ x
    say("transpose check", lhs, rhs, abs(lhs - rhs) / (np.linalg.norm(z) * np.linalg.norm(x)))
    assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(z) * np.linalg.norm(x)
    s.set_options(precision="mixed", gmres_tol=1e-8)
    g = s.backward(1.0, verts=False)
    say("backward", "status", g["status"])
    assert g["status"] == 0
    s.set_options(precision="fp64", gmres_tol=1e-14, scf_tol_debye=1e-12)
    rng = np.random.default_rng(20)
    atoms = np.sort(rng.choice(len(w["q"]), 4, replace=False))
    h = 1e-4
    gmax = np.abs(g["xyz"]).max()
    worst = 0.0
    for l in atoms:
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        e = []
        for sign in (1.0, -1.0):
            xyz = w["xyz"].copy()
            xyz[l] += sign * h * u
            s.set_sites(xyz, w["q"], w["d"], w["Q9"], w["alpha"])
            r = s.solve(outputs=False)
            assert r["status"] == 0
            e.append(r["dG"])
        fd = (e[0] - e[1]) / (2 * h)
        an = g["xyz"][l] @ u
        err = abs(an - fd) / max(abs(fd), 1e-2 * gmax)
        worst = max(worst, err)
        say("atom", l, "adjoint", an, "fd", fd, "rel", err)
    s.close()
    assert worst < 1e-4


def _traceless(rng, n):
    A = rng.normal(size=(n, 3, 3))
    A = A + A.transpose(0, 2, 1)
    A -= np.trace(A, axis1=1, axis2=2)[:, None, None] * np.eye(3) / 3.0
    return A.reshape(n, 9)


def test_fullsize_multipole_gradients_fd_globule_5000(say):
    """Gradients with respect to the charges, dipoles and quadrupoles of 20
    seeded atoms of the 5000-atom globule (treecode, P = 5) against central
    differences, one random direction per kind over all 20 atoms.  The
    solvation energy is a homogeneous quadratic form in the permanent
    multipoles (the right-hand side, the induced dipoles and the reaction
    potentials are linear in them and the energy pairs two such quantities),
    so a central difference is exact at any step: the step is large (0.5
    along a unit direction) and only the solve tolerance limits the
    agreement.  FP64 state at GMRES 1e-10 (its energy is within ~3e-6
    kcal/mol of the 1e-14 one), differentiated by mixed transposed solves
    at 1e-8 (the gradient's error follows the adjoint's, far below the
    bar)."""
    w, m = _work("globule_5000")
    s = _solver(w, precision="fp64", gmres_restart=100, gmres_maxit=20000, scf_maxit=500,
                warm_start=True)
    for gtol, stol in ((1e-6, 1e-6), (1e-10, 1e-9)):
        s.set_options(gmres_tol=gtol, scf_tol_debye=stol)
        base = s.solve(outputs=False)
        say("base stage", gtol, base["dG"], base["status"], base["scf_iters"],
            base["gmres_iters"])
        assert base["status"] == 0
    s.set_options(precision="mixed", gmres_tol=1e-8)
    g = s.backward(1.0, verts=False)
    say("backward status", g["status"])
    assert g["status"] == 0
    s.set_options(precision="fp64", gmres_tol=1e-10, scf_tol_debye=1e-9)
    rng = np.random.default_rng(22)
    atoms = np.sort(rng.choice(len(w["q"]), 20, replace=False))
    h = 0.5
    for kind, width in (("q", 1), ("d", 3), ("Q9", 9)):
        U = np.zeros((len(w["q"]), width))
        U[atoms] = _traceless(rng, 20) if kind == "Q9" else rng.normal(size=(20, width))
        U = U.reshape(w[kind].shape) / np.linalg.norm(U)
        e = []
        for sign in (1.0, -1.0):
            mp_ = {k: w[k] for k in ("q", "d", "Q9")}
            mp_[kind] = w[kind] + sign * h * U
            s.set_sites(w["xyz"], mp_["q"], mp_["d"], mp_["Q9"], w["alpha"])
            r = s.solve(outputs=False)
            say(kind, sign, r["dG"], r["status"], r["scf_iters"], r["gmres_iters"])
            assert r["status"] == 0
            e.append(r["dG"])
        fd = (e[0] - e[1]) / (2 * h)
        an = float(np.sum(g[kind] * U))
        rel = abs(an - fd) / abs(fd)
        say(kind, "adjoint", an, "fd", fd, "rel", rel)
        assert rel < 1e-4
    s.close()
