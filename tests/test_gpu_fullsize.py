"""The GPU path at the full workload sizes, in the configuration the
benchmark times (mixed precision, each workload's own mode, theta, order and
leaf size), through the C-ABI.

The FP64 oracle cannot run a whole product at these sizes, so it evaluates
sampled rows one at a time: operator-product rows, right-hand-side entries
and site fields.  Whole-solve results are checked through properties that
hold at any size: the mixed path against the FP64 path of the same method
(relative 1e-4 on the energy), and the FP64 treecode energy against the
FP64 direct solve (relative 1e-5).

Checks that take several minutes each on one GPU (the FP64 direct solve
of the 5000-atom globule, per-atom finite differences on it, the full
binding triad) run only with PBMP_LONG_TESTS=1; their last results are
recorded in profiles/fullsize_checks.md.

Bars on sampled rows (max-norm error over the sample divided by the
sample's max-norm): direct mixed 2e-5 (FP32 far field); treecode against
the oracle's direct operator 5e-4 at P = 4 and 2e-4 at P = 5 (the
treecode's own approximation; its 2-norm error is ~1e-4 at P = 4 on the
5120-panel sphere against the full oracle product, and a max-norm over a
sample sits above that), against the oracle's treecode product 1e-12
(FP64) and 2e-5 (mixed)."""

import os
import time

import numpy as np
import pytest

from oracle import bie, multipoles as mp
from synth import workload

pytestmark = pytest.mark.gpu

FULL = ["sphere_81920", "globule_1000", "globule_5000", "binding_complex"]
LONG = os.environ.get("PBMP_LONG_TESTS") == "1"
long_only = pytest.mark.skipif(
    not LONG, reason="several minutes on one GPU: run with PBMP_LONG_TESTS=1 "
                     "(results recorded in profiles/fullsize_checks.md)")
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
    return 5e-4 if P <= 4 else 2e-4


@pytest.mark.parametrize("name", FULL)
def test_fullsize_matvec_rows(name, say):
    """Sampled rows of the product in the benchmark's configuration against
    the oracle's direct operator (at the treecode's accuracy), and, for the
    treecode workloads, against the oracle's treecode product on the same
    octree (FP64 to rounding, mixed to the FP32 far field)."""
    w, m = _work(name)
    p = w["params"]
    say("case", name, "panels", m.N)
    s = _solver(w)
    rows = np.sort(np.random.default_rng(7).choice(m.N, ROWS, replace=False))
    xs = _densities(m, 3)
    for kind, x in xs.items():
        y = s.matvec(x)
        got = np.concatenate([y[rows], y[m.N + rows]])
        ref = _oracle_rows(m, x, rows, p["eps_in"], p["eps_out"])
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say(name, kind, p["mode"], "sampled-row error vs direct operator", err)
        assert err < _bar(w, p["mode"], kind)
    s.close()
    if p["mode"] != "treecode":
        return
    from oracle import treecode
    t0 = time.perf_counter()
    tc = treecode.Treecode(m, p["theta"], int(p["order_P"]), int(p["leaf_panels"]))
    x = xs["random"]
    ref = tc.matvec(x, p["eps_in"], p["eps_out"], rows=rows)
    say(name, "oracle treecode rows %.1f s" % (time.perf_counter() - t0))
    for precision, tol in (("fp64", 1e-12), ("mixed", 2e-5)):
        s = _solver(w, precision=precision)
        y = s.matvec(x)
        s.close()
        got = np.concatenate([y[rows], y[m.N + rows]])
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say(name, precision, "sampled-row error vs oracle treecode", err)
        assert err < tol


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


def _solve(w, say, label, **kw):
    t0 = time.perf_counter()
    r = _solver(w, gmres_restart=100, gmres_maxit=20000, **kw).solve(outputs=False)
    say(label, "status", r["status"], "scf", r["scf_iters"], "gmres", r["gmres_iters"],
        "relres", r["relres"], "dG", r["dG"], "%.1f s" % (time.perf_counter() - t0))
    assert r["status"] == 0
    return r


@pytest.mark.parametrize("name", ["sphere_81920", "globule_1000", "globule_5000"])
def test_fullsize_energy_properties(name, say):
    """Mixed vs FP64 on the same method (relative 1e-4); where the workload
    uses the treecode, the FP64 treecode energy against the FP64 direct
    solve (relative 1e-5; on the 5000-atom globule that direct solve is a
    long check of its own)."""
    w, m = _work(name)
    rm = _solve(w, say, name + " mixed")
    r64 = _solve(w, say, name + " fp64", precision="fp64")
    rel = abs(rm["dG"] - r64["dG"]) / abs(r64["dG"])
    say(name, "dG mixed vs fp64", rel)
    assert rel < 1e-4
    if w["params"]["mode"] == "treecode" and name != "globule_5000":
        rd = _solve(w, say, name + " fp64 direct", precision="fp64", mode="direct")
        rel_t = abs(r64["dG"] - rd["dG"]) / abs(rd["dG"])
        say(name, "dG fp64 treecode vs fp64 direct", rel_t)
        assert rel_t < 1e-5


@long_only
def test_fullsize_treecode_vs_fp64_direct_globule_5000(say):
    """The 5000-atom globule (theta 0.5, P 5): FP64 treecode energy against
    the FP64 direct solve, relative 1e-5."""
    w, m = _work("globule_5000")
    r64 = _solve(w, say, "globule_5000 fp64 treecode", precision="fp64", verbose=True)
    rd = _solve(w, say, "globule_5000 fp64 direct", precision="fp64", mode="direct",
                verbose=True)
    rel_t = abs(r64["dG"] - rd["dG"]) / abs(rd["dG"])
    say("globule_5000 dG fp64 treecode vs fp64 direct", rel_t)
    assert rel_t < 1e-5


def _fd_state(name, say, mixed_adjoint=True):
    """FP64 base state of a globule (treecode) solved to GMRES 1e-14 / SCF
    1e-12 D in stages of tightening tolerance (each warm-started from the
    last: the energy error of a solve is about the adjoint times its
    residual, and central differences at h = 1e-4 A need it below ~1e-9
    kcal/mol), and its adjoint gradients (mixed-precision transposed solves
    at 1e-8 whose FP64 refinement holds the tolerance, precision switched
    after the solve; or FP64 ones).  The gradient checks below share it and
    leave the solver at the base tolerances."""
    w, m = _work(name)
    s = _solver(w, precision="fp64", gmres_restart=100, gmres_maxit=20000, scf_maxit=500,
                warm_start=True, verbose=True)
    t0 = time.perf_counter()
    for gtol, stol in ((1e-6, 1e-6), (1e-10, 1e-9), (1e-14, 1e-12)):
        s.set_options(gmres_tol=gtol, scf_tol_debye=stol)
        base = s.solve(outputs=False)
        say(name, "base stage", gtol, base["dG"], base["status"], base["scf_iters"],
            base["gmres_iters"], "%.1f s" % (time.perf_counter() - t0))
        assert base["status"] == 0
    # the adjoint's operator is the exact transpose of the solve's
    rng0 = np.random.default_rng(21)
    x, z = rng0.normal(size=2 * m.N), rng0.normal(size=2 * m.N)
    lhs, rhs = z @ s.matvec(x), s.matvec(z, transpose=True) @ x
    say(name, "transpose check", abs(lhs - rhs) / (np.linalg.norm(z) * np.linalg.norm(x)))
    assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(z) * np.linalg.norm(x)
    s.set_options(precision="mixed" if mixed_adjoint else "fp64", gmres_tol=1e-8)
    g = s.backward(1.0, verts=False)
    say(name, "backward", "status", g["status"], "%.1f s" % (time.perf_counter() - t0))
    assert g["status"] == 0
    s.set_options(precision="fp64", gmres_tol=1e-14, scf_tol_debye=1e-12)
    return dict(w=w, m=m, s=s, g=g, dG=base["dG"], name=name)


@pytest.fixture(scope="module")
def g1000(say_module):
    st = _fd_state("globule_1000", say_module)
    yield st
    st["s"].close()


@pytest.fixture(scope="module")
def g5000(say_module):
    st = _fd_state("globule_5000", say_module)
    yield st
    st["s"].close()


def _energy_at(st, say, label, xyz=None, q=None, d=None, Q9=None):
    w, s = st["w"], st["s"]
    t0 = time.perf_counter()
    s.set_sites(w["xyz"] if xyz is None else xyz, w["q"] if q is None else q,
                w["d"] if d is None else d, w["Q9"] if Q9 is None else Q9, w["alpha"])
    r = s.solve(outputs=False)
    say(st["name"], label, r["dG"], r["status"], r["scf_iters"], r["gmres_iters"],
        "%.1f s" % (time.perf_counter() - t0))
    assert r["status"] == 0
    return r["dG"]


GRAD_ATOMS = 20


def _joint_position_check(st, say):
    """Adjoint position gradients of 20 seeded atoms against a central
    difference (h = 1e-4 A) along one joint random direction U that moves
    all 20 atoms at once (unit norm over the 60 coordinates): the adjoint
    gives sum_l g_l . U_l, the difference (E(+hU) - E(-hU)) / 2h; plain
    relative error below 1e-4."""
    w, g = st["w"], st["g"]
    rng = np.random.default_rng(20)
    atoms = np.sort(rng.choice(len(w["q"]), GRAD_ATOMS, replace=False))
    U = np.zeros_like(w["xyz"])
    U[atoms] = rng.normal(size=(GRAD_ATOMS, 3))
    U /= np.linalg.norm(U)
    h = 1e-4
    st["s"].set_options(gmres_tol=1e-14, scf_tol_debye=1e-12)
    e = [_energy_at(st, say, "joint %+g" % sg, xyz=w["xyz"] + sg * h * U) for sg in (1.0, -1.0)]
    fd = (e[0] - e[1]) / (2 * h)
    an = float(np.sum(g["xyz"] * U))
    rel = abs(an - fd) / abs(fd)
    say(st["name"], "joint direction over 20 atoms: adjoint", an, "fd", fd, "rel", rel)
    assert rel < 1e-4


def _per_atom_position_check(st, say, atoms_slice=slice(None)):
    """Per atom, for the 20 seeded atoms (or a slice of them): central
    difference (h = 1e-4 A) along a random unit direction u_l against
    g_l . u_l.  The error is taken relative to |g_l|, the norm of the atom's
    gradient (a random direction can be nearly orthogonal to it, so
    |g_l . u_l| has no floor); bar 1e-4."""
    w, g = st["w"], st["g"]
    rng = np.random.default_rng(23)
    atoms = np.sort(rng.choice(len(w["q"]), GRAD_ATOMS, replace=False))
    dirs = rng.normal(size=(GRAD_ATOMS, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    h = 1e-4
    st["s"].set_options(gmres_tol=1e-14, scf_tol_debye=1e-12)
    worst = 0.0
    for l, u in list(zip(atoms, dirs))[atoms_slice]:
        e = []
        for sg in (1.0, -1.0):
            xyz = w["xyz"].copy()
            xyz[l] += sg * h * u
            e.append(_energy_at(st, say, "atom %d %+g" % (l, sg), xyz=xyz))
        fd = (e[0] - e[1]) / (2 * h)
        an = g["xyz"][l] @ u
        err = abs(an - fd) / np.linalg.norm(g["xyz"][l])
        worst = max(worst, err)
        say(st["name"], "atom", l, "adjoint", an, "fd", fd, "|g_l|",
            np.linalg.norm(g["xyz"][l]), "err/|g_l|", err)
    assert worst < 1e-4


def _traceless(rng, n):
    A = rng.normal(size=(n, 3, 3))
    A = A + A.transpose(0, 2, 1)
    A -= np.trace(A, axis1=1, axis2=2)[:, None, None] * np.eye(3) / 3.0
    return A.reshape(n, 9)


def _multipole_check(st, say):
    """Gradients with respect to the charges, dipoles and quadrupoles of 20
    seeded atoms against central differences, one random direction per kind
    over all 20 atoms.  The solvation energy is a homogeneous quadratic form
    in the permanent multipoles (the right-hand side, the induced dipoles
    and the reaction potentials are linear in them and the energy pairs two
    such quantities), so a central difference is exact at any step: the
    step is large (0.5 along a unit direction) and only the solve tolerance
    limits the agreement (displaced solves at GMRES 1e-11, SCF 1e-10 D)."""
    w, g, s = st["w"], st["g"], st["s"]
    s.set_options(gmres_tol=1e-11, scf_tol_debye=1e-10)
    rng = np.random.default_rng(22)
    atoms = np.sort(rng.choice(len(w["q"]), GRAD_ATOMS, replace=False))
    h = 0.5
    for kind, width in (("q", 1), ("d", 3), ("Q9", 9)):
        U = np.zeros((len(w["q"]), width))
        U[atoms] = _traceless(rng, GRAD_ATOMS) if kind == "Q9" else \
            rng.normal(size=(GRAD_ATOMS, width))
        U = U.reshape(w[kind].shape) / np.linalg.norm(U)
        e = [_energy_at(st, say, "%s %+g" % (kind, sg), **{kind: w[kind] + sg * h * U})
             for sg in (1.0, -1.0)]
        fd = (e[0] - e[1]) / (2 * h)
        an = float(np.sum(g[kind] * U))
        rel = abs(an - fd) / abs(fd)
        say(st["name"], kind, "adjoint", an, "fd", fd, "rel", rel)
        assert rel < 1e-4
    s.set_options(gmres_tol=1e-14, scf_tol_debye=1e-12)


# The 1000-atom globule (about 30k panels, theta 0.5, P 4): the gradient
# checks of the workload definition, in the main suite (the per-atom
# differences of all 20 atoms as a long check).
def test_position_gradient_fd_joint_globule_1000(g1000, say):
    _joint_position_check(g1000, say)


def test_position_gradient_fd_per_atom_globule_1000(g1000, say):
    """The first 4 of the 20 seeded atoms (all 20: a long check)."""
    _per_atom_position_check(g1000, say, slice(0, 4))


@long_only
def test_position_gradient_fd_all_atoms_globule_1000(g1000, say):
    _per_atom_position_check(g1000, say, slice(4, None))


def test_multipole_gradients_fd_globule_1000(g1000, say):
    _multipole_check(g1000, say)


# The 5000-atom globule (about 150k panels, theta 0.5, P 5): the same
# checks, several minutes each (each displaced solve to GMRES 1e-14 takes
# about a minute on one GPU).  PBMP_LONG_ATOMS=a:b restricts the per-atom
# check to atoms a..b-1 of the 20, so that it can be spread over runs.
@long_only
def test_position_gradient_fd_joint_globule_5000(g5000, say):
    _joint_position_check(g5000, say)


@long_only
def test_position_gradient_fd_per_atom_globule_5000(g5000, say):
    sel = os.environ.get("PBMP_LONG_ATOMS", "")
    sl = slice(*(int(v) for v in sel.split(":"))) if sel else slice(None)
    _per_atom_position_check(g5000, say, sl)


@long_only
def test_multipole_gradients_fd_globule_5000(g5000, say):
    _multipole_check(g5000, say)


@long_only
def test_binding_triad_fullsize(say):
    """The full binding triad (receptor 3000 atoms / ~90k panels, ligand
    200 / ~8k, complex 3200 / ~96k; treecode theta 0.5, P 4): the relative
    binding energy (eq. rel_bind_energy) in mixed precision against FP64
    (relative 1e-4), and the derivative of the FP64 relative binding energy
    with respect to a rigid translation of the ligand (treecode adjoint,
    vertex terms with the treecode's lists and expansions) against central
    differences of direct solves of the complex (h = 1e-3 A along each
    axis: the octree would move with the ligand, so differences of treecode
    solves jump at the treecode's truncation level; the difference of
    direct solves is smooth).  The translation gradient is a sum over the
    ligand's sites and its ~5800 surface vertices whose terms largely
    cancel, so the treecode's approximation error weighs far more on it
    than on the energy: on the small triad of test_gpu_binding it is 8e-3
    of the gradient's norm at P 4 and 1e-3 at P 5 (against the direct-mode
    gradient; energies 3e-5 and 9e-6), and here the difference to direct
    solves is 4e-3 (x axis; bar 1e-2 of the gradient's norm).  The error
    falls with theta and P (small triad: 1.8e-5 at theta 0.3, P 6; a
    theta 0.3, P 6 solve and backward of this complex take over 15 minutes
    in FP64, beyond one run).  The
    displaced solves are FP64 (the mixed path's FP32 far readout leaves the
    induced dipoles a noise floor near 6e-9 D, above the 1e-9 D these
    differences need) and take about four minutes each, so PBMP_LONG_AXES
    (default "0"; "0,1,2" for all three) selects the axes of one run, and
    the check covers the selected components."""
    from paper_1810_03698_amd import Solver
    from paper_1810_03698_amd.binding import relative_binding
    wA, wB, wAB = (workload(n) for n in ("binding_receptor", "binding_ligand",
                                          "binding_complex"))
    nR = int(wAB["n_receptor"])
    p = wAB["params"]
    base = dict(eps_in=p["eps_in"], eps_out=p["eps_out"], kappa=p["kappa"], mode="treecode",
                theta=0.5, order_P=4, leaf_panels=300, gmres_restart=100, gmres_maxit=20000,
                scf_maxit=500, verbose=True)
    t0 = time.perf_counter()
    res = {}
    for precision, gtol, stol in (("mixed", 1e-8, 1e-8), ("fp64", 1e-10, 1e-9)):
        res[precision] = relative_binding(wAB, wA, wB, n_receptor=nR,
                                          grad=(precision == "fp64"), precision=precision,
                                          gmres_tol=gtol, scf_tol_debye=stol, **base)
        r = res[precision]
        say(precision, "ddG", r["ddG"], "vac", r["dG_bind_vac"], "diss", r["dG_bind_diss"],
            "dG AB/A/B", r["dG_complex"], r["dG_receptor"], r["dG_ligand"],
            "%.0f s" % (time.perf_counter() - t0))
    rel = abs(res["mixed"]["ddG"] - res["fp64"]["ddG"]) / abs(res["fp64"]["ddG"])
    say("ddG mixed vs fp64", rel)
    assert rel < 1e-4
    g = res["fp64"]["grad_t"]
    say("grad_t", g, "ligand vertices", res["fp64"]["ligand_vertices"])
    is_lig = np.arange(len(wAB["q"])) >= nR
    own = np.empty(len(wAB["verts"]), bool)
    for a in range(0, len(wAB["verts"]), 2048):
        dd = np.linalg.norm(wAB["verts"][a:a + 2048, None, :] - wAB["xyz"][None], axis=2)
        own[a:a + 2048] = is_lig[np.argmin(dd - wAB["radii"][None], axis=1)]
    assert res["fp64"]["ligand_vertices"] == int(own.sum())
    s = Solver(precision="fp64", **dict(base, mode="direct", gmres_tol=1e-10,
                                        scf_tol_debye=1e-9))
    axes = [int(v) for v in os.environ.get("PBMP_LONG_AXES", "0").split(",")]
    h = 1e-3
    fd = np.full(3, np.nan)
    for a in axes:
        e = []
        for sg in (1.0, -1.0):
            v = wAB["verts"].copy()
            v[own, a] += sg * h
            x = wAB["xyz"].copy()
            x[is_lig, a] += sg * h
            s.set_mesh(v, wAB["tris"])
            s.set_sites(x, wAB["q"], wAB["d"], wAB["Q9"], wAB["alpha"])
            r = s.solve(outputs=False)
            assert r["status"] == 0
            e.append(r["dG"])
            say("direct complex", a, sg, r["dG"], r["gmres_iters"], "%.0f s" % (time.perf_counter() - t0))
        fd[a] = (e[0] - e[1]) / (2 * h)
    s.close()
    # relative to the norm of the adjoint gradient (the differences may
    # cover only some axes)
    err = np.abs(g - fd)[axes].max() / np.linalg.norm(g)
    say("translation gradient: treecode adjoint", g, "direct FD", fd, "err/|g|", err)
    assert err < 1e-2
