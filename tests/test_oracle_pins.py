"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics (closed forms, identities, brute force, library routines).
CPU only."""

import math
import os

import numpy as np
import pytest
import scipy.special as sp
from scipy import integrate

from oracle import bie, kirkwood, multipoles as mp, quadrature, solver
from synth import icosphere, workload

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---------------------------------------------------------------- quadrature
def _moment_err(bary, w, i, j):
    x, y = bary[:, 1], bary[:, 2]
    return abs(np.sum(w * x ** i * y ** j) - quadrature.exact_moment(i, j))


def test_exact_moment_brute_force():
    # the moment formula itself against 2D adaptive quadrature
    for i, j in [(0, 0), (2, 1), (3, 3), (5, 0)]:
        val, _ = integrate.dblquad(lambda y, x: x ** i * y ** j, 0, 1, 0,
                                   lambda x: 1 - x)
        assert abs(2 * val - quadrature.exact_moment(i, j)) < 1e-13


def test_three_point_rule_degree_two():
    b, w = quadrature.tri3()
    assert abs(w.sum() - 1) < 1e-15
    for d in range(3):
        for i in range(d + 1):
            assert _moment_err(b, w, i, d - i) < 1e-15
    assert max(_moment_err(b, w, i, 3 - i) for i in range(4)) > 1e-4


def test_nineteen_point_rule_degree_nine():
    b, w = quadrature.tri19()
    assert len(w) == 19 and (w > 0).all() and (b > 0).all()
    assert abs(b.sum(1) - 1).max() < 1e-15
    for d in range(10):
        for i in range(d + 1):
            assert _moment_err(b, w, i, d - i) < 2e-15
    assert max(_moment_err(b, w, i, 10 - i) for i in range(11)) > 1e-9



def test_nineteen_point_rule_published_values():
    """The rule equals the published symmetric degree-9, 19-point rule
    (D. A. Dunavant, Int. J. Numer. Meth. Eng. 21 (1985) 1129, table for
    degree 9; weights normalised to sum 1, values printed to 15 digits),
    stored as the fixture tests/golden/dunavant_degree9_19pt.txt."""
    b, w = quadrature.tri19()
    rows = np.loadtxt(os.path.join(GOLDEN, "dunavant_degree9_19pt.txt"))
    # (weight, barycentric node of one orbit member); the centroid is 1/3
    # exactly, printed rounded
    printed = [(r[0], (1 / 3, 1 / 3, 1 / 3) if k == 0 else tuple(r[1:]))
               for k, r in enumerate(rows)]
    for wt, node in printed:
        d = np.abs(np.sort(b, axis=1) - np.sort(node)).max(axis=1)
        q = np.argmin(d)
        assert d[q] < 1e-14 and abs(w[q] - wt) < 1e-14
    # orbit multiplicities 1 + 3 + 3 + 3 + 3 + 6
    assert sorted(np.unique(np.round(w, 12), return_counts=True)[1]) == [1, 3, 3, 3, 3, 6]

# ---------------------------------------------------------- singular panels
def _adaptive_panel_integral(v, c, kernel):
    """int over triangle v of kernel(|c - y|) dy, by splitting at c into
    three sub-triangles and integrating each in polar form around c."""
    tot = 0.0
    for e in range(3):
        a, b = v[e], v[(e + 1) % 3]

        def f(s, t):
            # point on segment a->b at t, radial fraction s from c
            p = a + t * (b - a)
            d = p - c
            # Jacobian of (s, t) -> c + s (p - c): s * |(b - a) x (p - c)|
            jac = s * np.linalg.norm(np.cross(b - a, d))
            r = s * np.linalg.norm(d)
            return kernel(r) * jac

        val, _ = integrate.dblquad(f, 0, 1, 0, 1, epsabs=1e-14, epsrel=1e-13)
        tot += val
    return tot


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_self_integrals_vs_adaptive(seed):
    """Mesh-like panels (edge ~0.6 A, perturbed equilateral): the exact
    Laplace term and the 16-node edge rule for the Yukawa remainder agree
    with adaptive quadrature of the singular integrand."""
    rng = np.random.default_rng(seed)
    eq = np.array([[0, 0, 0], [1, 0, 0], [0.5, 3 ** 0.5 / 2, 0]])
    v = 0.6 * (eq + 0.25 * rng.normal(size=(3, 3)))
    c = v.mean(0)
    ref_l = _adaptive_panel_integral(v, c, lambda r: 1 / (4 * np.pi * r))
    for kappa in (0.125, 0.7):
        m = bie.Mesh(v, np.array([[0, 1, 2]]), kappa=kappa)
        vl, vy = m.self_integrals(0)
        ref_y = _adaptive_panel_integral(
            v, c, lambda r: np.exp(-kappa * r) / (4 * np.pi * r))
        assert abs(vl - ref_l) < 1e-12 * abs(ref_l)
        assert abs(vy - ref_y) < 1e-13 * abs(ref_y)


def test_self_yukawa_edge_rule_on_slivers():
    """A badly shaped unit-size panel: the 16-node edge rule (in u =
    asinh(s/h)) still reaches the adaptive reference."""
    v = np.random.default_rng(0).normal(size=(3, 3))
    c = v.mean(0)
    ref = _adaptive_panel_integral(v, c, lambda r: np.exp(-0.7 * r) / (4 * np.pi * r))
    got = bie.Mesh(v, np.array([[0, 1, 2]]), kappa=0.7).self_integrals(0)[1]
    assert abs(got - ref) < 1e-13 * abs(ref)


def test_self_yukawa_limits():
    v = np.array([[0.0, 0, 0], [1.3, 0.1, 0], [0.2, 0.9, 0.3]])
    A = 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
    vl0, vy0 = bie.Mesh(v, np.array([[0, 1, 2]]), kappa=0.0).self_integrals(0)
    assert vl0 == vy0
    # exp(-k r)/r = 1/r - k + k^2 r / 2 + O(k^3)
    Ir = _adaptive_panel_integral(v, v.mean(0), lambda r: r)
    for k in (1e-2, 1e-3):
        vl, vy = bie.Mesh(v, np.array([[0, 1, 2]]), kappa=k).self_integrals(0)
        series = (-k * A + 0.5 * k * k * Ir) / (4 * np.pi)
        assert abs((vy - vl) - series) < k ** 3 * A


# ------------------------------------------------------- operator identities
def _solid_angle(x, v0, v1, v2):
    """Signed solid angle of triangles seen from x (Van Oosterom and
    Strackee), positive when x is on the side opposite the normal."""
    a, b, c = v0 - x, v1 - x, v2 - x
    na, nb, nc = (np.linalg.norm(u, axis=-1) for u in (a, b, c))
    num = np.einsum("ij,ij->i", a, np.cross(b, c))
    dot = lambda u, v: np.einsum("ij,ij->i", u, v)
    den = na * nb * nc + dot(a, b) * nc + dot(a, c) * nb + dot(b, c) * na
    return 2 * np.arctan2(num, den)


def test_double_layer_vs_exact_solid_angles():
    """K_L[i,j] = -Omega_j(c_i)/(4 pi) exactly; the exact row sums give the
    double-layer identity -1/2 on a closed surface, and the oracle's
    quadrature entries approach them (3-point far, 19-point near)."""
    v, t = icosphere(3, 4.0)
    m = bie.Mesh(v, t, kappa=0.125)
    g = m.geo
    for i in (3, 100, 777):
        KL = m.dense_operators(rows=(i, i + 1))[1][0]
        om = _solid_angle(m.cen[i], g["v0"], g["v1"], g["v2"])
        om[i] = 0.0
        ex = -om / (4 * np.pi)
        assert abs(ex.sum() + 0.5) < 1e-12
        d = np.linalg.norm(m.cen - m.cen[i], axis=1)
        near = d < 2 * np.sqrt(m.area[i])
        near[i] = False
        far = ~near
        far[i] = False
        assert KL[i] == 0.0
        assert np.abs(KL[near] - ex[near]).max() < 1e-4
        assert np.abs(KL[far] - ex[far]).max() < 3e-5
        assert np.abs((KL[far] - ex[far]) / ex[far]).max() < 1e-2
        assert abs(KL.sum() + 0.5) < 1e-4


def _sphere_eigs(n, R, kappa):
    x = kappa * R
    i_n = sp.spherical_in(n, x)
    k_n = sp.spherical_kn(n, x) * 2 / np.pi  # sqrt(2/(pi x)) K_{n+1/2}
    kp_n = sp.spherical_kn(n, x, derivative=True) * 2 / np.pi
    # V_L, K_L, V_Y, K_Y eigenvalues for degree-n spherical harmonics
    return (R / (2 * n + 1), -1 / (2 * (2 * n + 1)),
            kappa * R ** 2 * i_n * k_n,
            kappa ** 2 * R ** 2 * i_n * kp_n + 0.5)


def test_sphere_eigenvalues_tabulated():
    """Eigenvalues of V_L, K_L, V_Y, K_Y on the sphere R = 4 A, kappa = 0.125
    for degrees 0-2, tabulated to 7 digits: R/(2n+1), -1/(2(2n+1)) and the
    modified-spherical-Bessel products of the Yukawa single and double
    layers."""
    ref = {0: (4, -0.5, 2.5284822, -0.4481808),
           1: (4 / 3, -1 / 6, 1.2436599, -0.1736491),
           2: (0.8, -0.1, 0.7820869, -0.1020011)}
    for n, vals in ref.items():
        got = _sphere_eigs(n, 4.0, 0.125)
        assert np.allclose(got, vals, atol=2e-7)


def test_sphere_eigenvalues_converge():
    errs = []
    for lev in (3, 4):
        v, t = icosphere(lev, 4.0)
        m = bie.Mesh(v, t, kappa=0.125)
        ops = m.dense_operators() if lev == 3 else None
        c = m.cen / np.linalg.norm(m.cen, axis=1, keepdims=True)
        funcs = {0: np.ones(m.N), 1: c[:, 2], 2: 3 * c[:, 2] ** 2 - 1}
        e = 0.0
        for n, f in funcs.items():
            if ops is not None:
                outs = [op @ f for op in ops]
            else:
                s = m.operator_sums(f, f)
                outs = [s[:, 0], s[:, 1], s[:, 2], s[:, 3]]
            ref = _sphere_eigs(n, 4.0, 0.125)
            for o, lam in zip(outs, ref):
                e = max(e, np.sqrt(np.mean((o - lam * f) ** 2)))
        errs.append(e)
    assert errs[1] < errs[0] / 3.0 and errs[1] < 3e-3


def test_gmres_matches_lu():
    w = workload("sphere_1280")
    m = bie.Mesh(w["verts"], w["tris"], 0.125)
    A = bie.dense_system(m, 1.0, 80.0)
    b = np.concatenate([mp.rhs(m.cen, w["xyz"], w["q"], w["d"], w["Q9"], 1.0),
                        np.zeros(m.N)])
    x_lu = bie.lu_solve(A, b)
    x_g, it, rr = bie.gmres(lambda x: A @ x, b, tol=1e-13)
    assert np.abs(x_g - x_lu).max() <= 1e-12 * np.abs(x_lu).max()
    # matrix-free product equals the dense one
    y = bie.matvec(m, x_lu, 1.0, 80.0)
    assert np.abs(y - A @ x_lu).max() < 1e-13 * np.abs(y).max()


# ------------------------------------------------------------- multipoles
def test_multipole_potential_from_charge_cluster():
    """eq. pot_multipole is the far-field expansion of a charge cloud with
    q = sum q_i, p = sum q_i r_i, Q = sum q_i (3 r r - r^2 I): the error
    falls like (s/R)^3 relative to the leading term."""
    rng = np.random.default_rng(5)
    pts = rng.normal(size=(6, 3)) * 0.1
    qs = rng.normal(size=6)
    q = qs.sum()
    p = (qs[:, None] * pts).sum(0)
    Q = sum(qi * (3 * np.outer(r, r) - r @ r * np.eye(3)) for qi, r in zip(qs, pts))
    errs = []
    for dist in (5.0, 10.0):
        x = np.array([[dist, 0.3 * dist, -0.2 * dist]])
        exact = (qs / np.linalg.norm(x - pts, axis=1)).sum()
        approx = mp.multipole_potential(x, np.zeros((1, 3)), np.array([q]),
                                        p[None], Q.reshape(1, 9))[0]
        errs.append(abs(exact - approx))
    assert errs[1] < errs[0] / 12  # ~ 1/R^4 -> factor 16


def _fd_grad(fun, x, h=1e-5):
    g = np.zeros(3)
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        g[i] = (fun(x + e) - fun(x - e)) / (2 * h)
    return g


def test_permanent_derivatives_fd_and_laplace():
    rng = np.random.default_rng(1)
    xyz = rng.normal(size=(3, 3))
    q, d, Q9, _ = __import__("synth").random_multipoles(rng, 3)
    x0 = np.array([2.0, -1.5, 1.0])
    mask = np.ones((1, 3), bool)
    phi, g, H = mp.permanent_derivs(x0[None], xyz, q, d, Q9, mask)
    f = lambda x: mp.multipole_potential(x[None], xyz, q, d, Q9)[0]
    assert abs(phi[0] - f(x0)) < 1e-13
    assert np.allclose(g[0], _fd_grad(f, x0), atol=1e-8)
    for k in range(3):
        gk = lambda x: mp.permanent_derivs(x[None], xyz, q, d, Q9, mask)[1][0, k]
        assert np.allclose(H[0, k], _fd_grad(gk, x0), atol=1e-7)
    assert abs(np.trace(H[0])) < 1e-12  # harmonic away from the sources


def test_appendix_quadrupole_second_derivative_missing_term():
    """The printed second derivative of R_i R_j / R^5 omits
    (delta_ik delta_jo + delta_io delta_jk)/R^5; the oracle's exact form
    matches finite differences, and the omitted term is nonzero."""
    R = np.array([0.7, -1.1, 0.4])
    r = np.linalg.norm(R)
    i, j, k, o = 0, 1, 0, 1
    f = lambda x: x[i] * x[j] / np.linalg.norm(x) ** 5
    h = 1e-4
    def d_o_d_k(x):
        ek, eo = np.eye(3)[k] * h, np.eye(3)[o] * h
        return (f(x + ek + eo) - f(x + ek - eo) - f(x - ek + eo)
                + f(x - ek - eo)) / (4 * h * h)
    fd = d_o_d_k(R)
    # oracle: unit quadrupole with Q_ij = Q_ji = 1 gives S = 2 R_i R_j
    Q = np.zeros((1, 3, 3))
    Q[0, i, j] = Q[0, j, i] = 1.0
    _, _, H = mp.permanent_derivs(R[None], np.zeros((1, 3)), np.zeros(1),
                                  np.zeros((1, 3)), Q.reshape(1, 9),
                                  np.ones((1, 1), bool))
    assert abs(H[0, k, o] - fd) < 1e-6 * max(1, abs(fd))
    printed = -5 / r ** 7 * (-7 * R[i] * R[j] * R[k] * R[o] / r ** 2
                             + R[j] * R[o] * (i == k) + R[k] * R[j] * (o == i)
                             + R[i] * R[k] * (j == o) + R[o] * R[i] * (k == j)
                             + R[j] * R[i] * (o == k))
    assert abs(printed - fd) > 1e-3 * abs(fd)
    assert abs(printed + 1 / r ** 5 - fd) < 1e-6 * max(1, abs(fd))


def test_thole_recursion_and_limits():
    r = np.linspace(0.3, 4.0, 50)
    al, am, a = 1.1, 0.7, 0.39
    l3, l5, l7 = mp.thole_lambdas(r, al, am, a)
    h = 1e-6
    d3 = (mp.thole_lambdas(r + h, al, am, a)[0] - mp.thole_lambdas(r - h, al, am, a)[0]) / (2 * h)
    d5 = (mp.thole_lambdas(r + h, al, am, a)[1] - mp.thole_lambdas(r - h, al, am, a)[1]) / (2 * h)
    assert np.allclose(l5, l3 - r / 3 * d3, atol=1e-8)
    assert np.allclose(l7, l5 - r / 5 * d5, atol=1e-8)
    big = mp.thole_lambdas(np.array([50.0]), al, am, a)
    assert all(abs(x - 1) < 1e-15 for x in big)
    zero = mp.thole_lambdas(r, 0.0, am, a)
    assert all(np.all(x == 1.0) for x in zero)


def test_damped_tensors_are_derivatives():
    rng = np.random.default_rng(3)
    xyz = rng.normal(size=(2, 3))
    mu = rng.normal(size=(2, 3))
    alpha = np.array([1.2, 0.8])
    x0 = np.array([0.4, 0.3, -0.5])
    ae = np.array([0.9])
    mask = np.ones((1, 2), bool)
    ev = lambda x: mp.induced_derivs(x[None], xyz, mu, ae, alpha, 0.39, mask)
    # the damped potential's FD gradient is NOT the damped field in general,
    # but the damped field's FD derivative IS the damped gradient tensor
    _, g, H = ev(x0)
    for k in range(3):
        assert np.allclose(H[0, k], _fd_grad(lambda x: ev(x)[1][0, k], x0),
                           atol=1e-7)
    # s = a u^3 -> infinity (a -> infinity) removes the damping; a -> 0
    # damps fully (every lambda -> 0)
    und = mp.induced_derivs(x0[None], xyz, mu, ae, alpha, 1e30, mask)
    full = mp.induced_derivs(x0[None], xyz, mu, ae, alpha, 0.0, mask)
    assert all(np.all(f == 0.0) for f in full)
    perm = mp.permanent_derivs(x0[None], xyz, np.zeros(2), mu, np.zeros((2, 9)), mask)
    for u, p in zip(und, perm):
        assert np.allclose(u, p, atol=1e-13)


# ---------------------------------------------------------------- Kirkwood
def test_kirkwood_h_n_is_legendre():
    r = np.array([0.5, -0.7, 1.1])
    rp = np.array([-0.3, 0.8, 0.2])
    nr, nrp = np.linalg.norm(r), np.linalg.norm(rp)
    c = r @ rp / (nr * nrp)
    a = 4.0
    # with f_n = delta_{n,N} the series is h_N / a^(2N+1)
    for N in (0, 1, 4, 9):
        coeffs = np.zeros(12)
        coeffs[N] = 1.0
        old = kirkwood.f_coefficients
        kirkwood.f_coefficients = lambda nmax, *args: coeffs[:nmax + 1]
        try:
            jet = kirkwood.greac_jet(r, rp, a, 1.0, 80.0, 0.1, 11)
        finally:
            kirkwood.f_coefficients = old
        ref = nr ** N * nrp ** N * sp.eval_legendre(N, c) / a ** (2 * N + 1)
        assert abs(jet[0, 0] - ref) < 1e-14 * max(1, abs(ref))


def test_kirkwood_g_n_vs_bessel():
    a, kappa = 4.0, 0.125
    f = kirkwood.f_coefficients(6, a, 1.0, 80.0, kappa)
    x = kappa * a
    for n in range(7):
        g = x * sp.spherical_kn(n, x, derivative=True) / sp.spherical_kn(n, x)
        ref = (1.0 * (n + 1) + 80.0 * g) / (1.0 * n - 80.0 * g)
        assert abs(f[n] - ref) < 1e-12 * abs(ref)


def test_born_and_centred_dipole_closed_forms():
    C = mp.COULOMB_KCAL
    assert abs(C - 332.0637133) < 1e-6
    sph = kirkwood.SphereSolvent(4.0, 1.0, 80.0, 0.125)
    r = sph.reaction(np.zeros((1, 3)), np.array([1.0]), np.zeros((1, 3)),
                     np.zeros((1, 9)))
    born = -(C / 8.0) * (1.0 - 1.0 / (80.0 * 1.5))
    assert abs(0.5 * C * r[0, 0] - born) < 1e-12 * abs(born)
    assert abs(born - (-41.16206)) < 1e-5
    res = solver.solvation(np.zeros((1, 3)), np.zeros(1), np.array([[0, 0, 1.0]]),
                           np.zeros((1, 9)), np.array([1.0]), sph,
                           tol_debye=1e-13)
    f1 = kirkwood.f_coefficients(1, 4.0, 1.0, 80.0, 0.125)[1]
    Rf = -f1 / 64.0
    assert abs(f1 - (-0.9827916)) < 1e-7
    mu = Rf / (1 - Rf)
    assert abs(res["mu_diss"][0, 2] - mu) < 1e-12
    dG = C * 0.5 * f1 / (64.0 * (1 - Rf))
    assert abs(res["dG"] - dG) < 1e-10 * abs(dG)
    assert abs(dG - (-2.589368)) < 1e-6


# --------------------------------------------------------- solver invariants
def test_scaling_invariance_and_nonpolarisable_limit():
    w = workload("sphere_1280")
    sph = kirkwood.SphereSolvent(4.0, 1.0, 80.0, 0.125)
    args = (w["xyz"], w["q"], w["d"], w["Q9"], w["alpha"])
    base = solver.solvation(*args, sph, tol_debye=1e-12)
    lam = 1.7
    sc = solver.solvation(w["xyz"], lam * w["q"], lam * w["d"], lam * w["Q9"],
                          w["alpha"], sph, tol_debye=1e-12)
    assert abs(sc["dG"] - lam ** 2 * base["dG"]) < 1e-9 * abs(sc["dG"])
    assert np.abs(sc["mu_diss"] - lam * base["mu_diss"]).max() < 1e-10
    # alpha = 0: no induced dipoles, only the solvent term survives
    np_ = solver.solvation(w["xyz"], w["q"], w["d"], w["Q9"],
                           np.zeros(8), sph, tol_debye=1e-12)
    assert np.abs(np_["mu_diss"]).max() == 0 and np_["e_pol"] == 0.0
    direct = sph.reaction(w["xyz"], w["q"], w["d"], w["Q9"])
    e = 0.5 * mp.COULOMB_KCAL * solver._apply_D(w["q"], w["d"], w["Q9"], direct)
    assert abs(np_["dG"] - e) < 1e-12 * abs(e)


def test_bem_homogeneous_dielectric_gives_zero():
    """eps_out = eps_in and kappa = 0: no reaction field up to the
    discretisation error, which falls with the panel area."""
    w = workload("sphere_1280")
    vals = []
    for lev in (2, 3):
        v, t = icosphere(lev, 4.0)
        sol = solver.BemSolvent(v, t, 1.0, 1.0, 0.0)
        r = sol.reaction(w["xyz"], w["q"], w["d"], w["Q9"])
        vals.append(np.abs(r[:, 0]).max())
    assert vals[1] < vals[0] / 3 and vals[1] < 2e-3


@pytest.mark.slow
def test_bem_converges_to_kirkwood_cfg0():
    """cfg0 sites: BEM error vs the exact series falls ~4x per subdivision
    (error proportional to the panel area) and the Richardson extrapolant
    is within 1e-4 of the series."""
    w = workload("sphere_1280")
    args = (w["xyz"], w["q"], w["d"], w["Q9"], w["alpha"])
    ref = solver.solvation(*args, kirkwood.SphereSolvent(4.0, 1.0, 80.0, 0.125))["dG"]
    vals = []
    for n in (1280, 5120):
        ww = workload("sphere_%d" % n)
        vals.append(solver.solvation(*args, solver.BemSolvent(
            ww["verts"], ww["tris"], 1.0, 80.0, 0.125))["dG"])
    e0, e1 = vals[0] - ref, vals[1] - ref
    assert 3.5 < e0 / e1 < 4.5
    rich = vals[1] + (vals[1] - vals[0]) / 3.0
    assert abs(rich - ref) < 1e-4 * abs(ref)


# ------------------------------------------------------- vacuum binding leg
def test_vacuum_energy_closed_forms():
    """eq. energy_multipole_polarizable in vacuum: two point charges give
    C q1 q2 / r; a charge facing a neutral polarisable site (no damping)
    gives the ion-induced-dipole energy -C alpha q^2 / (2 r^4), the
    polarisation work being carried by the d-form of the energy."""
    from oracle import solver as osolver, multipoles as omp
    C = omp.COULOMB_KCAL
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 3.0]])
    Z = np.zeros((2, 9))
    d0 = np.zeros((2, 3))
    q = np.array([0.7, -0.4])
    G = osolver.vacuum_energy(xyz, q, d0, Z, np.zeros(2), np.zeros((2, 3)))
    assert abs(G - C * 0.7 * -0.4 / 3.0) < 1e-12 * abs(G)
    q = np.array([0.8, 0.0])
    alpha = np.array([0.0, 1.3])
    grp = np.arange(2)
    mu, _, _ = osolver.scf(xyz, q, d0, Z, alpha, grp, 1.0, 1e30, 0.7, 1e-13, 1000)
    assert abs(mu[1, 2] - 1.3 * 0.8 / 9.0) < 1e-13
    G = osolver.vacuum_energy(xyz, q, d0, Z, alpha, mu, thole_a=1e30)
    assert abs(G - (-C * 1.3 * 0.8 ** 2 / (2 * 3.0 ** 4))) < 1e-10 * abs(G)


def test_total_dipole_units_and_origin():
    """Total dipole (Table "dipole", Debye): a unit charge pair 1 A apart is
    the textbook 4.803 D; a neutral set does not depend on the origin; a
    charged one moves by Q times the origin shift; permanent and induced
    dipoles add as vectors."""
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    q = np.array([-1.0, 1.0])
    z = np.zeros((2, 3))
    p = solver.total_dipole(xyz, q, z, z)
    assert abs(p[2] - 4.80320) < 1e-5 and abs(p[0]) + abs(p[1]) == 0.0
    rng = np.random.default_rng(7)
    xyz = rng.normal(size=(9, 3))
    q = rng.normal(size=9)
    d, mu = rng.normal(size=(9, 3)), rng.normal(size=(9, 3))
    qn = q - q.mean()
    shift = np.array([3.0, -1.0, 2.0])
    a = solver.total_dipole(xyz, qn, d, mu, origin=np.zeros(3))
    b = solver.total_dipole(xyz, qn, d, mu, origin=shift)
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()
    a = solver.total_dipole(xyz, q, d, mu, origin=np.zeros(3))
    b = solver.total_dipole(xyz, q, d, mu, origin=shift)
    assert np.abs((a - b) / mp.DEBYE_PER_EA - q.sum() * shift).max() < 1e-12
    pd = solver.total_dipole(xyz, np.zeros(9), d, z)
    pm = solver.total_dipole(xyz, np.zeros(9), z, mu)
    assert np.abs(pd + pm - solver.total_dipole(xyz, np.zeros(9), d, mu)).max() < 1e-12


def test_vacuum_binding_vanishes_at_separation():
    """G_AB - G_A - G_B tends to the monopole interaction of the two parts
    as they move apart."""
    from oracle import solver as osolver
    rng = np.random.default_rng(4)
    from synth.sites import sites_in_ball
    from synth import random_multipoles
    A = sites_in_ball(rng, 5, 2.0, 1.0)
    B = sites_in_ball(rng, 4, 2.0, 1.0)
    mA = random_multipoles(rng, 5)
    mB = random_multipoles(rng, 4)

    def G(xyz, m):
        q, d, Q9, al = m
        mu, _, _ = osolver.scf(xyz, q, d, Q9, al, np.arange(len(q)), 1.0, 0.39, 0.7, 1e-12, 2000)
        return osolver.vacuum_energy(xyz, q, d, Q9, al, mu)

    gA, gB = G(A, mA), G(B, mB)
    vals = []
    for sep in (10.0, 100.0, 1000.0):
        xyz = np.concatenate([A, B + [sep, 0, 0]])
        m = tuple(np.concatenate([a, b]) for a, b in zip(mA, mB))
        vals.append(G(xyz, m) - gA - gB)
    qA, qB = mA[0].sum(), mB[0].sum()
    from oracle import multipoles as omp
    lead = omp.COULOMB_KCAL * qA * qB
    # the binding energy approaches the monopole term C qA qB / sep, the
    # remainder falling as 1/sep^2 (charge-dipole order)
    e = [abs(v - lead / s) for v, s in zip(vals, (10.0, 100.0, 1000.0))]
    assert e[2] < 1e-2 * abs(lead / 1000.0)
    assert 50 < e[1] / e[2] < 200


# ------------------------------------------------------------ Stern layer
def test_stern_coefficients_reduce_and_solve_the_matching():
    """Kirkwood coefficients with an ion-exclusion shell: a shell of zero
    thickness gives the sphere's coefficients; a shell of the outer medium
    without salt changes nothing; and each f_n solves the four matching
    conditions (phi and eps dphi/dr continuous at a and b) written as a
    linear system."""
    from oracle import kirkwood as kw
    a, b, e1, es, eo, kap = 4.0, 5.0, 4.0, 30.0, 80.0, 0.125
    f_sph = kw.f_coefficients(25, a, e1, eo, kap)
    assert np.abs(kw.f_coefficients(25, a, e1, eo, kap, b=a, eps_stern=es) - f_sph).max() < 1e-13
    assert np.abs(kw.f_coefficients(25, a, e1, eo, 0.0, b=b, eps_stern=eo)
                  - kw.f_coefficients(25, a, e1, eo, 0.0)).max() < 1e-13
    f = kw.f_coefficients(25, a, e1, eo, kap, b=b, eps_stern=es)
    g = kw.g_coefficients(25, kap * b)
    for n in range(0, 26, 5):
        # unknowns A, B, C, D (interior r^n, shell r^n and r^-(n+1), exterior
        # value at b); source s r^-(n+1) with s = 1
        M = np.array([
            [a ** n, -a ** n, -a ** -(n + 1), 0.0],
            [e1 * n * a ** (n - 1) if n else 0.0, -es * n * a ** (n - 1) if n else 0.0,
             es * (n + 1) * a ** -(n + 2), 0.0],
            [0.0, b ** n, b ** -(n + 1), -1.0],
            [0.0, es * n * b ** (n - 1) if n else 0.0, -es * (n + 1) * b ** -(n + 2),
             -eo * g[n] / b]])
        rhs = np.array([-a ** -(n + 1), e1 * (n + 1) * a ** -(n + 2), 0.0, 0.0])
        A = np.linalg.solve(M, rhs)[0]
        assert abs(A * a ** (2 * n + 1) - f[n]) < 1e-10 * max(1.0, abs(f[n]))


@pytest.mark.slow
def test_stern_bem_converges_to_series():
    """The two-surface system on icospheres (4 A and 5 A) approaches the
    Stern-layer series for point charges at O(h^2): error ratio ~4 per
    subdivision."""
    from oracle import kirkwood as kw, stern, solver as osolver
    from synth import icosphere
    xyz = np.array([[0.0, 0, 0], [2.0, 0, 0], [0, 1.5, 0.5]])
    q = np.array([1.0, -0.5, 0.3])
    Z3, Z9, al = np.zeros((3, 3)), np.zeros((3, 9)), np.zeros(3)
    ref = osolver.solvation(xyz, q, Z3, Z9, al,
                            kw.SphereSolvent(4.0, 4.0, 80.0, 0.125, b=5.0, eps_stern=80.0),
                            eps_in=4.0)["dG"]
    errs = []
    for lev in (2, 3):
        v1, t1 = icosphere(lev, 4.0)
        v2, t2 = icosphere(lev, 5.0)
        sb = stern.SternBemSolvent(v1, t1, v2, t2, 4.0, 80.0, 80.0, 0.125)
        errs.append(abs(osolver.solvation(xyz, q, Z3, Z9, al, sb, eps_in=4.0)["dG"] - ref) / abs(ref))
    assert errs[0] < 0.03 and 3.5 < errs[0] / errs[1] < 4.6
