"""Pins of the oracle's treecode product and of its site readout against
facts that do not come from the oracle itself.  CPU only.

Treecode (section "The treecode algorithm"):
  * theta -> 0 accepts no box, so the product is the direct oracle product
    (far rule plus the near-field corrections) to rounding;
  * the error against the direct product falls geometrically with the
    Taylor order, separately for the single layer (x = [0; dphi]) and the
    double layer (x = [phi; 0]) -- a dropped term, a wrong sign or a wrong
    index in the moments or coefficients stops that convergence;
  * kappa -> 0 turns the Yukawa sums into the Laplace ones;
  * the batched series coefficients equal the scalar ones, which are
    pinned against direct evaluation in test_oracle_taylor.py.
Readout (eq. pot_solvent, eq. Efield_solv, eq. ddphi): the field is the
central difference of the potential, the field gradient that of the
field, and the trace of the second derivatives vanishes (every term is
harmonic away from its node)."""

import numpy as np
import pytest

from oracle import bie, taylor, treecode
from synth import workload


@pytest.fixture(scope="module")
def sph1280():
    w = workload("sphere_1280")
    return w, bie.Mesh(w["verts"], w["tris"], 0.125)


def _ragged():
    from synth import saw_molecule, random_multipoles, molecule_mesh
    rng = np.random.default_rng(7)
    pos, rad = saw_molecule(rng, 23, rg_target=4.0)
    q, d, Q9, alpha = random_multipoles(rng, 23)
    verts, tris = molecule_mesh(pos, rad, 1.0)
    verts = verts + np.random.default_rng(70).normal(scale=1e-3, size=verts.shape)
    return dict(verts=verts, tris=tris, xyz=pos)


def _smooth(m):
    c = m.cen - m.cen.mean(0)
    c = c / np.linalg.norm(c, axis=1, keepdims=True)
    return np.concatenate([1 + c[:, 2] + c[:, 0] * c[:, 1], 0.3 - c[:, 1]])


def test_theta_zero_is_the_direct_product(sph1280):
    w, m = sph1280
    x = np.random.default_rng(1).normal(size=2 * m.N)
    ref = bie.matvec(m, x, 1.0, 80.0)
    for leaf in (16, 300):
        y = treecode.Treecode(m, 1e-9, 4, leaf).matvec(x, 1.0, 80.0)
        assert np.abs(y - ref).max() < 1e-13 * np.abs(ref).max()


def test_treecode_converges_with_order_per_layer(sph1280):
    w, m = sph1280
    N = m.N
    xs = _smooth(m)
    cases = {"single": np.concatenate([np.zeros(N), xs[N:]]),
             "double": np.concatenate([xs[:N], np.zeros(N)])}
    for name, x in cases.items():
        ref = m.operator_sums(x[:N], x[N:])
        col = [0, 2] if name == "single" else [1, 3]
        errs = []
        for P in (1, 2, 3, 4):
            s = treecode.Treecode(m, 0.5, P, 16).operator_sums(x[:N], x[N:])
            errs.append(np.linalg.norm(s[:, col] - ref[:, col]) / np.linalg.norm(ref[:, col]))
        print(name, errs)
        # theta = 0.5: the remainder falls with every degree, and by well
        # over theta^2 every two degrees (on the sphere's symmetric boxes the
        # odd degrees gain less than the even ones)
        for a, b in zip(errs, errs[1:]):
            assert b < a
        for a, b in zip(errs, errs[2:]):
            assert b < 0.3 * a


def test_double_layer_order_is_one_above(sph1280):
    """The double layer carried to degree P + 1 of its moments is more
    accurate than at degree P (its moments of degree |k| hold h^(|k|-1));
    the single layer is unchanged."""
    w, m = sph1280
    N = m.N
    x = _smooth(m)
    ref = m.operator_sums(x[:N], x[N:])
    lo = treecode.Treecode(m, 0.5, 2, 16, double_layer_order=2).operator_sums(x[:N], x[N:])
    hi = treecode.Treecode(m, 0.5, 2, 16).operator_sums(x[:N], x[N:])
    err = lambda s, c: np.linalg.norm(s[:, c] - ref[:, c]) / np.linalg.norm(ref[:, c])
    assert abs(err(lo, [0, 2]) - err(hi, [0, 2])) < 1e-15
    assert err(hi, [1, 3]) < 0.2 * err(lo, [1, 3])


def test_yukawa_sums_reduce_to_laplace():
    w = _ragged()
    m = bie.Mesh(w["verts"], w["tris"], 1e-12)
    N = m.N
    x = np.random.default_rng(2).normal(size=2 * N)
    s = treecode.Treecode(m, 0.5, 3, 16).operator_sums(x[:N], x[N:])
    assert np.abs(s[:, 2] - s[:, 0]).max() < 1e-9 * np.abs(s[:, 0]).max()
    assert np.abs(s[:, 3] - s[:, 1]).max() < 1e-9 * np.abs(s[:, 1]).max()


def test_row_subset_equals_full_product():
    w = _ragged()
    m = bie.Mesh(w["verts"], w["tris"], 0.125)
    x = np.random.default_rng(3).normal(size=2 * m.N)
    tc = treecode.Treecode(m, 0.5, 4, 16)
    full = tc.matvec(x, 1.0, 80.0)
    rows = np.sort(np.random.default_rng(4).choice(m.N, 40, replace=False))
    sub = tc.matvec(x, 1.0, 80.0, rows=rows)
    assert np.array_equal(sub, np.concatenate([full[:m.N][rows], full[m.N:][rows]]))


def test_batched_coefficients_equal_scalar():
    rng = np.random.default_rng(5)
    D = rng.normal(size=(6, 3)) * 2.5
    for P in (2, 5, 7):
        bl = taylor.laplace_coefficients_batch(D, P)
        by = taylor.yukawa_coefficients_batch(D, P, 0.125)
        for i in range(len(D)):
            sl = taylor.laplace_coefficients(D[i], np.zeros(3), P)
            sy = taylor.yukawa_coefficients(D[i], np.zeros(3), P, 0.125)
            assert np.abs(bl[:, i] - sl).max() < 1e-14 * np.abs(sl).max()
            assert np.abs(by[:, i] - sy).max() < 1e-14 * np.abs(sy).max()


# ------------------------------------------------------------ site readout
def _interior_points(m, xyz, rng, n):
    """Points away from every near-rule threshold by more than the FD step."""
    pts = []
    for p in xyz:
        for _ in range(20):
            q = p + rng.normal(scale=0.2, size=3)
            d = np.linalg.norm(m.cen - q, axis=1)
            thr = m.eta * np.sqrt(m.area)
            inside = np.linalg.norm(q - m.cen.mean(0)) < np.linalg.norm(p - m.cen.mean(0)) + 0.5
            if inside and np.abs(d - thr).min() > 1e-3 and d.min() > 0.3:
                pts.append(q)
                break
        if len(pts) == n:
            break
    return np.array(pts)


@pytest.mark.parametrize("case", ["sphere_1280", "ragged"])
def test_readout_derivatives_are_consistent(case, sph1280):
    if case == "sphere_1280":
        w, m = sph1280
    else:
        w = _ragged()
        m = bie.Mesh(w["verts"], w["tris"], 0.125)
    rng = np.random.default_rng(11)
    x = rng.normal(size=2 * m.N)
    pts = _interior_points(m, w["xyz"], rng, 6)
    assert len(pts) >= 4
    out = m.readout(x, pts)
    h = 1e-5
    # second-derivative slots xx, xy, xz, yy, yz, zz
    slot = {(0, 0): 4, (0, 1): 5, (0, 2): 6, (1, 1): 7, (1, 2): 8, (2, 2): 9}
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        op, om = m.readout(x, pts + e), m.readout(x, pts - e)
        fd_phi = (op[:, 0] - om[:, 0]) / (2 * h)
        assert np.abs(fd_phi - out[:, 1 + a]).max() < 1e-7 * np.abs(out[:, 1:4]).max()
        for b in range(3):
            fd = (op[:, 1 + b] - om[:, 1 + b]) / (2 * h)
            got = out[:, slot[(min(a, b), max(a, b))]]
            assert np.abs(fd - got).max() < 1e-6 * np.abs(out[:, 4:]).max()
    trace = out[:, 4] + out[:, 7] + out[:, 9]
    assert np.abs(trace).max() < 1e-12 * np.abs(out[:, 4:]).max()
