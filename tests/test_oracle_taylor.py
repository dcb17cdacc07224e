"""Pins of the oracle's Taylor coefficients (truncated power series of the
Laplace and Yukawa kernels about a box centre) against direct evaluation:
the series reproduces G(x, y_c + h) with an O(|h|^(P+1)) remainder, its
first coefficients are the kernel and its finite-difference gradient, the
kappa -> 0 limit is the Laplace series, and a box expansion of many sources
approaches the direct sum as the box shrinks.  CPU only."""

import numpy as np

from oracle import taylor


def _series(c, ks, h):
    return sum(cc * h[0] ** k[0] * h[1] ** k[1] * h[2] ** k[2] for cc, k in zip(c, ks))


def test_taylor_remainder_order():
    x = np.array([2.1, -0.7, 1.3])
    yc = np.array([0.2, 0.1, -0.4])
    kappa = 0.3
    for P in (2, 4):
        ks = taylor.multi_indices(P)
        cl = taylor.laplace_coefficients(x, yc, P)
        cy = taylor.yukawa_coefficients(x, yc, P, kappa)
        errs_l, errs_y = [], []
        for s in (0.1, 0.05):
            h = s * np.array([0.6, -0.3, 0.74])
            r = np.linalg.norm(x - yc - h)
            errs_l.append(abs(_series(cl, ks, h) - 1 / r))
            errs_y.append(abs(_series(cy, ks, h) - np.exp(-kappa * r) / r))
        # halving h divides the remainder by ~2^(P+1)
        assert errs_l[0] / errs_l[1] > 0.7 * 2 ** (P + 1)
        assert errs_y[0] / errs_y[1] > 0.7 * 2 ** (P + 1)


def test_taylor_low_order_coefficients():
    x = np.array([1.0, 2.0, -0.5])
    yc = np.array([-0.3, 0.4, 0.2])
    kappa = 0.5
    cy = taylor.yukawa_coefficients(x, yc, 3, kappa)
    G = lambda y: np.exp(-kappa * np.linalg.norm(x - y)) / np.linalg.norm(x - y)
    assert abs(cy[0] - G(yc)) < 1e-15
    h = 1e-5
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (G(yc + e) - G(yc - e)) / (2 * h)
        assert abs(cy[1 + a] - fd) < 1e-9


def test_taylor_yukawa_to_laplace():
    x = np.array([1.5, -1.0, 0.4])
    yc = np.zeros(3)
    cl = taylor.laplace_coefficients(x, yc, 5)
    cy = taylor.yukawa_coefficients(x, yc, 5, 1e-9)
    assert np.abs(cy - cl).max() < 1e-8


def test_box_expansion_converges_to_direct_sum():
    rng = np.random.default_rng(0)
    x = np.array([6.0, 1.0, -2.0])
    kappa = 0.125
    P = 4
    ks = taylor.multi_indices(P)
    errs = []
    for size in (1.0, 0.5, 0.25):
        rng = np.random.default_rng(0)
        pts = rng.uniform(-size, size, size=(40, 3))
        nrm = rng.normal(size=(40, 3))
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        sv, sk = rng.normal(size=40), rng.normal(size=40)
        m, mk = taylor.moments(pts, nrm, sv, sk, np.zeros(3), P)
        cy = taylor.yukawa_coefficients(x, np.zeros(3), P, kappa)
        R = x - pts
        r = np.linalg.norm(R, axis=1)
        e = np.exp(-kappa * r)
        direct_v = np.sum(sv * e / r)
        direct_k = np.sum(sk * np.einsum("ij,ij->i", nrm, R) * (1 + kappa * r) * e / r ** 3)
        errs.append((abs(cy @ m - direct_v) / abs(direct_v),
                     abs(cy @ mk - direct_k) / abs(direct_k)))
    # single layer: remainder ~ (size/R)^(P+1), 32x per halving; double
    # layer (a derivative of the expansion) one order less
    assert errs[1][0] < errs[0][0] / 16 and errs[2][0] < errs[1][0] / 16
    assert errs[2][1] < errs[0][1] / 30 and errs[2][1] < errs[1][1]
    assert errs[2][0] < 1e-6 and errs[2][1] < 1e-5
