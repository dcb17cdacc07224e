"""Taylor coefficients of the free-space kernels about a box centre (test
infrastructure only).

The treecode (section "The treecode algorithm") expands G(x, y) in the
source point about the box centre y_c:  G(x, y_c + h) = sum_k a_k h^k with
a_k = (1/k!) d^k G / dy^k (x, y_c), for |k| <= P.  The paper cites the
Cartesian recurrences of Lindsay-Krasny (Laplace) and Li-Johnston-Krasny
(Yukawa) without printing them.  This module computes the same
coefficients by a different route, truncated multivariate power-series
("jet") arithmetic: with D = x - y_c,
    u(h) = |D - h|^2 = |D|^2 - 2 D.h + |h|^2        (exact polynomial)
    G_L  = u^{-1/2},   G_Y = exp(-kappa u^{1/2}) u^{-1/2}
using the binomial series for powers and the exponential series, all
truncated at total degree P.  Coefficients are ordered by total degree,
then by the x exponent descending, then the y exponent descending.
Kernels without the 1/(4 pi) factor.
"""

import math

import numpy as np


def multi_indices(P):
    out = []
    for s in range(P + 1):
        for i in range(s, -1, -1):
            for j in range(s - i, -1, -1):
                out.append((i, j, s - i - j))
    return out


class Jet:
    """Truncated power series in three variables, degree <= P."""

    def __init__(self, P, coef=None):
        self.P = P
        self.ks = multi_indices(P)
        self.index = {k: n for n, k in enumerate(self.ks)}
        self.c = np.zeros(len(self.ks)) if coef is None else np.asarray(coef, float)

    def new(self, coef=None):
        j = Jet.__new__(Jet)
        j.P, j.ks, j.index = self.P, self.ks, self.index
        j.c = np.zeros(len(self.ks)) if coef is None else coef
        return j

    def __add__(self, o):
        if isinstance(o, Jet):
            return self.new(self.c + o.c)
        c = self.c.copy()
        c[0] += o
        return self.new(c)

    def __mul__(self, o):
        if not isinstance(o, Jet):
            return self.new(self.c * o)
        out = np.zeros_like(self.c)
        for n1, k1 in enumerate(self.ks):
            if self.c[n1] == 0.0:
                continue
            for n2, k2 in enumerate(o.ks):
                s = (k1[0] + k2[0], k1[1] + k2[1], k1[2] + k2[2])
                if sum(s) <= self.P:
                    out[self.index[s]] += self.c[n1] * o.c[n2]
        return self.new(out)

    __rmul__ = __mul__
    __radd__ = __add__

    def power(self, alpha):
        """self^alpha by the binomial series about the constant term."""
        c0 = self.c[0]
        t = self.new(self.c / c0)
        t.c[0] = 0.0
        out = self.new()
        out.c[0] = 1.0
        term = self.new()
        term.c[0] = 1.0
        coef = 1.0
        for n in range(1, self.P + 1):
            coef *= (alpha - n + 1) / n
            term = term * t
            out = out + term * coef
        return out * (c0 ** alpha)

    def exp(self):
        c0 = self.c[0]
        t = self.new(self.c.copy())
        t.c[0] = 0.0
        out = self.new()
        out.c[0] = 1.0
        term = self.new()
        term.c[0] = 1.0
        for n in range(1, self.P + 1):
            term = term * t * (1.0 / n)
            out = out + term
        return out * math.exp(c0)


def _u_jet(D, P):
    u = Jet(P)
    u.c[0] = float(D @ D)
    for a in range(3):
        e = [0, 0, 0]
        e[a] = 1
        u.c[u.index[tuple(e)]] = -2.0 * D[a]
        e[a] = 2
        u.c[u.index[tuple(e)]] = 1.0
    return u


def laplace_coefficients(x, yc, P):
    D = np.asarray(x, float) - np.asarray(yc, float)
    return _u_jet(D, P).power(-0.5).c


def yukawa_coefficients(x, yc, P, kappa):
    D = np.asarray(x, float) - np.asarray(yc, float)
    u = _u_jet(D, P)
    return ((u.power(0.5) * (-kappa)).exp() * u.power(-0.5)).c


def moments(points, normals, sv, sk, yc, P):
    """Single-layer m_k = sum sv h^k and double-layer
    mK_k = sum sk sum_a k_a n_a h^(k - e_a), h = y - yc."""
    ks = multi_indices(P)
    h = np.asarray(points, float) - np.asarray(yc, float)
    m = np.zeros(len(ks))
    mk = np.zeros(len(ks))
    for n, k in enumerate(ks):
        m[n] = np.sum(sv * h[:, 0] ** k[0] * h[:, 1] ** k[1] * h[:, 2] ** k[2])
        acc = np.zeros(len(h))
        for a in range(3):
            if k[a] == 0:
                continue
            km = list(k)
            km[a] -= 1
            acc += k[a] * normals[:, a] * h[:, 0] ** km[0] * h[:, 1] ** km[1] * h[:, 2] ** km[2]
        mk[n] = np.sum(sk * acc)
    return m, mk


# ------------------------------------------------------------------ batches
# The same truncated power series for many expansion points at once:
# coefficient arrays of shape [ncoef, n], one column per (target, centre)
# pair.  Used by the oracle's treecode product, where the scalar Jet would
# be too slow; pinned against the scalar functions above.

def _product_table(P):
    """For every coefficient n of a product: the index pairs (n1, n2) of
    the factors' coefficients whose multi-indices add up to it."""
    ks = multi_indices(P)
    index = {k: n for n, k in enumerate(ks)}
    terms = [([], []) for _ in ks]
    for n1, k1 in enumerate(ks):
        for n2, k2 in enumerate(ks):
            s = (k1[0] + k2[0], k1[1] + k2[1], k1[2] + k2[2])
            if sum(s) <= P:
                terms[index[s]][0].append(n1)
                terms[index[s]][1].append(n2)
    return [(np.array(a), np.array(b)) for a, b in terms]


class BatchJet:
    """Truncated series in three variables for n expansion points."""

    _tables = {}

    def __init__(self, P, c):
        self.P = P
        self.c = c
        if P not in BatchJet._tables:
            BatchJet._tables[P] = _product_table(P)

    def __mul__(self, o):
        if not isinstance(o, BatchJet):
            return BatchJet(self.P, self.c * o)
        out = np.empty_like(self.c)
        for n, (a, b) in enumerate(BatchJet._tables[self.P]):
            out[n] = np.einsum("ij,ij->j", self.c[a], o.c[b])
        return BatchJet(self.P, out)

    __rmul__ = __mul__

    def __add__(self, o):
        return BatchJet(self.P, self.c + o.c)

    def _unit(self):
        u = np.zeros_like(self.c)
        u[0] = 1.0
        return BatchJet(self.P, u)

    def power(self, alpha):
        c0 = self.c[0].copy()
        t = BatchJet(self.P, self.c / c0)
        t.c[0] = 0.0
        out, term, coef = self._unit(), self._unit(), 1.0
        for n in range(1, self.P + 1):
            coef *= (alpha - n + 1) / n
            term = term * t
            out = out + term * coef
        return out * (c0 ** alpha)

    def exp(self):
        c0 = self.c[0].copy()
        t = BatchJet(self.P, self.c.copy())
        t.c[0] = 0.0
        out, term = self._unit(), self._unit()
        for n in range(1, self.P + 1):
            term = term * t * (1.0 / n)
            out = out + term
        return out * np.exp(c0)


def _u_batch(D, P):
    """u(h) = |D - h|^2 for D [n, 3] as a batch of series."""
    ks = multi_indices(P)
    index = {k: n for n, k in enumerate(ks)}
    c = np.zeros((len(ks), len(D)))
    c[0] = np.einsum("ij,ij->i", D, D)
    for a in range(3):
        e = [0, 0, 0]
        e[a] = 1
        c[index[tuple(e)]] = -2.0 * D[:, a]
        if P >= 2:
            e[a] = 2
            c[index[tuple(e)]] = 1.0
    return BatchJet(P, c)


def laplace_coefficients_batch(D, P):
    """Coefficients [ncoef, n] of 1/|D - h| for D = x - y_c [n, 3]."""
    return _u_batch(np.asarray(D, float), P).power(-0.5).c


def yukawa_coefficients_batch(D, P, kappa):
    """Coefficients [ncoef, n] of exp(-kappa |D - h|)/|D - h|."""
    u = _u_batch(np.asarray(D, float), P)
    return ((u.power(0.5) * (-kappa)).exp() * u.power(-0.5)).c
