"""Quadrature rules used by the oracle (test infrastructure only).

Far-field rule (Algorithmic details, "boundary element method": 1, 3 or 4
Gauss nodes far from the collocation point).  The 3-point rule read here is
the interior degree-2 rule with barycentric nodes (2/3, 1/6, 1/6) and
permutations, equal weights 1/3.  The 1-point rule is the centroid.

Near-singular rule (same passage: 19 Gauss nodes inside the 2 sqrt(A)
threshold).  The paper does not print the nodes; the reading taken is the
fully symmetric degree-9 rule with orbit structure
  1 centroid + 4 orbits (a, a, 1-2a) + 1 orbit (a, b, 1-a-b)   (19 nodes),
whose 12 unknowns are fixed by exactness on every monomial of degree <= 9.
It is obtained here by solving those moment equations (nonlinear least
squares from a rough start, then Gauss-Newton at 40 significant digits),
and accepted only if all weights are positive, all nodes interior and
every moment is exact to 1e-30 before rounding to double.

Weights are normalised to sum to 1 (multiply by the panel area).
"""

import math
import numpy as np
from scipy.optimize import least_squares


def tri1():
    return np.array([[1 / 3, 1 / 3, 1 / 3]]), np.array([1.0])


def tri3():
    b = np.array([[2 / 3, 1 / 6, 1 / 6],
                  [1 / 6, 2 / 3, 1 / 6],
                  [1 / 6, 1 / 6, 2 / 3]])
    return b, np.full(3, 1.0 / 3.0)


def exact_moment(i, j):
    """(1/area) * integral of x^i y^j over the reference triangle
    (0,0), (1,0), (0,1)."""
    return 2.0 * math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)


def _expand19(t):
    w0 = t[0]
    pts, wts = [(1 / 3, 1 / 3, 1 / 3)], [w0]
    for k in range(4):
        a, w = t[1 + 2 * k], t[2 + 2 * k]
        for p in ((a, a, 1 - 2 * a), (a, 1 - 2 * a, a), (1 - 2 * a, a, a)):
            pts.append(p)
            wts.append(w)
    a, b, w = t[9], t[10], t[11]
    c = 1 - a - b
    for p in ((a, b, c), (a, c, b), (b, a, c), (b, c, a), (c, a, b), (c, b, a)):
        pts.append(p)
        wts.append(w)
    return np.array(pts), np.array(wts)


def _residual19(t, deg=9):
    bary, w = _expand19(t)
    x, y = bary[:, 1], bary[:, 2]
    r = []
    for i in range(deg + 1):
        for j in range(deg + 1 - i):
            r.append(np.sum(w * x ** i * y ** j) - exact_moment(i, j))
    return np.array(r)


_RULE19 = None


def _refine19(t, digits=40, iters=6):
    """Gauss-Newton on the moment equations in mpmath arithmetic.  The
    system is ill-conditioned (a double-precision solution with residual
    ~1e-16 can sit ~1e-11 away from the rule), so the rule is refined at
    `digits` decimal digits and each barycentric coordinate and weight is
    rounded to double once, at the end."""
    import mpmath as mp
    with mp.workdps(digits):
        def nodes(t):
            third = mp.mpf(1) / 3
            pts, wts = [(third, third)], [t[0]]
            for k in range(4):
                a, w = t[1 + 2 * k], t[2 + 2 * k]
                for p in ((a, 1 - 2 * a), (1 - 2 * a, a), (a, a)):
                    pts.append(p)
                    wts.append(w)
            a, b, w = t[9], t[10], t[11]
            c = 1 - a - b
            for p in ((b, c), (c, b), (a, c), (c, a), (a, b), (b, a)):
                pts.append(p)
                wts.append(w)
            return pts, wts

        def residual(t):
            pts, wts = nodes(t)
            r = []
            for i in range(10):
                for j in range(10 - i):
                    ex = 2 * mp.factorial(i) * mp.factorial(j) / mp.factorial(i + j + 2)
                    r.append(mp.fsum(w * x ** i * y ** j for w, (x, y) in zip(wts, pts)) - ex)
            return mp.matrix(r)

        t = mp.matrix([mp.mpf(float(v)) for v in t])
        h = mp.mpf(10) ** (-(digits * 2) // 3)
        for _ in range(iters):
            r = residual(t)
            J = mp.matrix(len(r), 12)
            for k in range(12):
                tp = t.copy()
                tp[k] += h
                rp = residual(tp)
                for i in range(len(r)):
                    J[i, k] = (rp[i] - r[i]) / h
            t = t + mp.lu_solve(J.T * J, -(J.T * r))
        res = max(abs(v) for v in residual(t))
        pts, wts = nodes(t)
        bary = np.array([[float(1 - x - y), float(x), float(y)] for x, y in pts])
        w = np.array([float(v) for v in wts])
        return bary, w, float(res)


def tri19():
    """Barycentric nodes [19,3] and weights [19] of the degree-9 rule."""
    global _RULE19
    if _RULE19 is None:
        t0 = np.array([0.1, 0.49, 0.03, 0.44, 0.08, 0.19, 0.08, 0.045,
                       0.025, 0.037, 0.22, 0.043])
        sol = least_squares(_residual19, t0, xtol=1e-15, ftol=1e-15,
                            gtol=1e-15, method="lm")
        bary, w, res = _refine19(sol.x)
        if not (res < 1e-30 and (w > 0).all() and (bary > 0).all()):
            raise RuntimeError("19-point rule did not converge (res=%g)" % res)
        _RULE19 = (bary, w)
    return _RULE19


def gauss_legendre(n):
    """Nodes and weights on [-1, 1]."""
    return np.polynomial.legendre.leggauss(n)


def far_rule(k):
    if k == 1:
        return tri1()
    if k == 3:
        return tri3()
    raise ValueError("far rule with %d nodes not provided" % k)
