"""Boundary-integral operators, linear system and site readout (test
infrastructure only).

System (eq. integral_eq, Yoon-Lenhoff), unknowns x = [phi; dphi/dn] on the
panels, normal pointing out of the molecule:
    [ 1/2 I + K_L     -V_L          ] [phi ]   [ f ]
    [ 1/2 I - K_Y     (e1/e2) V_Y   ] [dphi] = [ 0 ]
f is the multipole potential divided by eps_in (eq. rhs_multipole).

The reaction potential at interior points is
    phi_solv = -K_L(phi) + V_L(dphi)                      (eq. pot_solvent)
with first and second derivatives in the evaluation point (eq. Efield_solv,
eq. ddphi, appendix).  All values here are in the normalisation of the
integral equation, G = 1/(4 pi r); the physical potential in e/A is 4 pi
times larger.
"""

import ctypes
import os
import subprocess

import numpy as np
import scipy.linalg

from . import quadrature, geometry

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bie_c.c")
_LIB = os.path.join(_HERE, "_bie_c.so")
_lib = None


def build(force=False):
    """Compile the oracle's C loops with gcc (-O2, OpenMP, IEEE FP64)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".%d.tmp" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", "-o",
                               tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
    return _lib


class _CMesh(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int),
                ("verts", ctypes.c_void_p), ("tris", ctypes.c_void_p),
                ("cen", ctypes.c_void_p), ("nrm", ctypes.c_void_p),
                ("area", ctypes.c_void_p),
                ("nf", ctypes.c_int), ("fb", ctypes.c_void_p), ("fw", ctypes.c_void_p),
                ("nn", ctypes.c_int), ("nb", ctypes.c_void_p), ("nw", ctypes.c_void_p),
                ("ngl", ctypes.c_int), ("glx", ctypes.c_void_p), ("glw", ctypes.c_void_p),
                ("kappa", ctypes.c_double), ("eta", ctypes.c_double)]


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Mesh:
    """A triangle mesh with its quadrature data, ready for the C loops.

    kappa in 1/A, eta = near-singular threshold factor (near iff
    |c_i - c_j| < eta sqrt(A_i)), far = number of far-field nodes (1 or 3),
    ngl = Gauss-Legendre nodes per edge for the singular Yukawa remainder.
    """

    def __init__(self, verts, tris, kappa, eta=2.0, far=3, ngl=16):
        self.verts = np.ascontiguousarray(verts, dtype=np.float64)
        self.tris = np.ascontiguousarray(tris, dtype=np.int32)
        self.N = len(self.tris)
        g = geometry.panels(self.verts, self.tris)
        self.geo = g
        self.cen = np.ascontiguousarray(g["centroid"])
        self.nrm = np.ascontiguousarray(g["normal"])
        self.area = np.ascontiguousarray(g["area"])
        fb, fw = quadrature.far_rule(far)
        nb, nw = quadrature.tri19()
        glx, glw = quadrature.gauss_legendre(ngl)
        self._keep = [np.ascontiguousarray(a, dtype=np.float64)
                      for a in (fb, fw, nb, nw, glx, glw)]
        fb, fw, nb, nw, glx, glw = self._keep
        self.kappa, self.eta = float(kappa), float(eta)
        self.c = _CMesh(self.N, _p(self.verts).value, _p(self.tris).value,
                        _p(self.cen).value, _p(self.nrm).value,
                        _p(self.area).value,
                        len(fw), _p(fb).value, _p(fw).value,
                        len(nw), _p(nb).value, _p(nw).value,
                        len(glw), _p(glx).value, _p(glw).value,
                        self.kappa, self.eta)

    # -- operators -----------------------------------------------------
    def dense_operators(self, rows=None):
        """Dense V_L, K_L, V_Y, K_Y (rows i0:i1 of each, default all)."""
        i0, i1 = (0, self.N) if rows is None else rows
        out = [np.empty((i1 - i0, self.N)) for _ in range(4)]
        _load().orc_entries(ctypes.byref(self.c), ctypes.c_int(i0),
                            ctypes.c_int(i1), *[_p(a) for a in out])
        return out

    def operator_sums(self, phi, dphi, rows=None):
        """[n,4] = (V_L dphi, K_L phi, V_Y dphi, K_Y phi) for rows i0:i1."""
        i0, i1 = (0, self.N) if rows is None else rows
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        dphi = np.ascontiguousarray(dphi, dtype=np.float64)
        out = np.empty((i1 - i0, 4))
        _load().orc_operator_sums(ctypes.byref(self.c), ctypes.c_int(i0),
                                  ctypes.c_int(i1), _p(phi), _p(dphi), _p(out))
        return out

    def near_correction_sums(self, phi, dphi, rows=None):
        """[n,4] near-field corrections (method's entry minus far-rule entry
        over the singular and near-singular pairs) applied to the densities,
        in the order (V_L dphi, K_L phi, V_Y dphi, K_Y phi), rows i0:i1."""
        i0, i1 = (0, self.N) if rows is None else rows
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        dphi = np.ascontiguousarray(dphi, dtype=np.float64)
        out = np.empty((i1 - i0, 4))
        _load().orc_near_correction_sums(ctypes.byref(self.c), ctypes.c_int(i0),
                                         ctypes.c_int(i1), _p(phi), _p(dphi), _p(out))
        return out

    def self_integrals(self, j, point=None):
        c = self.cen[j] if point is None else np.asarray(point, dtype=np.float64)
        c = np.ascontiguousarray(c)
        out = np.empty(2)
        _load().orc_self_integrals(ctypes.byref(self.c), ctypes.c_int(j),
                                   _p(c), _p(out))
        return out

    def readout(self, x, points):
        """Reaction potential data [M,10] at interior points:
        phi_solv, grad (3), and second derivatives xx, xy, xz, yy, yz, zz."""
        N = self.N
        x = np.asarray(x, dtype=np.float64)
        phi = np.ascontiguousarray(x[:N])
        dphi = np.ascontiguousarray(x[N:])
        pts = np.ascontiguousarray(points, dtype=np.float64)
        out = np.empty((len(pts), 10))
        _load().orc_readout(ctypes.byref(self.c), ctypes.c_int(len(pts)),
                            _p(pts), _p(phi), _p(dphi), _p(out))
        return out


def system_apply(sums, phi, eps_in, eps_out):
    """Combine operator sums into y = A x (eq. integral_eq)."""
    vl, kl, vy, ky = sums[:, 0], sums[:, 1], sums[:, 2], sums[:, 3]
    y1 = 0.5 * phi + kl - vl
    y2 = 0.5 * phi - ky + (eps_in / eps_out) * vy
    return np.concatenate([y1, y2])


def matvec(mesh, x, eps_in, eps_out, rows=None):
    N = mesh.N
    s = mesh.operator_sums(x[:N], x[N:])
    return system_apply(s, x[:N], eps_in, eps_out)


def dense_system(mesh, eps_in, eps_out):
    VL, KL, VY, KY = mesh.dense_operators()
    N = mesh.N
    I = np.eye(N)
    A = np.empty((2 * N, 2 * N))
    A[:N, :N] = 0.5 * I + KL
    A[:N, N:] = -VL
    A[N:, :N] = 0.5 * I - KY
    A[N:, N:] = (eps_in / eps_out) * VY
    return A


def lu_solve(A, b):
    return scipy.linalg.lu_solve(scipy.linalg.lu_factor(A), b)


def gmres(apply, b, x0=None, restart=50, tol=1e-12, maxit=2000):
    """Plain restarted GMRES (Saad-Schultz) with modified Gram-Schmidt and
    Givens rotations, no preconditioner.  Stops on the true relative
    residual |b - A x| / |b| <= tol checked at every restart.
    Returns (x, iterations, relres)."""
    n = len(b)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), 0, 0.0
    it = 0
    while True:
        r = b - apply(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol or it >= maxit:
            return x, it, beta / bnorm
        V = np.zeros((restart + 1, n))
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k_done = 0
        for k in range(restart):
            w = apply(V[k])
            for i in range(k + 1):
                H[i, k] = w @ V[i]
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0:
                V[k + 1] = w / H[k + 1, k]
            for i in range(k):
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = H[k, k] / den, H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            it += 1
            k_done = k + 1
            if abs(g[k + 1]) / bnorm <= 0.1 * tol or it >= maxit:
                break
        y = scipy.linalg.solve_triangular(H[:k_done, :k_done], g[:k_done])
        x = x + V[:k_done].T @ y
