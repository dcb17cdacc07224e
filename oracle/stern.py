"""Two-surface boundary-integral system with an ion-exclusion (Stern)
layer, as in the paper's spherical-cavity verification case: region 1
inside the molecular surface G1 (eps_in, the multipoles), region 2 between
G1 and the outer surface G2 (eps_stern, no ions: Laplace), region 3 outside
G2 (eps_out, kappa).  Test infrastructure only.

Unknowns phi_1, q_1 = dphi/dn on G1 (region-1 side) and phi_2, q_2 on G2
(region-2 side), normals outward; fluxes continue as eps q.  Green's second
identity in each region, with the layer-potential limits of the
one-surface case (interior side of a surface: K - 1/2; exterior: K + 1/2),
gives the block system
  G1, region 1:  1/2 phi1 + K11 phi1 - V11 q1                          = f
  G1, region 2:  1/2 phi1 - K11 phi1 + (e1/es) V11 q1 + K21 phi2 - V21 q2 = 0
  G2, region 2:  -K12 phi1 + (e1/es) V12 q1 + 1/2 phi2 + K22 phi2 - V22 q2 = 0
  G2, region 3:  1/2 phi2 - KY22 phi2 + (es/eo) VY22 q2                 = 0
with Laplace operators except KY, VY; Kab, Vab map densities on Gb to the
collocation points of Ga.  Each surface's own pair of rows is the
one-surface operator (G1 with kappa = 0 and ratio e1/es, G2 with kappa and
ratio es/eo); the cross terms are layer potentials of one surface evaluated
at the other's collocation points (the near rule applies where a point is
within eta sqrt(A_j) of panel j, as for the site readout).  The reaction
field at the sites comes from G1's densities alone.
"""

import numpy as np

from . import bie, multipoles as mp

FOUR_PI = 4.0 * np.pi


class SternBemSolvent:
    def __init__(self, verts1, tris1, verts2, tris2, eps_in, eps_stern, eps_out, kappa,
                 gmres_tol=1e-13):
        self.m1 = bie.Mesh(verts1, tris1, 0.0)
        self.m2 = bie.Mesh(verts2, tris2, kappa)
        self.e1, self.es, self.eo = eps_in, eps_stern, eps_out
        self.gmres_tol = gmres_tol
        self.x = None
        self.solves = 0

    def apply(self, X):
        N1, N2 = self.m1.N, self.m2.N
        x1, x2 = X[:2 * N1], X[2 * N1:]
        y1 = bie.matvec(self.m1, x1, self.e1, self.es)
        y2 = bie.matvec(self.m2, x2, self.es, self.eo)
        # V2[q2] - K2[phi2] at G1, and V1[(e1/es) q1] - K1[phi1] at G2
        y1[N1:] -= self.m2.readout(x2, self.m1.cen)[:, 0]
        s1 = np.concatenate([x1[:N1], (self.e1 / self.es) * x1[N1:]])
        y2[:N2] += self.m1.readout(s1, self.m2.cen)[:, 0]
        return np.concatenate([y1, y2])

    def solve_for(self, xyz, q, p, Q9):
        N1, N2 = self.m1.N, self.m2.N
        f = mp.rhs(self.m1.cen, xyz, q, p, Q9, self.e1)
        b = np.concatenate([f, np.zeros(N1 + 2 * N2)])
        x, _, _ = bie.gmres(self.apply, b, x0=self.x, tol=self.gmres_tol)
        self.x = x
        self.solves += 1
        return x

    def reaction(self, xyz, q, p, Q9):
        x = self.solve_for(xyz, q, p, Q9)
        return FOUR_PI * self.m1.readout(x[:2 * self.m1.N], xyz)
