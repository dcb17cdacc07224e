"""Induced-dipole self-consistent loop and solvation energy (test
infrastructure only).

Self-consistent scheme (section "Self-consistent induced field"):
  1. mu = 0;  2. solve the boundary-integral system with p = d + mu;
  3. reaction field E_solv (eq. Efield_solv) and multipole field E_mult
     (eq. Efield_mult) at the sites;  4. E = E_solv + E_mult (eq. Efield_tot);
  5. mu_new = (1 - w) mu + w alpha E with w = 0.7 (the relaxation
     coefficient of the paper's update);  6. repeat until the RMS over sites
     of |mu_new - mu| (in Debye) is below the tolerance.
E_mult: permanent multipoles of other polarisation groups, undamped, plus
the induced dipoles of all other sites, Thole-damped.  Vacuum state: the
same loop without E_solv (homogeneous dielectric eps_in).

Solvation energy (eq. energy_general with the polarisable energy form
eq. energy_multipole_polarizable): with the permanent dipole d in place of
the total dipole, and the permanent-permanent Coulomb terms cancelling
between the dissolved and vacuum states,
  dG = C * 1/2 sum_l D_l [phi_solv + phi_ind(mu_diss) - phi_ind(mu_vac)](r_l),
  D_l = q_l + d_l . grad + (1/6) Q_l : grad grad,
where phi_ind is the damped potential of the other sites' induced dipoles
(unmasked) and C = e^2 N_A / (4 pi eps0 A) in kcal/mol.

The "solvent" is pluggable: ``BemSolvent`` solves the discretised integral
equation, ``kirkwood.SphereSolvent`` evaluates the exact series for a
spherical cavity.
"""

import numpy as np

from . import bie, multipoles as mp

FOUR_PI = 4.0 * np.pi


class BemSolvent:
    """Reaction field from the boundary-integral system (dense LU up to
    ``dense_max`` panels, else matrix-free GMRES)."""

    def __init__(self, verts, tris, eps_in, eps_out, kappa, eta=2.0, far=3,
                 dense_max=5120, gmres_tol=1e-13):
        self.mesh = bie.Mesh(verts, tris, kappa, eta=eta, far=far)
        self.eps_in, self.eps_out = eps_in, eps_out
        self.gmres_tol = gmres_tol
        self.A = None
        if self.mesh.N <= dense_max:
            import scipy.linalg
            self.A = bie.dense_system(self.mesh, eps_in, eps_out)
            self.lu = scipy.linalg.lu_factor(self.A)
        self.x = None
        self.solves = 0

    def apply(self, x):
        return bie.matvec(self.mesh, x, self.eps_in, self.eps_out)

    def solve_for(self, xyz, q, p, Q9):
        import scipy.linalg
        N = self.mesh.N
        f = mp.rhs(self.mesh.cen, xyz, q, p, Q9, self.eps_in)
        b = np.concatenate([f, np.zeros(N)])
        if self.A is not None:
            x = scipy.linalg.lu_solve(self.lu, b)
        else:
            x, _, _ = bie.gmres(self.apply, b, x0=self.x, tol=self.gmres_tol)
        self.x = x
        self.solves += 1
        return x

    def reaction(self, xyz, q, p, Q9):
        """Physical reaction potential data [M,10] at the sites for total
        dipoles p; also remembers the surface solution in self.x."""
        x = self.solve_for(xyz, q, p, Q9)
        return FOUR_PI * self.mesh.readout(x, xyz)


def _rms_debye(dmu):
    return float(np.sqrt((np.linalg.norm(dmu, axis=1) ** 2).mean())) \
        * mp.DEBYE_PER_EA


def scf(xyz, q, d, Q9, alpha, group, eps_in, thole_a, omega, tol_debye,
        maxit, solvent=None, damp_direct=False):
    """Returns (mu, iterations, last reaction data or None)."""
    M = len(xyz)
    offdiag = ~np.eye(M, dtype=bool)
    other_group = group[:, None] != group[None, :]
    if damp_direct:
        raise NotImplementedError("damp_direct is not part of the oracle")
    _, gp, _ = mp.permanent_derivs(xyz, xyz, q, d, Q9, other_group & offdiag)
    E_perm = -gp / eps_in
    mu = np.zeros((M, 3))
    reac = None
    for it in range(1, maxit + 1):
        E = E_perm.copy()
        _, gi, _ = mp.induced_derivs(xyz, xyz, mu, alpha, alpha, thole_a,
                                     offdiag)
        E -= gi / eps_in
        if solvent is not None:
            reac = solvent.reaction(xyz, q, d + mu, Q9)
            E -= reac[:, 1:4]
        mu_new = (1.0 - omega) * mu + omega * alpha[:, None] * E
        dmu = _rms_debye(mu_new - mu)
        mu = mu_new
        if dmu < tol_debye:
            return mu, it, reac
    return mu, maxit, reac


def _apply_D(q, d, Q9, data):
    """sum_l q phi + d.grad phi + (1/6) Q:grad grad phi for data [M,10]."""
    Q = Q9.reshape(-1, 3, 3)
    H = np.empty((len(q), 3, 3))
    idx = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for k, (i, j) in enumerate(idx):
        H[:, i, j] = data[:, 4 + k]
        H[:, j, i] = data[:, 4 + k]
    return (q * data[:, 0] + np.einsum("li,li->l", d, data[:, 1:4])
            + np.einsum("lij,lij->l", Q, H) / 6.0).sum()


def _pack(phi, g, H):
    out = np.empty((len(phi), 10))
    out[:, 0] = phi
    out[:, 1:4] = g
    for k, (i, j) in enumerate([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
        out[:, 4 + k] = H[:, i, j]
    return out


def vacuum_energy(xyz, q, d, Q9, alpha, mu_v, eps_in=1.0, thole_a=0.39):
    """Coulomb energy of the vacuum state (eq. energy_multipole_polarizable:
    the polarisation work is carried by using d in place of d + mu), with phi
    the potential of the other sites' permanent multipoles, unmasked and
    undamped, plus their Thole-damped vacuum induced dipoles.  Differences
    of it over a complex and its parts give the vacuum binding energy
    (eq. bind_vac).  kcal/mol."""
    M = len(xyz)
    offdiag = ~np.eye(M, dtype=bool)
    perm = _pack(*mp.permanent_derivs(xyz, xyz, q, d, Q9, offdiag)) / eps_in
    ind = _pack(*mp.induced_derivs(xyz, xyz, mu_v, alpha, alpha, thole_a,
                                   offdiag)) / eps_in
    return mp.COULOMB_KCAL * 0.5 * _apply_D(q, d, Q9, perm + ind)


def total_dipole(xyz, q, d, mu, origin=None):
    """Total dipole moment of the molecule in Debye (the diagnostic of the
    comparison with Tinker-APBS, Table "dipole"): sum over sites of
    q_l (r_l - origin) + d_l + mu_l.  The paper names no origin; here it is
    the unweighted mean of the site positions (for a neutral molecule the
    result does not depend on it)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    o = xyz.mean(axis=0) if origin is None else np.asarray(origin, dtype=np.float64)
    p = (np.asarray(q)[:, None] * (xyz - o)).sum(axis=0) + np.asarray(d).sum(axis=0) \
        + np.asarray(mu).sum(axis=0)
    return p * mp.DEBYE_PER_EA


def solvation(xyz, q, d, Q9, alpha, solvent, group=None, eps_in=1.0,
              thole_a=0.39, omega=0.7, tol_debye=1e-6, maxit=1000):
    """Full polarisable solvation energy.  Returns a dict with dG (kcal/mol),
    mu_diss, mu_vac, the surface solution x (if BEM), iteration counts and
    the energy's two parts."""
    xyz = np.asarray(xyz, dtype=np.float64)
    M = len(xyz)
    group = np.arange(M) if group is None else np.asarray(group)
    mu_v, it_v, _ = scf(xyz, q, d, Q9, alpha, group, eps_in, thole_a, omega,
                        tol_debye, maxit, solvent=None)
    mu_d, it_d, reac = scf(xyz, q, d, Q9, alpha, group, eps_in, thole_a, omega,
                           tol_debye, maxit, solvent=solvent)
    offdiag = ~np.eye(M, dtype=bool)
    ind_d = _pack(*mp.induced_derivs(xyz, xyz, mu_d, alpha, alpha, thole_a,
                                     offdiag)) / eps_in
    ind_v = _pack(*mp.induced_derivs(xyz, xyz, mu_v, alpha, alpha, thole_a,
                                     offdiag)) / eps_in
    e_solv = 0.5 * _apply_D(q, d, Q9, reac)
    e_pol = 0.5 * _apply_D(q, d, Q9, ind_d - ind_v)
    dG = mp.COULOMB_KCAL * (e_solv + e_pol)
    return dict(dG=dG, G_vac=vacuum_energy(xyz, q, d, Q9, alpha, mu_v, eps_in, thole_a),
                dipole_vac=total_dipole(xyz, q, d, mu_v),
                dipole_diss=total_dipole(xyz, q, d, mu_d),
                mu_diss=mu_d, mu_vac=mu_v, scf_iters=it_d,
                scf_iters_vac=it_v, reaction=reac,
                x=getattr(solvent, "x", None),
                e_solv=mp.COULOMB_KCAL * e_solv, e_pol=mp.COULOMB_KCAL * e_pol)
