"""Point-multipole electrostatics (test infrastructure only).

Units: lengths in A, charges in e, potentials in e/A (physical, i.e. the
Coulomb potential q/r, divided by the dielectric constant where one applies).

* Multipole potential (eq. pot_multipole), for R = r - r_k:
      phi = q/R + p.R/R^3 + (1/2) Q_ij R_i R_j / R^5
  with Q the traceless Buckingham quadrupole.  Its first and second
  derivatives in r are the exact chain-rule derivatives of each term (the
  appendix's eq. derivatives_Emult / second_derivative, with the missing
  delta-delta term of the quadrupole's second derivative restored).
* Right-hand side (eq. rhs_multipole): phi / (4 pi eps_in) at the
  collocation points, total dipole p = d + mu (eq. dipole_decomposition).
* Thole damping of induced-dipole interactions (cited, formula not printed;
  read as the AMOEBA form): u = R / (alpha_l alpha_m)^(1/6), s = a u^3,
      l3 = 1 - e^-s,  l5 = 1 - (1+s) e^-s,  l7 = 1 - (1 + s + 3/5 s^2) e^-s,
  and the damped dipole potential, field and field gradient
      phi = l3 mu.R/R^3
      d_k phi = l3 mu_k/R^3 - 3 l5 (mu.R) R_k/R^5
      d_k d_o phi = -3 l5 (mu_k R_o + mu_o R_k + (mu.R) delta_ko)/R^5
                    + 15 l7 (mu.R) R_k R_o / R^7
  which reduce to the undamped dipole expressions when all l = 1.
"""

import numpy as np

FOUR_PI = 4.0 * np.pi

# CODATA 2018 (exact SI definitions for e and N_A)
E_CHARGE = 1.602176634e-19
N_AVOGADRO = 6.02214076e23
EPS0 = 8.8541878128e-12
KCAL = 4184.0
COULOMB_KCAL = E_CHARGE ** 2 * N_AVOGADRO / (FOUR_PI * EPS0 * 1e-10 * KCAL)
C_LIGHT = 299792458.0
DEBYE_PER_EA = E_CHARGE * 1e-10 / (1e-21 / C_LIGHT)


def _R(r_eval, r_src):
    R = r_eval[:, None, :] - r_src[None, :, :]
    r = np.linalg.norm(R, axis=2)
    return R, r


def multipole_potential(points, xyz, q, p, Q9):
    """Literal eq. pot_multipole summed over all sources: [npts]."""
    Q = Q9.reshape(-1, 3, 3)
    R, r = _R(points, xyz)
    pR = np.einsum("lmi,mi->lm", R, p)
    QRR = np.einsum("lmi,mij,lmj->lm", R, Q, R)
    return (q[None] / r + pR / r ** 3 + 0.5 * QRR / r ** 5).sum(1)


def rhs(centroids, xyz, q, p, Q9, eps_in):
    """Right-hand side f (eq. rhs_multipole) in the integral-equation
    normalisation: multipole potential / (4 pi eps_in)."""
    return multipole_potential(centroids, xyz, q, p, Q9) / (FOUR_PI * eps_in)


def permanent_derivs(r_eval, xyz, q, p, Q9, pair_mask):
    """Potential, gradient and Hessian at r_eval [L,3] of the multipoles at
    xyz [M,3]; pair (l, m) contributes only where pair_mask[l, m].
    Returns phi [L], g [L,3], H [L,3,3]."""
    Q = Q9.reshape(-1, 3, 3)
    R, r = _R(r_eval, xyz)
    r = np.where(pair_mask, r, 1.0)
    w = pair_mask.astype(np.float64)
    I = np.eye(3)
    r3, r5, r7, r9 = r ** 3, r ** 5, r ** 7, r ** 9
    pR = np.einsum("lmi,mi->lm", R, p)
    QR = np.einsum("mij,lmj->lmi", Q, R)
    S = np.einsum("lmi,lmi->lm", R, QR)
    RR = R[..., :, None] * R[..., None, :]
    # charge
    phi = q[None] / r
    g = -q[None, :, None] * R / r3[..., None]
    H = q[None, :, None, None] * (3 * RR / r5[..., None, None]
                                  - I / r3[..., None, None])
    # dipole
    phi = phi + pR / r3
    g = g + p[None] / r3[..., None] - 3 * pR[..., None] * R / r5[..., None]
    pRo = p[None, :, :, None] * R[..., None, :]
    H = H + (-3 * (pRo + np.swapaxes(pRo, -1, -2)) / r5[..., None, None]
             - 3 * pR[..., None, None] * I / r5[..., None, None]
             + 15 * pR[..., None, None] * RR / r7[..., None, None])
    # quadrupole: (1/2) S / R^5 with S = Q_ij R_i R_j
    phi = phi + 0.5 * S / r5
    g = g + QR / r5[..., None] - 2.5 * S[..., None] * R / r7[..., None]
    QRo = QR[..., :, None] * R[..., None, :]
    H = H + (Q[None] / r5[..., None, None]
             - 5 * (QRo + np.swapaxes(QRo, -1, -2)) / r7[..., None, None]
             - 2.5 * S[..., None, None] * I / r7[..., None, None]
             + 17.5 * S[..., None, None] * RR / r9[..., None, None])
    phi = (phi * w).sum(1)
    g = (g * w[..., None]).sum(1)
    H = (H * w[..., None, None]).sum(1)
    return phi, g, H


def thole_lambdas(r, alpha_l, alpha_m, a):
    """(l3, l5, l7) for distances r [..] and polarisabilities."""
    prod = alpha_l * alpha_m
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.where(prod > 0, a * r ** 3 / np.sqrt(np.where(prod > 0, prod, 1.0)),
                     np.inf)
    es = np.exp(-s)
    l3 = 1.0 - es
    l5 = 1.0 - (1.0 + s) * es
    l7 = 1.0 - (1.0 + s + 0.6 * s * s) * es
    fin = np.isfinite(s)
    l3 = np.where(fin, l3, 1.0)
    l5 = np.where(fin, l5, 1.0)
    l7 = np.where(fin, l7, 1.0)
    return l3, l5, l7


def induced_derivs(r_eval, xyz, mu, alpha_eval, alpha_src, a, pair_mask):
    """Thole-damped potential, gradient and Hessian of dipoles mu at xyz,
    evaluated at r_eval; alpha_eval/alpha_src are the polarisabilities of
    the evaluation and source sites."""
    R, r = _R(r_eval, xyz)
    r = np.where(pair_mask, r, 1.0)
    w = pair_mask.astype(np.float64)
    l3, l5, l7 = thole_lambdas(r, alpha_eval[:, None], alpha_src[None, :], a)
    I = np.eye(3)
    r3, r5, r7 = r ** 3, r ** 5, r ** 7
    mR = np.einsum("lmi,mi->lm", R, mu)
    RR = R[..., :, None] * R[..., None, :]
    phi = l3 * mR / r3
    g = (l3 / r3)[..., None] * mu[None] - (3 * l5 * mR / r5)[..., None] * R
    mRo = mu[None, :, :, None] * R[..., None, :]
    H = (-3 * (l5 / r5)[..., None, None] * (mRo + np.swapaxes(mRo, -1, -2)
                                             + mR[..., None, None] * I)
         + (15 * l7 * mR / r7)[..., None, None] * RR)
    phi = (phi * w).sum(1)
    g = (g * w[..., None]).sum(1)
    H = (H * w[..., None, None]).sum(1)
    return phi, g, H
