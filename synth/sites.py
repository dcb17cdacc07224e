"""Point-multipole sites: positions plus permanent charge q, dipole d,
traceless symmetric quadrupole Q (Buckingham convention, full 3x3 row-major)
and isotropic polarisability alpha.

Distributions (all units: Angstrom, e):
  q ~ U[-0.5, 0.5];  |d| ~ U[0, 0.3] with direction uniform on the sphere;
  Q: the six upper-triangle entries iid N(0, 0.2), symmetrised, trace/3
  removed from the diagonal;  alpha ~ U[0.3, 1.5] A^3.
"""

import numpy as np


def sites_in_ball(rng, m, radius=2.5, min_sep=1.0, max_tries=100000):
    """m points uniform in a ball, rejecting draws closer than min_sep to an
    already accepted point (keeps the undamped permanent fields moderate)."""
    pts = []
    tries = 0
    while len(pts) < m:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place sites")
        p = rng.uniform(-radius, radius, size=3)
        if p @ p >= radius * radius:
            continue
        if any(np.linalg.norm(p - q) < min_sep for q in pts):
            continue
        pts.append(p)
    return np.array(pts, dtype=np.float64)


def random_multipoles(rng, m, q_range=0.5, d_max=0.3, q_sigma=0.2,
                      alpha_range=(0.3, 1.5)):
    """Draw (q, d, Q9, alpha) for m sites, in the fixed draw order
    charge, dipole direction, dipole magnitude, quadrupole, polarisability."""
    q = rng.uniform(-q_range, q_range, size=m)
    u = rng.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    dmag = rng.uniform(0.0, d_max, size=m)
    d = u * dmag[:, None]
    upper = rng.normal(0.0, q_sigma, size=(m, 6))
    Q = np.zeros((m, 3, 3))
    iu = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for k, (i, j) in enumerate(iu):
        Q[:, i, j] = upper[:, k]
        Q[:, j, i] = upper[:, k]
    tr = np.trace(Q, axis1=1, axis2=2)
    for i in range(3):
        Q[:, i, i] -= tr / 3.0
    alpha = rng.uniform(alpha_range[0], alpha_range[1], size=m)
    return q, d, Q.reshape(m, 9), alpha
