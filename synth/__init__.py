"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package only produces input data: triangle meshes (icospheres and
marching-tetrahedra isosurfaces of synthetic molecules) and point-multipole
sites (positions, charges, dipoles, quadrupoles, polarisabilities).  It holds
none of the boundary-integral arithmetic; both the oracle and the HIP library
consume what it returns.

Every generator draws from ``numpy.random.default_rng(seed)`` in a fixed
order (positions, charges, dipole direction, dipole magnitude, quadrupole,
polarisability), so a given seed always yields the same arrays.
"""

from .icosphere import icosphere
from .sites import random_multipoles, sites_in_ball
from .molecule import saw_molecule, isosurface_mesh, molecule_mesh
from .configs import workload, WORKLOADS

__all__ = [
    "icosphere",
    "random_multipoles",
    "sites_in_ball",
    "saw_molecule",
    "isosurface_mesh",
    "molecule_mesh",
    "workload",
    "WORKLOADS",
]
