"""FP64 CPU oracle for the boundary-integral Poisson-Boltzmann method with
polarisable point multipoles (Cooper, "A boundary-integral approach for the
Poisson-Boltzmann equation with polarizable force fields").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
runs this package: it exists so that tests, the smoke check and the CPU
baseline leg of the benchmark can compare the HIP library against a plain,
slow, obviously correct implementation.  It shares no code, tables or
constants with the HIP library; the only common inputs come from the
``synth`` generators.

Modules
  quadrature  triangle rules (3-point interior rule, 19-point degree-9 rule
              obtained by solving the moment equations) and Gauss-Legendre
  geometry    per-panel centroid, normal, area and quadrature points
  bie         dense operators, matrix-free matvec and site readout; the pair
              loops live in ``bie_c.c`` (plain C, OpenMP over targets)
  multipoles  point-multipole potentials/fields (eq. pot_multipole,
              rhs_multipole, Efield_mult, appendix derivatives), Thole damping
  solver      induced-dipole self-consistent loop and solvation energy
  kirkwood    Kirkwood / Kong-Ponder series for a spherical cavity
  taylor      Taylor coefficients of the Laplace and Yukawa kernels by
              truncated multivariate power-series arithmetic (treecode pin)
"""
