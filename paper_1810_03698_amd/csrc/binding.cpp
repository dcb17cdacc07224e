// Binding energies of a complex from the solves of the complex and of its
// two parts (section "Calculation of the binding energy"), and the
// derivative of the relative binding energy with respect to a rigid
// translation of the ligand.
//   relative   ddG       = dG_solv(AB) - dG_solv(A) - dG_solv(B)   (eq. rel_bind_energy)
//   vacuum     dG_vac    = G_AB - G_A - G_B                          (eq. bind_vac)
//   dissolved  dG_diss   = ddG + dG_vac                              (eq. bind_energy)
// with G the vacuum-state Coulomb energy of each solve.  Translating the
// ligand B by t moves B's sites in the complex and the part of the complex
// surface that belongs to B; B's own surface translates as a whole, which
// leaves dG_solv(B) unchanged, and A does not move, so
//   d ddG / dt = sum over B's sites of dG_AB/dr + sum over B's vertices of dG_AB/dv.
// A complex vertex belongs to the molecule whose atom minimises
// |v - r_a| - R_a (the distance to the atom's sphere).
#include <cmath>

#include "runtime.hpp"

namespace pbmp {

void launch_translation_sum(hipStream_t s, int nv, int m, int first_ligand,
                            const double *verts, const double *xyz, const double *radii,
                            const double *g_verts, const double *g_xyz, int *owner,
                            double *out);

void Runtime::binding_terms(double *dG, double *G_vac) const {
  PBMP_REQUIRE(solved_, PBMP_ESTATE, "binding energies need a completed solve of each context");
  *dG = last_dG_;
  *G_vac = last_Gvac_;
}

int Runtime::ligand_translation_gradient(int64_t first_ligand, const double *radii, int where,
                                         double g_t[3], int64_t *n_ligand_vertices) {
  PBMP_REQUIRE(solved_, PBMP_ESTATE, "the gradient needs a completed solve of the complex");
  PBMP_REQUIRE(first_ligand >= 0 && first_ligand < M_, PBMP_EARG,
               "first ligand site out of range");
  PBMP_REQUIRE(radii != nullptr && g_t != nullptr, PBMP_EARG, "null radii or output");
  PBMP_REQUIRE(where == PBMP_HOST || where == PBMP_DEVICE, PBMP_EARG, "bad where");
  Dbuf<double> gx, gv, rad, out;
  Dbuf<int> owner;
  gx.alloc(3 * (size_t)M_);
  gv.alloc(3 * (size_t)Nv_);
  rad.alloc(M_);
  out.alloc(4);
  owner.alloc(std::max(1, Nv_));
  PBMP_HIP(hipMemcpyAsync(rad.p, radii, sizeof(double) * M_,
                          where == PBMP_DEVICE ? hipMemcpyDeviceToDevice
                                               : hipMemcpyHostToDevice, s_));
  const int rc = backward(1.0, gx.p, nullptr, nullptr, nullptr, gv.p, PBMP_DEVICE);
  launch_translation_sum(s_, Nv_, M_, (int)first_ligand, verts_.p, sxyz_.p, rad.p, gv.p, gx.p,
                         owner.p, out.p);
  double h[4];
  PBMP_HIP(hipMemcpyAsync(h, out.p, sizeof(h), hipMemcpyDeviceToHost, s_));
  sync();
  for (int c = 0; c < 3; ++c) g_t[c] = h[c];
  if (n_ligand_vertices) *n_ligand_vertices = (int64_t)h[3];
  return rc;
}

}  // namespace pbmp
