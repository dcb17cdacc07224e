// Transposed operator and the adjoint (backward) pass.
#include "runtime.hpp"

namespace pbmp {

void Runtime::apply_transpose(const double *x, double *y) {
  PBMP_REQUIRE(!use_tree(), PBMP_EARG, "the transposed product needs direct mode");
  launch_transpose(s_, fp64(), ru_.nf, N_, src64_.p, src32_.p, geo_.p, tgt32_.p, x, o.kappa,
                   p2p_chunks_, part_.p, trow_.p, tcol_.p, tent_.p, nval_.p,
                   o.eps_in / o.eps_out, y);
  ++matvecs_;
}

int Runtime::backward(double, double *, double *, double *, double *, double *, int) {
  throw Error(PBMP_EARG, "backward is not available in this build");
}

}  // namespace pbmp
