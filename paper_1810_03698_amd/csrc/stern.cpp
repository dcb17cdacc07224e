// Ion-exclusion (Stern) layer: a second, enclosing surface G2 between the
// molecule's surface G1 and the salt solution (section "Spherical cavity":
// the verification case has a 1 A layer).  Regions: 1 inside G1 (eps_in,
// the multipoles), 2 between G1 and G2 (eps_stern, no ions: Laplace),
// 3 outside G2 (eps_out, kappa).  Green's second identity in every region,
// with the one-surface layer-potential limits, gives for the densities
// X = [phi1, q1, phi2, q2] (q: dphi/dn on the inner side of each surface)
//   1/2 phi1 + K11 phi1 - V11 q1                               = f
//   1/2 phi1 - K11 phi1 + (e1/es) V11 q1 + K21 phi2 - V21 q2   = 0
//   -K12 phi1 + (e1/es) V12 q1 + 1/2 phi2 + K22 phi2 - V22 q2  = 0
//   1/2 phi2 - KY22 phi2 + (es/eo) VY22 q2                     = 0
// (Laplace operators except KY, VY).  Each surface's pair of rows is the
// one-surface operator -- G1 with kappa = 0 and ratio e1/es, G2 with kappa
// and es/eo -- and the cross terms are the layer potentials V[q] - K[phi]
// of one surface at the other's collocation points, evaluated by the
// site-readout kernels (near rule where a point is within eta sqrt(A_j) of
// panel j).  The reaction field at the sites comes from G1 alone.
#include <algorithm>
#include <cmath>

#include "runtime.hpp"

namespace pbmp {

void launch_add_strided(hipStream_t s, int n, double sign, const double *p, int stride,
                        double *y);

void Runtime::set_probe(int M, const std::vector<double> &pts) {
  Mp_ = M;
  std::vector<int> row, col;
  point_lists(pts, M, row, col);
  pxyz_.upload(pts.data(), pts.size(), s_);
  prow_.upload(row.data(), row.size(), s_);
  pcol_.upload(col.data(), col.size(), s_);
  p_chunks_ = readout_chunks(N_, M);
  ppart_.alloc((size_t)p_chunks_ * M * 10);
  pout_.alloc(4 * (size_t)M);
  sync();
}

void Runtime::probe(const double *x, bool f64, double *out4) {
  launch_pack_strengths(s_, N_, ru_.nf, geo_.p, x, src64_.p, src32_.p);
  launch_readout(s_, fp64() || f64, false, N_, Mp_, src64_.p, src32_.p, geo_.p, verts_.p,
                 tri_.p, ru_, x, pxyz_.p, prow_.p, pcol_.p, p_chunks_, ppart_.p, out4);
}

void Runtime::set_stern(int64_t nv, const double *verts, int64_t nt, const int32_t *tris,
                        double eps_stern, int where) {
  ax_holds_x_ = gax_holds_x_ = false;
  adj_ok_ = false;
  PBMP_REQUIRE(N_ > 0, PBMP_ESTATE, "set_mesh must precede pbmp_set_stern");
  if (nt == 0) {
    if (outer_) {
      o.kappa = kappa_ext_;
      o.eps_out = eps_out_ext_;
      outer_.reset();
      build_near_lists();
    }
    warm_ok_ = false;
    solved_ = false;
    return;
  }
  PBMP_REQUIRE(!tree_active_, PBMP_EARG, "the Stern layer is available in direct mode only");
  PBMP_REQUIRE(std::isfinite(eps_stern) && eps_stern > 0, PBMP_EARG, "eps_stern must be > 0");
  if (!outer_) {
    kappa_ext_ = o.kappa;
    eps_out_ext_ = o.eps_out;
  }
  pbmp_options oo = o;
  oo.eps_in = eps_stern;
  oo.eps_out = eps_out_ext_;
  oo.kappa = kappa_ext_;
  oo.mode = PBMP_MODE_DIRECT;
  oo.hip_stream = s_;
  std::unique_ptr<Runtime> outer(new Runtime(oo));
  outer->set_mesh(nv, verts, nt, tris, where);
  // the molecular surface must lie inside the outer one
  const int N1 = N_, N2 = outer->N_;
  std::vector<double> c1(3 * (size_t)N1), c2(3 * (size_t)N2);
  for (int i = 0; i < N1; ++i)
    for (int d = 0; d < 3; ++d) c1[3 * i + d] = h_geo_[(size_t)d * N1 + i];
  for (int j = 0; j < N2; ++j)
    for (int d = 0; d < 3; ++d) c2[3 * j + d] = outer->h_geo_[(size_t)d * N2 + j];
  {
    Dbuf<double> pts, wind;
    pts.upload(c1.data(), c1.size(), s_);
    wind.alloc(N1);
    launch_winding(s_, N2, N1, outer->verts_.p, outer->tri_.p, pts.p, wind.p);
    std::vector<double> hw(N1);
    wind.download(hw.data(), N1, s_);
    sync();
    for (int i = 0; i < N1; ++i)
      PBMP_REQUIRE(hw[i] > 0.5, PBMP_EMESH,
                   "the Stern surface must enclose the molecular surface");
  }
  outer_ = std::move(outer);
  eps_stern_ = eps_stern;
  // inner surface: Laplace on both sides, ratio eps_in / eps_stern
  o.kappa = 0.0;
  o.eps_out = eps_stern;
  build_near_lists();
  outer_->set_probe(N1, c1);
  set_probe(N2, c2);
  const size_t n = 2 * (size_t)N1 + 2 * (size_t)N2;
  sX_.alloc(n);
  sB_.alloc(n);
  sY_.alloc(n);
  sT_.alloc(2 * (size_t)N1);
  warm_ok_ = false;
  partial_.reserve((size_t)(o.gmres_restart + 2) * ((n + 4095) / 4096 + 1));
  solved_ = false;
}

void Runtime::apply_stern(const double *X, double *Y, bool f64) {
  const int N1 = N_, N2 = outer_->N_;
  apply(X, Y, f64);
  outer_->apply(X + 2 * (size_t)N1, Y + 2 * (size_t)N1, f64);
  // G1 region-2 row: - (V21 q2 - K21 phi2) at G1 (the readout kernels
  // return physical potentials, 4 pi times the integral-equation ones)
  const double inv4pi = 1.0 / (4.0 * M_PI);
  outer_->probe(X + 2 * (size_t)N1, f64, outer_->pout_.p);
  launch_add_strided(s_, N1, -inv4pi, outer_->pout_.p, 4, Y + N1);
  // G2 region-2 row: + (V12 (e1/es) q1 - K12 phi1) at G2
  launch_scale(s_, N1, 1.0, X, sT_.p);
  launch_scale(s_, N1, o.eps_in / eps_stern_, X + N1, sT_.p + N1);
  probe(sT_.p, f64, pout_.p);
  launch_add_strided(s_, N2, inv4pi, pout_.p, 4, Y + 2 * (size_t)N1);
}

void Runtime::precond_stern(const double *v, double *z) {
  const int N1 = N_, N2 = outer_->N_;
  launch_precond(s_, N1, diag_.p, o.eps_in / o.eps_out, v, z);
  launch_precond(s_, N2, outer_->diag_.p, outer_->o.eps_in / outer_->o.eps_out,
                 v + 2 * (size_t)N1, z + 2 * (size_t)N1);
}

int Runtime::gmres_stern(const double *b, double *x, int *iters) {
  const int N1 = N_;
  const size_t n = sX_.n;
  PBMP_HIP(hipMemsetAsync(sB_.p, 0, sizeof(double) * n, s_));
  PBMP_HIP(hipMemcpyAsync(sB_.p, b, sizeof(double) * 2 * N1, hipMemcpyDeviceToDevice, s_));
  const int rc = gmres_generic(
      (int)n, [&](const double *in, double *out, bool f64) { apply_stern(in, out, f64); },
      [&](const double *in, double *out) { precond_stern(in, out); }, sB_.p, sX_.p, iters,
      &gax_holds_x_);
  PBMP_HIP(hipMemcpyAsync(x, sX_.p, sizeof(double) * 2 * N1, hipMemcpyDeviceToDevice, s_));
  return rc;
}

void Runtime::stern_matvec_user(const double *x, double *y, int where) {
  const int N1 = N_;
  to_internal(x, sX_.p, 2, where);
  outer_->to_internal(x + 2 * (size_t)N1, sX_.p + 2 * (size_t)N1, 2, where);
  apply_stern(sX_.p, sY_.p, false);
  to_user(sY_.p, y, 2, where);
  outer_->to_user(sY_.p + 2 * (size_t)N1, y + 2 * (size_t)N1, 2, where);
}

}  // namespace pbmp
