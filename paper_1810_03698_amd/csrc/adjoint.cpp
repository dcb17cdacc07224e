// Transposed operator and the adjoint (backward) pass of the solvation
// energy with respect to site positions and multipole parameters.
//
// Converged forward state (vacuum mu_v; dissolved x, mu_d):
//   g_v = mu_v - alpha (E_perm + T mu_v)                       = 0
//   g_x = A x - [f(d + mu_d); 0]                               = 0
//   g_d = mu_d - alpha (E_perm + T mu_d + E_s(x))              = 0
//   J   = C/2 sum_l D_l [reac_l(x) + ind_l(mu_d - mu_v)]
// Lagrangian J + l_v.g_v + l_x.g_x + l_d.g_d; stationarity gives
//   l_v = T alpha l_v + J_mu                        (relaxed fixed point)
//   A^T l_x = -d/dx [W'.reac],  W' = C/2 D + (0, alpha l_d, 0)
//   l_d = T alpha l_d + F^T l_x1 - J_mu             (F = df/dp)
// with J_mu = dJ/dmu_d = -dJ/dmu_v (T is symmetric, alpha diagonal).  These
// are solved by the same relaxed iteration as the forward loop (the
// iteration matrix is the transpose of the forward one), each dissolved
// step with GMRES on A^T.  The gradient is the explicit derivative of the
// Lagrangian at fixed states.
#include <chrono>
#include <cmath>
#include <cstdio>

#include "runtime.hpp"

namespace pbmp {

void launch_make_weights(hipStream_t s, int M, double c, const double *q, const double *d,
                         const double *Q, const double *wd, double *W);
void launch_readout_T(hipStream_t s, int N, int M, const double *src64, const double *geo,
                      const double *verts, const int *tri, const RuleArgs &ru,
                      const double *xyz, const double *W, const int *tsrow, const int *tscol,
                      double *out);
void launch_charge_field(hipStream_t s, int N, int M, const double *geo, const double *sigma,
                         const double *xyz, double *out);
void launch_jmu(hipStream_t s, int M, const double *W, const double *xyz, const double *alpha,
                double ta, double eps_in, double *out);
void launch_site_pairs(hipStream_t s, int M, const double *xyz, const double *q,
                       const double *d, const double *Q, const int *group,
                       const double *alpha, double ta, double eps_in, const double *Wc,
                       const double *wv, const double *wd, const double *mu_v,
                       const double *mu_d, double *g_r, double *g_q, double *g_d,
                       double *g_Q);
void launch_readout_grad(hipStream_t s, int N, int M, const double *src64, const double *verts,
                         const int *tri, const RuleArgs &ru, const double *geo,
                         const double *x, const double *xyz, const double *W,
                         const int *srow, const int *scol, double *g_r);
void launch_rhs_grad(hipStream_t s, int N, int M, const double *geo, const double *sigma,
                     const double *xyz, const double *q, const double *p, const double *Q,
                     double *g_r, double *g_q, double *g_d, double *g_Q);
void launch_precond_T(hipStream_t s, int N, const double *diag, double eps_ratio,
                      const double *u, double *z);
void launch_scale_sites(hipStream_t s, int M, const double *alpha, const double *lam,
                        double *w);
void launch_adj_update(hipStream_t s, int M, double omega, const double *E, const double *F,
                       const double *J, double Jsign, double *lam, double *out2);
void launch_mesh_adjoint(hipStream_t s, int N, int M, int nf, const double *src64,
                         const double *geo, const double *verts, const int *tri,
                         const RuleArgs &ru, const int *rowptr, const int *col,
                         const int *trow, const int *tent, const int *tsrow,
                         const int *tscol, const double *x, const double *lam,
                         const double *sigma, const double *xyz, const double *q,
                         const double *p, const double *Q, const double *Wp, double kappa,
                         double eps_ratio, double *work, double *ge, double *out, Tree *tree,
                         double *part, double *partT);

void Runtime::apply_transpose(const double *x, double *y, bool f64) {
  const bool use64 = f64 || fp64();
  const double *val = (use64 && !fp64()) ? nval64_.p : nval_.p;
  if (use_tree())
    tree_apply_transpose(*tree_, s_, use64, ru_.nf, N_, geo_.p, src64_.p, src32_.p, tgt32_.p,
                         x, o.kappa, part_.p, trow_.p, tcol_.p, tent_.p, val,
                         o.eps_in / o.eps_out, y);
  else
    launch_transpose(s_, use64, ru_.nf, N_, src64_.p, src32_.p, geo_.p, tgt32_.p, x, o.kappa,
                     p2p_chunks_, part_.p, trow_.p, tcol_.p, tent_.p, val,
                     o.eps_in / o.eps_out, y);
  ++matvecs_;
}

void Runtime::precond_T(const double *u, double *z) {
  launch_precond_T(s_, N_, diag_.p, o.eps_in / o.eps_out, u, z);
}

int Runtime::backward(double dGbar, double *g_xyz, double *g_q, double *g_d, double *g_Q,
                      double *g_verts, int where) {
  PBMP_REQUIRE(solved_, PBMP_ESTATE, "backward needs a completed solve on this context");
  PBMP_REQUIRE(!outer_, PBMP_ESTATE, "backward is not available with a Stern layer");
  PBMP_REQUIRE(where == PBMP_HOST || where == PBMP_DEVICE, PBMP_EARG, "bad where");
  const int M = M_, N = N_;
  const double c = dGbar * coulomb_kcal() * 0.5;
  const double ta = o.thole_a, eps = o.eps_in;
  Dbuf<double> Wc, Wp, Jmu, wv, wd, E, F, sig, rhs, red;
  // multipliers, kept on the context: with warm_start a backward starts
  // from the previous backward's (same mesh and site count), rescaled to
  // this dG_bar
  Dbuf<double> &lv = adj_lv_, &ld = adj_ld_, &lx = adj_lx_;
  const bool warm = o.warm_start && adj_ok_ && adj_M_ == M && adj_bar_ != 0.0 &&
                    lx.n == 2 * (size_t)N;
  adj_ok_ = false;
  Wc.alloc(10 * (size_t)M);
  Wp.alloc(10 * (size_t)M);
  Jmu.alloc(3 * (size_t)M);
  lv.alloc(3 * (size_t)M);
  ld.alloc(3 * (size_t)M);
  wv.alloc(3 * (size_t)M);
  wd.alloc(3 * (size_t)M);
  E.alloc(3 * (size_t)M);
  F.alloc(3 * (size_t)M);
  sig.alloc(N);
  lx.alloc(2 * (size_t)N);
  rhs.alloc(2 * (size_t)N);
  red.alloc(2);
  if (warm && dGbar != adj_bar_) {
    const double f = dGbar / adj_bar_;
    launch_scale(s_, 3 * M, f, lv.p, lv.p);
    launch_scale(s_, 3 * M, f, ld.p, ld.p);
    launch_scale(s_, 2 * N, f, lx.p, lx.p);
  }
  launch_make_weights(s_, M, c, sq_.p, sd_.p, sQ_.p, nullptr, Wc.p);
  launch_jmu(s_, M, Wc.p, sxyz_.p, salpha_.p, ta, eps, Jmu.p);
  // the relaxed transposed loops stop at a relative change of a tenth of
  // the GMRES tolerance (at least 1e-11, at most 1e-7): the adjoint needs
  // only the accuracy asked of the gradient, not that of the forward solve
  const double rel_tol = std::min(1e-7, std::max(1e-11, 0.1 * o.gmres_tol));
  int warn = 0;
  const auto t_start = std::chrono::steady_clock::now();
  auto relax = [&](bool dissolved, Dbuf<double> &lam, Dbuf<double> &w) {
    if (!warm) {
      PBMP_HIP(hipMemsetAsync(lam.p, 0, sizeof(double) * 3 * M, s_));
      if (dissolved) PBMP_HIP(hipMemsetAsync(lx.p, 0, sizeof(double) * 2 * N, s_));
    }
    for (int it = 1; it <= o.scf_maxit; ++it) {
      int gi = 0;
      launch_scale_sites(s_, M, salpha_.p, lam.p, w.p);
      if (dissolved) {
        launch_make_weights(s_, M, c, sq_.p, sd_.p, sQ_.p, w.p, Wp.p);
        launch_readout_T(s_, N, M, src64_.p, geo_.p, verts_.p, tri_.p, ru_, sxyz_.p, Wp.p,
                         tsrow_.p, tscol_.p, rhs.p);
        const int rc = gmres(rhs.p, lx.p, true, &gi);
        if (rc > 0) warn = rc;
        launch_scale(s_, N, 1.0 / (4.0 * M_PI * eps), lx.p, sig.p);
        launch_charge_field(s_, N, M, geo_.p, sig.p, sxyz_.p, F.p);
      }
      launch_induced(s_, false, M, sxyz_.p, w.p, salpha_.p, ta, eps, E.p);
      launch_adj_update(s_, M, o.scf_omega, E.p, dissolved ? F.p : nullptr, Jmu.p,
                        dissolved ? -1.0 : 1.0, lam.p, red.p);
      double h[2];
      PBMP_HIP(hipMemcpyAsync(h, red.p, sizeof(h), hipMemcpyDeviceToHost, s_));
      sync();
      if (o.verbose)
        std::fprintf(stderr, "pbmp backward: %s iteration %d gmres %d change %.3e %.1f s\n",
                     dissolved ? "dissolved" : "vacuum", it, gi,
                     h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : 0.0,
                     std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start)
                         .count());
      if (!std::isfinite(h[0])) throw Error(PBMP_WSCF, "adjoint iteration diverged");
      if (std::sqrt(h[0]) <= rel_tol * std::sqrt(h[1]) || h[1] == 0.0) {
        launch_scale_sites(s_, M, salpha_.p, lam.p, w.p);
        return;
      }
    }
    launch_scale_sites(s_, M, salpha_.p, lam.p, w.p);
    warn = PBMP_WSCF;
  };
  // pack the forward solution's strengths again (the last products may have
  // packed other vectors)
  launch_pack_strengths(s_, N, ru_.nf, geo_.p, x_.p, src64_.p, src32_.p);
  relax(false, lv, wv);
  relax(true, ld, wd);
  launch_pack_strengths(s_, N, ru_.nf, geo_.p, x_.p, src64_.p, src32_.p);
  // ---- explicit derivatives at fixed states
  Dbuf<double> gr1, gr2, gr3, gq1, gq3, gd1, gd3, gQ1, gQ3;
  for (auto *b : {&gr1, &gr2, &gr3, &gd1, &gd3}) b->alloc(3 * (size_t)M);
  for (auto *b : {&gq1, &gq3}) b->alloc(M);
  for (auto *b : {&gQ1, &gQ3}) b->alloc(9 * (size_t)M);
  launch_site_pairs(s_, M, sxyz_.p, sq_.p, sd_.p, sQ_.p, sgroup_.p, salpha_.p, ta, eps, Wc.p,
                    wv.p, wd.p, mu_v_.p, mu_d_.p, gr1.p, gq1.p, gd1.p, gQ1.p);
  launch_make_weights(s_, M, c, sq_.p, sd_.p, sQ_.p, wd.p, Wp.p);
  launch_readout_grad(s_, N, M, src64_.p, verts_.p, tri_.p, ru_, geo_.p, x_.p, sxyz_.p, Wp.p,
                      srow_.p, scol_.p, gr2.p);
  launch_scale(s_, N, 1.0 / (4.0 * M_PI * eps), lx.p, sig.p);
  launch_scale(s_, 3 * M, 1.0, sd_.p, p_.p);
  launch_axpy(s_, 3 * M, 1.0, mu_d_.p, p_.p);
  launch_rhs_grad(s_, N, M, geo_.p, sig.p, sxyz_.p, sq_.p, p_.p, sQ_.p, gr3.p, gq3.p, gd3.p,
                  gQ3.p);
  // host assembly with the direct terms c * (reac + ind) data
  std::vector<double> reac(10 * (size_t)M), ind(10 * (size_t)M), a(3 * (size_t)M),
      b(3 * (size_t)M), cc(3 * (size_t)M), q1(M), q3(M), d1(3 * (size_t)M), d3(3 * (size_t)M),
      Q1(9 * (size_t)M), Q3(9 * (size_t)M);
  reac_.download(reac.data(), reac.size(), s_);
  ind_.download(ind.data(), ind.size(), s_);
  gr1.download(a.data(), a.size(), s_);
  gr2.download(b.data(), b.size(), s_);
  gr3.download(cc.data(), cc.size(), s_);
  gq1.download(q1.data(), M, s_);
  gq3.download(q3.data(), M, s_);
  gd1.download(d1.data(), d1.size(), s_);
  gd3.download(d3.data(), d3.size(), s_);
  gQ1.download(Q1.data(), Q1.size(), s_);
  gQ3.download(Q3.data(), Q3.size(), s_);
  sync();
  std::vector<double> oxyz(3 * (size_t)M), oq(M), od(3 * (size_t)M), oQ(9 * (size_t)M);
  const int up[3][3] = {{4, 5, 6}, {5, 7, 8}, {6, 8, 9}};
  for (int l = 0; l < M; ++l) {
    const double *r = &reac[10 * (size_t)l], *in = &ind[10 * (size_t)l];
    for (int k = 0; k < 3; ++k) oxyz[3 * l + k] = a[3 * l + k] + b[3 * l + k] + cc[3 * l + k];
    oq[l] = c * (r[0] + in[0]) + q1[l] + q3[l];
    for (int k = 0; k < 3; ++k)
      od[3 * l + k] = c * (r[1 + k] + in[1 + k]) + d1[3 * l + k] + d3[3 * l + k];
    for (int x = 0; x < 3; ++x)
      for (int y = 0; y < 3; ++y)
        oQ[9 * l + 3 * x + y] = c * (r[up[x][y]] + in[up[x][y]]) / 6.0 + Q1[9 * l + 3 * x + y] +
                                Q3[9 * l + 3 * x + y];
  }
  std::vector<double> overts;
  if (g_verts) {
    // mesh: operator entries, right-hand side at the collocation points and
    // the readout, chained to the vertices
    Dbuf<double> work, ge, pv, partT;
    work.alloc(25 * (size_t)N);
    ge.alloc(12 * (size_t)std::max(nnz_, 1));
    pv.alloc(9 * (size_t)N);
    Tree *tr = use_tree() ? tree_.get() : nullptr;
    if (tr) partT.alloc(13 * (size_t)std::max(1, tr->max_slots_T) * N);
    launch_mesh_adjoint(s_, N, M, ru_.nf, src64_.p, geo_.p, verts_.p, tri_.p, ru_, nrow_.p,
                        ncol_.p, trow_.p, tent_.p, tsrow_.p, tscol_.p, x_.p, lx.p, sig.p,
                        sxyz_.p, sq_.p, p_.p, sQ_.p, Wp.p, o.kappa, o.eps_in / o.eps_out,
                        work.p, ge.p, pv.p, tr, part_.p, partT.p);
    std::vector<double> hp(9 * (size_t)N);
    pv.download(hp.data(), hp.size(), s_);
    sync();
    overts.assign(3 * (size_t)Nv_, 0.0);
    for (int j = 0; j < N; ++j)
      for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d)
          overts[3 * (size_t)h_tri_[3 * (size_t)j + a] + d] += hp[9 * (size_t)j + 3 * a + d];
  }
  auto put = [&](double *dst, const std::vector<double> &src) {
    if (!dst) return;
    PBMP_HIP(hipMemcpyAsync(dst, src.data(), sizeof(double) * src.size(),
                            where == PBMP_DEVICE ? hipMemcpyHostToDevice
                                                 : hipMemcpyHostToHost, s_));
  };
  put(g_xyz, oxyz);
  put(g_q, oq);
  put(g_d, od);
  put(g_Q, oQ);
  put(g_verts, overts);
  sync();
  adj_ok_ = true;
  adj_bar_ = dGbar;
  adj_M_ = M;
  return warn;
}

}  // namespace pbmp
