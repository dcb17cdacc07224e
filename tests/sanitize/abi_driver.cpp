// Driver of the C-ABI for a build of the library whose host code carries
// AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers_cpu.py
// builds it host-only, without kernels, and runs the paths that need no GPU:
// option validation, null contexts, the quadrature set-up of pbmp_create up
// to its first HIP call).  With a GPU and a full build it also runs a small
// solve and its backward.  Exit status 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/pbmp.h"

namespace {

int failures = 0;

void check(bool ok, const char *what) {
  if (!ok) {
    std::printf("FAIL %s\n", what);
    std::fflush(stdout);
    ++failures;
  }
}

// octahedron refined twice and projected to radius r: 128 panels,
// counter-clockwise seen from outside
void sphere(double r, std::vector<double> &v, std::vector<int32_t> &t) {
  v = {1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1};
  t = {0, 2, 4, 2, 1, 4, 1, 3, 4, 3, 0, 4, 2, 0, 5, 1, 2, 5, 3, 1, 5, 0, 3, 5};
  for (int level = 0; level < 2; ++level) {
    std::vector<int32_t> nt;
    auto mid = [&](int a, int b) {
      double p[3];
      for (int d = 0; d < 3; ++d) p[d] = 0.5 * (v[3 * a + d] + v[3 * b + d]);
      const double n = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
      for (int d = 0; d < 3; ++d) p[d] /= n;
      for (size_t k = 0; k < v.size() / 3; ++k)
        if (std::fabs(v[3 * k] - p[0]) + std::fabs(v[3 * k + 1] - p[1]) +
                std::fabs(v[3 * k + 2] - p[2]) < 1e-12)
          return (int)k;
      v.insert(v.end(), p, p + 3);
      return (int)(v.size() / 3 - 1);
    };
    for (size_t f = 0; f < t.size() / 3; ++f) {
      const int a = t[3 * f], b = t[3 * f + 1], c = t[3 * f + 2];
      const int ab = mid(a, b), bc = mid(b, c), ca = mid(c, a);
      const int q[12] = {a, ab, ca, ab, b, bc, ca, bc, c, ab, bc, ca};
      nt.insert(nt.end(), q, q + 12);
    }
    t.swap(nt);
  }
  for (double &x : v) x *= r;
}

}  // namespace

int main() {
  pbmp_options o;
  pbmp_default_options(&o);
  pbmp_ctx *c = nullptr;

  // option validation happens before any device call
  struct Bad {
    const char *name;
    void (*set)(pbmp_options &);
  } bad[] = {
      {"eps_in", [](pbmp_options &x) { x.eps_in = -1.0; }},
      {"kappa", [](pbmp_options &x) { x.kappa = -0.1; }},
      {"gauss_far", [](pbmp_options &x) { x.gauss_far = 2; }},
      {"theta", [](pbmp_options &x) { x.theta = 1.5; }},
      {"order_P", [](pbmp_options &x) { x.order_P = 9; }},
      {"leaf_panels", [](pbmp_options &x) { x.leaf_panels = 2; }},
      {"gmres_restart", [](pbmp_options &x) { x.gmres_restart = 0; }},
      {"scf_omega", [](pbmp_options &x) { x.scf_omega = 2.5; }},
      {"precision", [](pbmp_options &x) { x.precision = 7; }},
  };
  for (const Bad &b : bad) {
    pbmp_options x = o;
    b.set(x);
    const int rc = pbmp_create(&x, &c);
    check(rc == PBMP_EARG && c == nullptr, b.name);
    check(std::strlen(pbmp_last_error(nullptr)) > 0, "create error message");
  }
  check(pbmp_create(nullptr, &c) == PBMP_EARG, "null options");
  check(pbmp_solve(nullptr, nullptr) == PBMP_EARG, "null context solve");
  check(pbmp_set_mesh(nullptr, 0, nullptr, 0, nullptr, PBMP_HOST) == PBMP_EARG,
        "null context set_mesh");
  check(pbmp_site_fields(nullptr, nullptr, nullptr, PBMP_HOST) == PBMP_EARG,
        "null context site_fields");
  check(pbmp_site_fields_noalloc(nullptr, nullptr, nullptr) == PBMP_EARG,
        "null context site_fields_noalloc");
  check(pbmp_set_options(nullptr, &o) == PBMP_EARG, "null context set_options");
  check(pbmp_matvec(nullptr, nullptr, nullptr, 0, PBMP_HOST) == PBMP_EARG,
        "null context matvec");
  check(pbmp_rhs(nullptr, nullptr, nullptr, PBMP_HOST) == PBMP_EARG, "null context rhs");
  check(pbmp_backward(nullptr, 1.0, nullptr, nullptr, nullptr, nullptr, nullptr, PBMP_HOST) ==
            PBMP_EARG,
        "null context backward");
  check(pbmp_kernel_stats(nullptr, 0, nullptr) == PBMP_EARG, "null context kernel_stats");
  {
    double out3[3];
    check(pbmp_binding_energies(nullptr, nullptr, nullptr, out3) == PBMP_EARG,
          "null contexts binding_energies");
    int64_t nlv = 0;
    check(pbmp_ligand_translation_gradient(nullptr, 0, nullptr, out3, &nlv, PBMP_HOST) ==
              PBMP_EARG,
          "null context ligand_translation_gradient");
  }
  check(std::strlen(pbmp_last_error(nullptr)) > 0, "last_error without a context");
  pbmp_destroy(nullptr);

  // valid options: the quadrature rules are set up, then the first HIP call
  // either succeeds (a GPU) or fails with PBMP_EHIP
  o.mode = PBMP_MODE_DIRECT;
  o.precision = PBMP_FP64;
  const int rc = pbmp_create(&o, &c);
  if (rc == PBMP_EHIP) {
    std::printf("no GPU: create stopped at its first HIP call (%s)\n",
                pbmp_last_error(nullptr));
    std::printf("%s\n", failures ? "FAILED" : "OK");
    std::fflush(stdout);
    return failures ? 1 : 0;
  }
  check(rc == PBMP_OK && c != nullptr, "create");
  if (rc == PBMP_OK) {
    std::vector<double> v;
    std::vector<int32_t> t;
    sphere(4.0, v, t);
    check(pbmp_set_mesh(c, (int64_t)v.size() / 3, v.data(), (int64_t)t.size() / 3, t.data(),
                        PBMP_HOST) == PBMP_OK,
          "set_mesh");
    const double xyz[12] = {0.5, 0.1, 0.0, -0.6, 0.3, 0.2, 0.0, -0.8, 0.4, 0.2, 0.4, -0.9};
    const double q[4] = {0.4, -0.3, 0.2, -0.1};
    const double d[12] = {0.1, 0.0, 0.05, 0.0, -0.1, 0.0, 0.02, 0.03, -0.01, 0.0, 0.0, 0.1};
    double Q9[36] = {0};
    Q9[0] = 0.1, Q9[4] = -0.05, Q9[8] = -0.05;
    const double alpha[4] = {1.0, 0.8, 1.2, 0.5};
    check(pbmp_set_sites(c, 4, xyz, q, d, Q9, alpha, nullptr, PBMP_HOST) == PBMP_OK,
          "set_sites");
    std::vector<double> phi(t.size() / 3), dphi(t.size() / 3), mud(12), muv(12);
    pbmp_result r;
    std::memset(&r, 0, sizeof(r));
    r.where = PBMP_HOST;
    r.phi = phi.data();
    r.dphidn = dphi.data();
    r.mu_diss = mud.data();
    r.mu_vac = muv.data();
    check(pbmp_solve(c, &r) == PBMP_OK, "solve");
    check(std::isfinite(r.dG_kcal) && r.dG_kcal < 0.0, "solvation energy finite and negative");
    std::vector<double> gx(12), gq(4), gd(12), gQ(36), gv(v.size());
    check(pbmp_backward(c, 1.0, gx.data(), gq.data(), gd.data(), gQ.data(), gv.data(),
                        PBMP_HOST) == PBMP_OK,
          "backward");
    double s = 0.0;
    for (double g : gx) s += g * g;
    check(std::isfinite(s), "gradients finite");
    std::printf("GPU: dG %.6f kcal/mol, %d SCF iterations\n", r.dG_kcal, r.scf_iters);
    pbmp_destroy(c);
  }
  std::printf("%s\n", failures ? "FAILED" : "OK");
  std::fflush(stdout);
  return failures ? 1 : 0;
}
