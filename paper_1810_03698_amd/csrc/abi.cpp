// C-ABI entry points (include/pbmp.h).  Every call converts library errors
// into status codes and a per-context message.
#include <cstring>
#include <memory>

#include "runtime.hpp"

using pbmp::Error;

namespace {

thread_local std::string g_create_error;

template <class F> int guarded(pbmp_ctx *c, F &&f) {
  if (!c) return PBMP_EARG;
  try {
    int rc = f();
    if (rc == 0) c->err.clear();
    return rc;
  } catch (const Error &e) {
    c->err = e.what();
    return e.code;
  } catch (const std::exception &e) {
    c->err = e.what();
    return PBMP_EHIP;
  }
}

}  // namespace

extern "C" {

void pbmp_default_options(pbmp_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->eps_in = 1.0;
  o->eps_out = 80.0;
  o->kappa = 0.125;
  o->gauss_far = 3;
  o->near_eta = 2.0;
  o->mode = PBMP_MODE_AUTO;
  o->theta = 0.5;
  o->order_P = 4;
  o->leaf_panels = 300;
  o->gmres_restart = 50;
  o->gmres_tol = 1e-6;
  o->gmres_maxit = 1000;
  o->scf_tol_debye = 1e-6;
  o->scf_omega = 0.7;
  o->scf_maxit = 200;
  o->thole_a = 0.39;
  o->precision = PBMP_MIXED;
  o->hip_stream = nullptr;
  o->warm_start = 0;
  o->verbose = 0;
}

int pbmp_create(const pbmp_options *o, pbmp_ctx **out) {
  if (!o || !out) return PBMP_EARG;
  *out = nullptr;
  try {
    // the context is released if the runtime's constructor throws
    std::unique_ptr<pbmp_ctx> c(new pbmp_ctx());
    c->rt.reset(new pbmp::Runtime(*o));
    *out = c.release();
    return PBMP_OK;
  } catch (const Error &e) {
    g_create_error = e.what();
    return e.code;
  } catch (const std::exception &e) {
    g_create_error = e.what();
    return PBMP_EHIP;
  }
}

int pbmp_set_mesh(pbmp_ctx *c, int64_t nv, const double *verts, int64_t nt,
                  const int32_t *tris, int where) {
  return guarded(c, [&] {
    c->rt->set_mesh(nv, verts, nt, tris, where);
    return 0;
  });
}

int pbmp_set_sites(pbmp_ctx *c, int64_t m, const double *xyz, const double *q,
                   const double *d, const double *Q9, const double *alpha,
                   const int32_t *group, int where) {
  return guarded(c, [&] {
    c->rt->set_sites(m, xyz, q, d, Q9, alpha, group, where);
    return 0;
  });
}

int pbmp_solve(pbmp_ctx *c, pbmp_result *r) {
  return guarded(c, [&] { return c->rt->solve(r); });
}

int pbmp_matvec(pbmp_ctx *c, const double *x, double *y, int transpose, int where) {
  return guarded(c, [&] {
    c->rt->matvec_user(x, y, transpose, where);
    return 0;
  });
}

int pbmp_rhs(pbmp_ctx *c, const double *p_total, double *f, int where) {
  return guarded(c, [&] {
    c->rt->rhs_user(p_total, f, where);
    return 0;
  });
}

int pbmp_site_fields(pbmp_ctx *c, const double *x, double *out, int where) {
  return guarded(c, [&] {
    c->rt->site_fields_user(x, out, where);
    return 0;
  });
}

int pbmp_site_fields_noalloc(pbmp_ctx *c, const double *x, double *out) {
  return guarded(c, [&] {
    c->rt->site_fields_noalloc(x, out);
    return 0;
  });
}

int pbmp_backward(pbmp_ctx *c, double dG_bar, double *g_xyz, double *g_q,
                  double *g_d, double *g_Q9, double *g_verts, int where) {
  return guarded(c, [&] {
    return c->rt->backward(dG_bar, g_xyz, g_q, g_d, g_Q9, g_verts, where);
  });
}

int pbmp_kernel_stats(pbmp_ctx *c, int mode, pbmp_kstats *out) {
  return guarded(c, [&] {
    auto &k = c->rt->clock;
    if (mode == 1) {
      k.reset();
      k.on = true;
    } else if (mode == 0) {
      k.on = false;
    }
    k.resolve();
    if (out) {
      out->p2p_ms = k.p2p_ms;
      out->m2p_ms = k.m2p_ms;
      out->p2m_ms = k.p2m_ms;
      out->matvec_ms = k.matvec_ms;
      out->p2p_launches = k.p2p_launches;
      out->m2p_launches = k.m2p_launches;
      out->matvec_calls = k.matvec_calls;
      out->p2p_pairs = k.p2p_pairs;
      out->m2p_pairs = k.m2p_pairs;
    }
    return 0;
  });
}

int pbmp_set_options(pbmp_ctx *c, const pbmp_options *o) {
  return guarded(c, [&] {
    PBMP_REQUIRE(o != nullptr, PBMP_EARG, "null options");
    c->rt->set_options(*o);
    return 0;
  });
}

int pbmp_set_stern(pbmp_ctx *c, int64_t nv, const double *verts, int64_t nt,
                   const int32_t *tris, double eps_stern, int where) {
  return guarded(c, [&] {
    c->rt->set_stern(nv, verts, nt, tris, eps_stern, where);
    return 0;
  });
}

int pbmp_tree_export(pbmp_ctx *c, int64_t counts[4], int32_t *perm, int32_t *box_range,
                     int32_t *box_level, double *box_centre, double *box_radius,
                     int32_t *leaf_box, int32_t *m2p_ptr, int32_t *m2p_box,
                     int32_t *p2p_ptr, int32_t *p2p_box) {
  return guarded(c, [&] {
    c->rt->tree_export(counts, perm, box_range, box_level, box_centre, box_radius, leaf_box,
                       m2p_ptr, m2p_box, p2p_ptr, p2p_box);
    return 0;
  });
}

int pbmp_binding_energies(pbmp_ctx *complex, pbmp_ctx *receptor, pbmp_ctx *ligand,
                          double out[3]) {
  if (!receptor || !ligand) return PBMP_EARG;
  return guarded(complex, [&] {
    PBMP_REQUIRE(out != nullptr, PBMP_EARG, "null output");
    double ab, gab, a, ga, b, gb;
    complex->rt->binding_terms(&ab, &gab);
    receptor->rt->binding_terms(&a, &ga);
    ligand->rt->binding_terms(&b, &gb);
    out[0] = ab - a - b;
    out[1] = gab - ga - gb;
    out[2] = out[0] + out[1];
    return 0;
  });
}

int pbmp_ligand_translation_gradient(pbmp_ctx *complex, int64_t first_ligand_site,
                                     const double *radii, double g_t[3],
                                     int64_t *n_ligand_vertices, int where) {
  return guarded(complex, [&] {
    return complex->rt->ligand_translation_gradient(first_ligand_site, radii, where, g_t,
                                                    n_ligand_vertices);
  });
}

const char *pbmp_last_error(const pbmp_ctx *c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

void pbmp_destroy(pbmp_ctx *c) { delete c; }

}  // extern "C"
